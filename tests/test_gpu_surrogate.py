"""GPU checks of the surrogate kernels against the FP64 reference (oracle.conv).

Inputs are rounded to BF16 on the host first, so both sides see the same
operands; the GPU accumulates in FP32 and rounds its output to BF16, which
bounds the difference by ~2^-8 of the output scale (forward, input gradient)
and by FP32 summation error (weight gradient)."""
import numpy as np
import pytest

from oracle import conv

pytestmark = pytest.mark.gpu


def _sur():
    from paper_1007_1388_amd import surrogate
    return surrogate


def bf(a):
    return conv.bf16_round(a)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


CASES = [
    dict(n=2, d=6, h=8, w=10, ci=16, co=24, k=3, s=1),
    dict(n=1, d=8, h=6, w=4, ci=8, co=32, k=3, s=2),
    dict(n=1, d=5, h=7, w=9, ci=64, co=80, k=3, s=1),
    dict(n=2, d=4, h=4, w=6, ci=32, co=8, k=1, s=1),
    dict(n=1, d=9, h=3, w=5, ci=24, co=16, k=3, s=2),
    # gathered channels a multiple of 32: the tap-major kernels, every tile
    # shape (32, 64, 128 columns and a partial second column tile), the
    # stride-2 input gradient by parity classes on odd and even extents
    dict(n=2, d=7, h=6, w=9, ci=32, co=64, k=3, s=2),
    dict(n=1, d=6, h=5, w=11, ci=64, co=32, k=3, s=1),
    dict(n=1, d=4, h=6, w=8, ci=128, co=160, k=3, s=1),
    dict(n=1, d=5, h=3, w=7, ci=32, co=32, k=1, s=1),
    dict(n=1, d=9, h=4, w=5, ci=96, co=128, k=3, s=2),
    # weight gradient by halos (3x3x3, Cin a multiple of 32, dy width a
    # divisor of 32 or at least 32): rows of 16, 8 and 2 voxels per step,
    # partial row blocks, a partial second 32-voxel block, both strides, a
    # partial output-channel tile
    dict(n=1, d=5, h=6, w=16, ci=32, co=32, k=3, s=1),
    dict(n=2, d=3, h=5, w=40, ci=32, co=64, k=3, s=1),
    dict(n=1, d=6, h=7, w=16, ci=64, co=48, k=3, s=2),
    dict(n=1, d=4, h=5, w=2, ci=32, co=32, k=3, s=1),
    dict(n=1, d=3, h=3, w=70, ci=32, co=32, k=3, s=2),
    # stride-1 3x3x3 onto rows of whole 32-voxel pieces with at most 64
    # output columns: the halo-staged forward and input gradient, 32 and 64
    # columns (a partial one of 48), one to three 32-channel chunks, a
    # partial 8-row block, two pieces per row
    dict(n=2, d=5, h=11, w=32, ci=32, co=32, k=3, s=1),
    dict(n=1, d=3, h=8, w=64, ci=64, co=32, k=3, s=1),
    dict(n=1, d=4, h=7, w=32, ci=64, co=64, k=3, s=1),
    dict(n=1, d=4, h=5, w=32, ci=96, co=48, k=3, s=1),
    # weight gradient of the 8-channel input layer (all 27 taps per
    # workgroup): rows of 16, 32 + a partial 8 and 2 voxels per step, one to
    # two output-channel tiles (partial ones included)
    dict(n=2, d=5, h=6, w=16, ci=8, co=32, k=3, s=1),
    dict(n=1, d=4, h=5, w=40, ci=8, co=48, k=3, s=1),
    dict(n=1, d=3, h=7, w=2, ci=8, co=16, k=3, s=1),
    # pointwise products: 16 to 64 input channels, partial output-channel
    # tiles
    dict(n=1, d=3, h=5, w=9, ci=64, co=8, k=1, s=1),
    dict(n=1, d=2, h=7, w=13, ci=16, co=24, k=1, s=1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("relu", [False, True])
def test_conv_forward(case, relu):
    S = _sur()
    c = CASES[case]
    rng = np.random.default_rng(case)
    x = bf(rng.standard_normal((c["n"], c["d"], c["h"], c["w"], c["ci"])))
    w = bf(rng.standard_normal((c["co"], c["k"] ** 3, c["ci"])) * 0.1)
    b = rng.standard_normal(c["co"]).astype(np.float32) * 0.1
    layer = S.Conv(c["ci"], c["co"], k=c["k"], stride=c["s"], relu=relu)
    layer.set_weights(w, b)
    X = S.from_numpy(x)
    ref = conv.conv3d(x, w, b.astype(np.float64), c["k"], c["s"], relu)
    Y = S.Act(c["n"], *ref.shape[1:4], c["co"])
    layer.forward(X, Y)
    got = Y.to_numpy()
    assert rel(got, ref) < 8e-3, rel(got, ref)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_conv_input_gradient_with_relu_mask(case):
    S = _sur()
    c = CASES[case]
    rng = np.random.default_rng(10 + case)
    xs = (c["n"], c["d"], c["h"], c["w"], c["ci"])
    w = bf(rng.standard_normal((c["co"], c["k"] ** 3, c["ci"])) * 0.1)
    layer = S.Conv(c["ci"], c["co"], k=c["k"], stride=c["s"], relu=False)
    layer.set_weights(w, np.zeros(c["co"]))
    ys = conv.conv3d(np.zeros(xs), w, None, c["k"], c["s"]).shape
    dy = bf(rng.standard_normal(ys))
    act = bf(rng.standard_normal(xs))       # ReLU'(act) masks the result
    ref = conv.conv3d_bwd_data(dy, w, xs, c["k"], c["s"]) * (act > 0)
    DX = S.Act(*xs)
    from paper_1007_1388_amd.surrogate import lib
    L = lib()
    DY, ACT = S.from_numpy(dy), S.from_numpy(act)   # keep the buffers alive during the calls
    st = L.lbm_conv3d_bwd_data(DY.ref, layer.wt.data_ptr(), DX.ref, ACT.ref, c["k"], c["s"], 0, None)
    assert st == 0
    got = DX.to_numpy()
    assert rel(got, ref) < 8e-3, rel(got, ref)
    # accumulate mode adds a second copy
    prev = bf(rng.standard_normal(xs))
    DX2 = S.from_numpy(prev)
    st = L.lbm_conv3d_bwd_data(DY.ref, layer.wt.data_ptr(), DX2.ref, None, c["k"], c["s"], 1, None)
    assert st == 0
    ref2 = prev + conv.conv3d_bwd_data(dy, w, xs, c["k"], c["s"])
    assert rel(DX2.to_numpy(), ref2) < 8e-3


@pytest.mark.parametrize("case", range(len(CASES)))
def test_conv_weight_gradient(case):
    S = _sur()
    c = CASES[case]
    rng = np.random.default_rng(20 + case)
    xs = (c["n"], c["d"], c["h"], c["w"], c["ci"])
    x = bf(rng.standard_normal(xs))
    layer = S.Conv(c["ci"], c["co"], k=c["k"], stride=c["s"], relu=False)
    ys = conv.conv3d(x, np.zeros((c["co"], c["k"] ** 3, c["ci"])), None, c["k"], c["s"]).shape
    dy = bf(rng.standard_normal(ys))
    layer.zero_grad()
    layer.backward(S.from_numpy(x), S.from_numpy(dy), None)
    dw_ref, db_ref = conv.conv3d_bwd_weight(x, dy, c["k"], c["s"])
    gw = layer.gw.cpu().numpy()[:, :c["k"] ** 3 * c["ci"]].reshape(dw_ref.shape)
    assert rel(gw, dw_ref) < 1e-5, rel(gw, dw_ref)
    assert rel(layer.gb.cpu().numpy(), db_ref) < 1e-5
    assert np.all(layer.gw.cpu().numpy()[:, c["k"] ** 3 * c["ci"]:] == 0)


def test_upsample_pair():
    S = _sur()
    from paper_1007_1388_amd.surrogate import lib
    rng = np.random.default_rng(3)
    x = bf(rng.standard_normal((2, 3, 2, 4, 16)))
    X = S.from_numpy(x)
    Y = S.Act(2, 6, 4, 8, 16)
    assert lib().lbm_upsample2(X.ref, Y.ref, None) == 0
    assert np.array_equal(Y.to_numpy(), conv.upsample2(x))
    dy = bf(rng.standard_normal((2, 6, 4, 8, 16)))
    DX = S.Act(2, 3, 2, 4, 16)
    DY = S.from_numpy(dy)
    assert lib().lbm_upsample2_bwd(DY.ref, DX.ref, 0, None) == 0
    assert rel(DX.to_numpy(), conv.upsample2_bwd(dy)) < 8e-3


def test_mse_and_adam():
    import torch
    S = _sur()
    from paper_1007_1388_amd.surrogate import lib
    rng = np.random.default_rng(4)
    pred = bf(rng.standard_normal((1, 4, 4, 4, 8)))
    tgt = rng.standard_normal((64, 4)).astype(np.float32)
    wgt = (rng.random(64) > 0.3).astype(np.uint8)
    P = S.from_numpy(pred)
    D = S.Act(1, 4, 4, 4, 8)
    t = torch.from_numpy(tgt).cuda()
    wt = torch.from_numpy(wgt).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    inv = 1.0 / (4 * wgt.sum())
    assert lib().lbm_mse_loss(P.ref, t.data_ptr(), wt.data_ptr(), 4, inv, D.ref, loss.data_ptr(), None) == 0
    p = pred.reshape(64, 8)[:, :4]
    ref_loss = (((p - tgt) ** 2).sum(1) * wgt).sum() * inv
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)
    g = D.to_numpy().reshape(64, 8)
    ref_g = 2 * (p - tgt) * inv * wgt[:, None]
    assert np.abs(g[:, :4] - ref_g).max() <= 8e-3 * np.abs(ref_g).max() and np.all(g[:, 4:] == 0)
    # one Adam step from zero moments moves each weight by lr * sign(grad)
    w = torch.zeros(100, device="cuda")
    gr = torch.from_numpy(rng.standard_normal(100).astype(np.float32)).cuda()
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    assert lib().lbm_adam_step(w.data_ptr(), gr.data_ptr(), m.data_ptr(), v.data_ptr(), 100, 1e-2, 0.9, 0.999,
                               1e-12, 1, None) == 0
    assert np.allclose(w.cpu().numpy(), -1e-2 * np.sign(gr.cpu().numpy()), rtol=1e-5, atol=1e-7)


def _layer_graph(net):
    """The U-Net's graph, layer by layer in forward order: (name, layer, input
    Act, gradient Act of the input or None, the gradient Act of the layer's
    pre-activation output, the layer whose data gradient adds to the same
    input gradient first or None).  Inputs and outputs are the forward's own
    buffers (net.io()); a tensor's gradient lives in net.g under the tensor's
    name, channel slices of a concatenation in slices of its gradient."""
    c0, c1, c2, _ = net.CH
    g = net._gs
    grad_of = {"a0": g("a0"), "skip0": g("cat0", c0, c0), "l1in": g("l1in"), "a1": g("a1"),
               "skip1": g("cat1", c1, c1), "l2in": g("l2in"), "a2": g("a2"), "skip2": g("cat2", c2, c2),
               "l3in": g("l3in"), "a3": g("a3"), "b3": g("b3"), "u2": g("u2"), "upc2": g("cat2", 0, c2),
               "cat2": g("cat2"), "d2": g("d2"), "d2o": g("d2o"), "u1": g("u1"), "upc1": g("cat1", 0, c1),
               "cat1": g("cat1"), "d1": g("d1"), "d1o": g("d1o"), "u0": g("u0"), "upc0": g("cat0", 0, c0),
               "cat0": g("cat0"), "d0": g("d0"), "d0o": g("d0o")}
    name_of = {id(v): k for k, v in vars(net).items() if k in grad_of}
    # a skip tensor feeds the decoder's concatenation (whose layer writes the
    # whole gradient of the concatenation) and the next stride-2 layer (which
    # adds its data gradient to the skip part)
    first = {"dn0": "d0a", "dn1": "d1a", "dn2": "d2a"}
    out = []
    for name, l, x, y in net.io():
        xin = name_of.get(id(x))
        yname = name_of.get(id(y))
        out.append((name, l, x, None if xin is None else grad_of[xin], None if yname is None else grad_of[yname],
                    first.get(name)))
    return out


def test_network_layers_forward_and_gradients_match_fp64_reference_layer_by_layer():
    # Each layer is checked on its own, on the operands the GPU itself stored:
    # its BF16 input activation and the BF16 gradient of its pre-activation
    # output as the backward pass left them.  Per layer: output (forward with
    # bias and ReLU), weight and bias gradients, and the data gradient masked
    # by ReLU'(input) (added onto the decoder layer's gradient of a skip
    # tensor), each against oracle.conv in FP64 at 1e-2 relative (infinity
    # norm over the largest reference value).  The three upsampling adjoints
    # are checked the same way.
    S = _sur()
    rng = np.random.default_rng(7)
    net = S.UNet(1, 16, 8, 8, seed=3)
    x = np.zeros((1, 16, 8, 8, 8))
    x[..., :3] = rng.standard_normal((1, 16, 8, 8, 3))
    X = S.from_numpy(bf(x))
    net.x.buf.copy_(X.buf)
    pred = net.forward()
    dpred = np.zeros(pred.to_numpy().shape)
    dpred[..., :4] = bf(rng.standard_normal(dpred[..., :4].shape))
    D = S.from_numpy(dpred)
    net.zero_grad()
    net.backward(D)
    c0, c1, c2, _ = net.CH
    # the GPU's stored BF16 weights of every layer
    W = {}
    for name, l, _, _ in net.io():
        w = l.w.cpu().numpy()[:, :l.taps * l.cin].reshape(l.cout, l.taps, l.cin).astype(np.float64)
        W[name] = bf(w)
    graph = _layer_graph(net)
    tol = 1e-2
    dx_part = {}
    for name, l, xa, gx, gy, first in graph:
        xin = xa.to_numpy()
        # forward: the layer's stored output from its stored input
        _, _, _, y = next(t for t in net.io() if t[0] == name)
        yref = conv.conv3d(xin, W[name], l.b.cpu().numpy().astype(np.float64), l.k, l.stride, l.relu)
        assert rel(y.to_numpy(), yref) < tol, (name, "forward", rel(y.to_numpy(), yref))
        dy = dpred if name == "head" else gy.to_numpy()
        dw, db = conv.conv3d_bwd_weight(xin, dy, l.k, l.stride)
        gw = l.gw.cpu().numpy()[:, :l.taps * l.cin].reshape(dw.shape)
        assert rel(gw, dw) < tol, (name, "weight gradient", rel(gw, dw))
        # bias gradient: the sum of dy over voxels, against the scale of the
        # summands where cancellation makes the sum itself small
        gb = l.gb.cpu().numpy()
        scale = max(np.abs(db).max(), 1e-3 * np.abs(dy).sum(axis=(0, 1, 2, 3)).max())
        assert np.abs(gb - db).max() < tol * scale, (name, "bias gradient")
        if gx is not None:
            dx_part[name] = conv.conv3d_bwd_data(dy, W[name], xin.shape, l.k, l.stride) * (xin > 0)
    skips = {"dn0": slice(c0, 2 * c0), "dn1": slice(c1, 2 * c1), "dn2": slice(c2, 2 * c2)}
    for name, l, xa, gx, gy, first in graph:
        if gx is None or name in ("d0a", "d1a", "d2a"):
            continue  # a decoder layer's skip part is checked with the stride-2 layer that adds to it
        dx = dx_part[name]
        if first is not None:
            # the decoder layer wrote its (rounded) gradient of the skip part first
            dx = bf(dx_part[first][..., skips[name]]) + dx
        got = gx.to_numpy()
        assert rel(got, dx) < tol, (name, "data gradient", rel(got, dx))
    # the up-path part of the decoder concatenations' gradients
    for name, cs in (("d0a", c0), ("d1a", c1), ("d2a", c2)):
        gcat = net.g["cat" + name[1]].to_numpy()[..., :cs]
        assert rel(gcat, dx_part[name][..., :cs]) < tol, (name, "data gradient (up part)")
    # upsampling adjoints: the gradient of each decoder level's output
    for src, dst in (("u0", "d1o"), ("u1", "d2o"), ("u2", "b3")):
        ref = conv.upsample2_bwd(net.g[src].to_numpy())
        assert rel(net.g[dst].to_numpy(), ref) < tol, (src, "upsample adjoint")
