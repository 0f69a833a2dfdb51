"""Learned warm start: a 3-D convolutional encoder-decoder on the GPU.

The network maps (obstacle mask, body force) of a porous channel to its
steady (rho, u) field, normalised by the force (Stokes-like linearity); the
prediction initialises the lattice Boltzmann solver through
lbm_set_equilibrium, and the solver then runs to its own steady state, so the
plain method both falls back for and judges the network.

All arithmetic runs in the HIP kernels of include/lbm_surrogate.h (BF16 MFMA
convolutions with FP32 accumulation, loss, Adam, input/target conversion);
this module only allocates torch buffers, wires the layers and marshals
pointers.  Architecture: 4 levels with 32/64/128/256 channels, two 3x3x3
convolutions per level and side, stride-2 convolutions down, nearest-neighbour
upsampling followed by a 3x3x3 convolution up, skip connections by channel
concatenation, ReLU, and a 1x1x1 head.
"""
import ctypes
import math

import numpy as np

from paper_1007_1388_amd import lbm

_sig_done = False


class lbm_tensor5(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("n", ctypes.c_int32), ("d", ctypes.c_int32),
                ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("c", ctypes.c_int32),
                ("ldc", ctypes.c_int32)]


SYMBOLS = ["lbm_conv_kpad", "lbm_conv3d_fwd", "lbm_conv3d_bwd_data", "lbm_conv3d_bwd_weight",
           "lbm_conv3d_weight_t", "lbm_upsample2", "lbm_upsample2_bwd", "lbm_mse_loss", "lbm_adam_step",
           "lbm_surrogate_input", "lbm_surrogate_target", "lbm_surrogate_fields"]


def lib():
    global _sig_done
    L = lbm.load()
    if not _sig_done:
        T = ctypes.POINTER(lbm_tensor5)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        d = ctypes.c_double
        f = ctypes.c_float
        sig = {
            "lbm_conv3d_fwd": [T, P, P, T, i32, i32, i32, P],
            "lbm_conv3d_bwd_data": [T, P, T, T, i32, i32, i32, P],
            "lbm_conv3d_bwd_weight": [T, T, P, P, i32, i32, P],
            "lbm_conv3d_weight_t": [P, i32, i32, i32, P, P, P],
            "lbm_upsample2": [T, T, P],
            "lbm_upsample2_bwd": [T, T, i32, P],
            "lbm_mse_loss": [T, P, P, i32, f, T, P, P],
            "lbm_adam_step": [P, P, P, P, ctypes.c_int64, f, f, f, f, i32, P],
            "lbm_surrogate_input": [P, d, T, P],
            "lbm_surrogate_target": [P, P, P, d, d, d, ctypes.c_int64, P, P, P],
            "lbm_surrogate_fields": [T, P, d, d, d, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lbm_conv_kpad.argtypes = [i32, i32]
        L.lbm_conv_kpad.restype = i32
        _sig_done = True
    return L


def _ck(status, where):
    if status != 0:
        raise lbm.LBMError(status, where)


class Act:
    """A channels-last BF16 activation buffer [n, d, h, w, ldc] (torch int16
    storage) and channel slices of it."""

    def __init__(self, n, d, h, w, c, buf=None, off=0, ldc=None):
        import torch
        self.n, self.d, self.h, self.w, self.c = n, d, h, w, c
        if buf is None:
            self.buf = torch.zeros((n, d, h, w, c), dtype=torch.int16, device="cuda")
            self.ldc = c
            self.off = 0
        else:
            self.buf, self.off, self.ldc = buf, off, ldc
        self.t5 = lbm_tensor5(self.buf.data_ptr() + 2 * self.off, n, d, h, w, c, self.ldc)
        self.t5._owner = self   # a byref of t5 keeps the buffer alive

    def slice(self, off, c):
        return Act(self.n, self.d, self.h, self.w, c, buf=self.buf, off=self.off + off, ldc=self.ldc)

    @property
    def ref(self):
        return ctypes.byref(self.t5)

    def to_numpy(self):
        """FP64 copy of the used channels (for tests)."""
        import torch
        v = self.buf.view(torch.int16)[..., self.off:self.off + self.c].contiguous()
        u = v.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return u.view(np.float32).astype(np.float64)

    def zero_(self):
        self.buf.zero_()


def from_numpy(a):
    """BF16 (round to nearest even, done on the host) Act from [n,d,h,w,c] FP32/64."""
    import torch
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    n, d, h, w, c = a.shape
    t = Act(n, d, h, w, c)
    t.buf.copy_(torch.from_numpy(u.view(np.int16)))
    return t


class Conv:
    """One convolution layer: FP32 master weights w[co][kpad] (K-major,
    k = tap*cin + ci), FP32 bias, BF16 forward and transposed copies, grads and
    Adam moments."""

    def __init__(self, cin, cout, k=3, stride=1, relu=True, seed=0):
        import torch
        self.cin, self.cout, self.k, self.stride, self.relu = cin, cout, k, stride, relu
        self.taps = k ** 3
        L = lib()
        self.kpad = L.lbm_conv_kpad(self.taps, cin)
        self.kpad_t = L.lbm_conv_kpad(self.taps, cout)
        rng = np.random.default_rng(seed)
        std = math.sqrt(2.0 / (self.taps * cin)) if relu else math.sqrt(1.0 / (self.taps * cin))
        w = np.zeros((cout, self.kpad), np.float32)
        w[:, :self.taps * cin] = rng.standard_normal((cout, self.taps * cin)) * std
        dev = "cuda"
        self.w = torch.from_numpy(w).to(dev)
        self.b = torch.zeros(cout, dtype=torch.float32, device=dev)
        self.wb = torch.zeros((cout, self.kpad), dtype=torch.int16, device=dev)
        self.wt = torch.zeros((cin, self.kpad_t), dtype=torch.int16, device=dev)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.refresh()

    def set_weights(self, w_co_t_ci, b):
        """Load weights given as [cout, taps, cin] (FP32/64) and bias [cout]."""
        import torch
        w = np.zeros((self.cout, self.kpad), np.float32)
        w[:, :self.taps * self.cin] = np.asarray(w_co_t_ci, np.float32).reshape(self.cout, -1)
        self.w.copy_(torch.from_numpy(w))
        self.b.copy_(torch.from_numpy(np.asarray(b, np.float32)))
        self.refresh()

    def refresh(self, stream=None):
        _ck(lib().lbm_conv3d_weight_t(self.w.data_ptr(), self.taps, self.cin, self.cout, self.wb.data_ptr(),
                                      self.wt.data_ptr(), stream), "lbm_conv3d_weight_t")

    def forward(self, x, y, stream=None):
        _ck(lib().lbm_conv3d_fwd(x.ref, self.wb.data_ptr(), self.b.data_ptr(), y.ref, self.k, self.stride,
                                 1 if self.relu else 0, stream), "lbm_conv3d_fwd")

    def backward(self, x, dy, dx, x_act=True, accumulate=False, stream=None):
        """Accumulate weight grads; write (or add) dx masked by ReLU'(x) when x
        came out of a ReLU layer (x_act)."""
        L = lib()
        _ck(L.lbm_conv3d_bwd_weight(x.ref, dy.ref, self.gw.data_ptr(), self.gb.data_ptr(), self.k, self.stride,
                                    stream), "lbm_conv3d_bwd_weight")
        if dx is not None:
            _ck(L.lbm_conv3d_bwd_data(dy.ref, self.wt.data_ptr(), dx.ref, x.ref if x_act else None, self.k,
                                      self.stride, 1 if accumulate else 0, stream), "lbm_conv3d_bwd_data")

    def zero_grad(self):
        self.gw.zero_()
        self.gb.zero_()

    def adam(self, t, lr, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        L = lib()
        _ck(L.lbm_adam_step(self.w.data_ptr(), self.gw.data_ptr(), self.mw.data_ptr(), self.vw.data_ptr(),
                            self.w.numel(), lr, b1, b2, eps, t, stream), "lbm_adam_step")
        _ck(L.lbm_adam_step(self.b.data_ptr(), self.gb.data_ptr(), self.mb.data_ptr(), self.vb.data_ptr(),
                            self.b.numel(), lr, b1, b2, eps, t, stream), "lbm_adam_step")
        self.refresh(stream)

    def flops(self, out_voxels):
        return 2.0 * out_voxels * self.taps * self.cin * self.cout


class UNet:
    """Encoder-decoder for inputs [n, D, H, W, 8]; D, H, W divisible by 8."""

    CH = (32, 64, 128, 256)

    def __init__(self, n, D, H, W, seed=0):
        c0, c1, c2, c3 = self.CH
        self.n, self.D, self.H, self.W = n, D, H, W
        s = iter(range(seed * 100, seed * 100 + 100))
        C = lambda ci, co, **kw: Conv(ci, co, seed=next(s), **kw)
        self.e0a, self.e0b = C(8, c0), C(c0, c0)
        self.dn0 = C(c0, c1, stride=2)
        self.e1a, self.e1b = C(c1, c1), C(c1, c1)
        self.dn1 = C(c1, c2, stride=2)
        self.e2a, self.e2b = C(c2, c2), C(c2, c2)
        self.dn2 = C(c2, c3, stride=2)
        self.e3a, self.e3b = C(c3, c3), C(c3, c3)
        self.up2, self.d2a, self.d2b = C(c3, c2), C(2 * c2, c2), C(c2, c2)
        self.up1, self.d1a, self.d1b = C(c2, c1), C(2 * c1, c1), C(c1, c1)
        self.up0, self.d0a, self.d0b = C(c1, c0), C(2 * c0, c0), C(c0, c0)
        self.head = C(c0, 8, k=1, relu=False)
        self.layers = [self.e0a, self.e0b, self.dn0, self.e1a, self.e1b, self.dn1, self.e2a, self.e2b, self.dn2,
                       self.e3a, self.e3b, self.up2, self.d2a, self.d2b, self.up1, self.d1a, self.d1b, self.up0,
                       self.d0a, self.d0b, self.head]
        self._alloc()
        self.t = 0

    def _alloc(self):
        n, D, H, W = self.n, self.D, self.H, self.W
        c0, c1, c2, c3 = self.CH
        dims = [(D, H, W), (D // 2, H // 2, W // 2), (D // 4, H // 4, W // 4), (D // 8, H // 8, W // 8)]
        A = lambda lvl, c: Act(n, *dims[lvl], c)
        self.x = A(0, 8)
        self.a0 = A(0, c0)
        self.cat0 = A(0, 2 * c0)             # [up-path | skip]
        self.skip0 = self.cat0.slice(c0, c0)
        self.upc0 = self.cat0.slice(0, c0)
        self.a1, self.cat1 = A(1, c1), A(1, 2 * c1)
        self.skip1, self.upc1 = self.cat1.slice(c1, c1), self.cat1.slice(0, c1)
        self.a2, self.cat2 = A(2, c2), A(2, 2 * c2)
        self.skip2, self.upc2 = self.cat2.slice(c2, c2), self.cat2.slice(0, c2)
        self.l1in, self.l2in, self.l3in = A(1, c1), A(2, c2), A(3, c3)
        self.a3, self.b3 = A(3, c3), A(3, c3)
        self.u2 = A(2, c3)                   # upsampled b3
        self.d2 = A(2, c2)
        self.d2o = A(2, c2)
        self.u1 = A(1, c2)
        self.d1 = A(1, c1)
        self.d1o = A(1, c1)
        self.u0 = A(0, c1)
        self.d0 = A(0, c0)
        self.d0o = A(0, c0)
        self.pred = A(0, 8)
        # gradient buffers (same shapes)
        self.g = {k: Act(v.n, v.d, v.h, v.w, v.c) for k, v in list(vars(self).items())
                  if isinstance(v, Act) and v.off == 0 and v.c == v.buf.shape[-1] and k != "x"}

    def _gs(self, name, off=0, c=None):
        g = self.g[name]
        return g if (off == 0 and c is None) else g.slice(off, c)

    def forward(self, stream=None):
        L = lib()
        self.e0a.forward(self.x, self.a0, stream)
        self.e0b.forward(self.a0, self.skip0, stream)
        self.dn0.forward(self.skip0, self.l1in, stream)
        self.e1a.forward(self.l1in, self.a1, stream)
        self.e1b.forward(self.a1, self.skip1, stream)
        self.dn1.forward(self.skip1, self.l2in, stream)
        self.e2a.forward(self.l2in, self.a2, stream)
        self.e2b.forward(self.a2, self.skip2, stream)
        self.dn2.forward(self.skip2, self.l3in, stream)
        self.e3a.forward(self.l3in, self.a3, stream)
        self.e3b.forward(self.a3, self.b3, stream)
        _ck(L.lbm_upsample2(self.b3.ref, self.u2.ref, stream), "lbm_upsample2")
        self.up2.forward(self.u2, self.upc2, stream)
        self.d2a.forward(self.cat2, self.d2, stream)
        self.d2b.forward(self.d2, self.d2o, stream)
        _ck(L.lbm_upsample2(self.d2o.ref, self.u1.ref, stream), "lbm_upsample2")
        self.up1.forward(self.u1, self.upc1, stream)
        self.d1a.forward(self.cat1, self.d1, stream)
        self.d1b.forward(self.d1, self.d1o, stream)
        _ck(L.lbm_upsample2(self.d1o.ref, self.u0.ref, stream), "lbm_upsample2")
        self.up0.forward(self.u0, self.upc0, stream)
        self.d0a.forward(self.cat0, self.d0, stream)
        self.d0b.forward(self.d0, self.d0o, stream)
        self.head.forward(self.d0o, self.pred, stream)
        return self.pred

    def backward(self, dpred, stream=None):
        """dpred: gradient of the loss w.r.t. pred (Act); fills layer grads.

        Convention: the gradient handed to a layer's backward is already taken
        with respect to its pre-activation output; each data gradient is
        masked by ReLU'(input) of the layer that produced that input (an
        upsampled tensor is positive exactly where its parent is)."""
        L = lib()
        g = self._gs
        c0, c1, c2, _ = self.CH
        self.head.backward(self.d0o, dpred, g("d0o"), stream=stream)
        self.d0b.backward(self.d0, g("d0o"), g("d0"), stream=stream)
        self.d0a.backward(self.cat0, g("d0"), g("cat0"), stream=stream)
        self.up0.backward(self.u0, g("cat0", 0, c0), g("u0"), stream=stream)
        _ck(L.lbm_upsample2_bwd(g("u0").ref, g("d1o").ref, 0, stream), "lbm_upsample2_bwd")
        self.d1b.backward(self.d1, g("d1o"), g("d1"), stream=stream)
        self.d1a.backward(self.cat1, g("d1"), g("cat1"), stream=stream)
        self.up1.backward(self.u1, g("cat1", 0, c1), g("u1"), stream=stream)
        _ck(L.lbm_upsample2_bwd(g("u1").ref, g("d2o").ref, 0, stream), "lbm_upsample2_bwd")
        self.d2b.backward(self.d2, g("d2o"), g("d2"), stream=stream)
        self.d2a.backward(self.cat2, g("d2"), g("cat2"), stream=stream)
        self.up2.backward(self.u2, g("cat2", 0, c2), g("u2"), stream=stream)
        _ck(L.lbm_upsample2_bwd(g("u2").ref, g("b3").ref, 0, stream), "lbm_upsample2_bwd")
        self.e3b.backward(self.a3, g("b3"), g("a3"), stream=stream)
        self.e3a.backward(self.l3in, g("a3"), g("l3in"), stream=stream)
        # a skip tensor feeds the decoder (cat) and the next stride-2 conv
        self.dn2.backward(self.skip2, g("l3in"), g("cat2", c2, c2), accumulate=True, stream=stream)
        self.e2b.backward(self.a2, g("cat2", c2, c2), g("a2"), stream=stream)
        self.e2a.backward(self.l2in, g("a2"), g("l2in"), stream=stream)
        self.dn1.backward(self.skip1, g("l2in"), g("cat1", c1, c1), accumulate=True, stream=stream)
        self.e1b.backward(self.a1, g("cat1", c1, c1), g("a1"), stream=stream)
        self.e1a.backward(self.l1in, g("a1"), g("l1in"), stream=stream)
        self.dn0.backward(self.skip0, g("l1in"), g("cat0", c0, c0), accumulate=True, stream=stream)
        self.e0b.backward(self.a0, g("cat0", c0, c0), g("a0"), stream=stream)
        self.e0a.backward(self.x, g("a0"), None, stream=stream)

    def zero_grad(self):
        for l in self.layers:
            l.zero_grad()

    def adam(self, lr, stream=None):
        self.t += 1
        for l in self.layers:
            l.adam(self.t, lr, stream=stream)

    def io(self):
        """(name, layer, input, output) of every convolution, forward order."""
        return [("e0a", self.e0a, self.x, self.a0), ("e0b", self.e0b, self.a0, self.skip0),
                ("dn0", self.dn0, self.skip0, self.l1in), ("e1a", self.e1a, self.l1in, self.a1),
                ("e1b", self.e1b, self.a1, self.skip1), ("dn1", self.dn1, self.skip1, self.l2in),
                ("e2a", self.e2a, self.l2in, self.a2), ("e2b", self.e2b, self.a2, self.skip2),
                ("dn2", self.dn2, self.skip2, self.l3in), ("e3a", self.e3a, self.l3in, self.a3),
                ("e3b", self.e3b, self.a3, self.b3), ("up2", self.up2, self.u2, self.upc2),
                ("d2a", self.d2a, self.cat2, self.d2), ("d2b", self.d2b, self.d2, self.d2o),
                ("up1", self.up1, self.u1, self.upc1), ("d1a", self.d1a, self.cat1, self.d1),
                ("d1b", self.d1b, self.d1, self.d1o), ("up0", self.up0, self.u0, self.upc0),
                ("d0a", self.d0a, self.cat0, self.d0), ("d0b", self.d0b, self.d0, self.d0o),
                ("head", self.head, self.d0o, self.pred)]

    def flops_forward(self):
        n, D, H, W = self.n, self.D, self.H, self.W
        v = [n * D * H * W // (8 ** k) for k in range(4)]
        lv = {self.e0a: 0, self.e0b: 0, self.dn0: 1, self.e1a: 1, self.e1b: 1, self.dn1: 2, self.e2a: 2,
              self.e2b: 2, self.dn2: 3, self.e3a: 3, self.e3b: 3, self.up2: 2, self.d2a: 2, self.d2b: 2,
              self.up1: 1, self.d1a: 1, self.d1b: 1, self.up0: 0, self.d0a: 0, self.d0b: 0, self.head: 0}
        return sum(l.flops(v[lv[l]]) for l in self.layers)
