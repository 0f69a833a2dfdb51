"""Learned warm start of the porous-channel solver: data, training, prediction.

1. Data: porous channels (default 64 x 64 x 128: x, y periodic, walls in z),
   solid fraction uniform in [5 %, 20 %], sphere radii 3..8 (trapped cells
   and isolated pores filled, see inputs.fill_trapped_cells), g_x
   log-uniform in [5e-7, 5e-6], tau 0.7, each run from rest by the lattice
   Boltzmann solver until the residual ||u^n - u^(n-2)|| / (2 ||u^n||) drops
   below 1e-6.
2. Training: the U-Net of surrogate.py on (mask, g_x) -> (u, rho - rho0)/g_x,
   BF16 MFMA kernels, FP32 master weights, Adam, masked MSE on fluid cells.
3. Use: the prediction sets the initial state (an equilibrium of the
   predicted rho and u, stepped once and averaged with the next state, see
   `start_from`) and the same solver runs to the same residual criterion;
   `solve` times a run end to end, from rest or from the prediction
   (inference included).

The solver judges the network: a prediction only sets the initial state, and
both runs stop on the same residual criterion of the same solver.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1007_1388_amd import inputs, lbm  # noqa: E402

DIMS = (64, 64, 128)      # (nx, ny, nz)
TAU = 0.7
RHO0 = 1.0
TOL = 1e-6


def sample(seed, dims=DIMS):
    """Geometry and force of one sample (seeded)."""
    rng = np.random.default_rng(1_000_003 + seed)
    frac = float(rng.uniform(0.05, 0.20))
    gx = float(10 ** rng.uniform(np.log10(5e-7), np.log10(5e-6)))
    solid = inputs.porous_spheres(dims, target_fraction=frac, radius=(3, 8), seed=seed)
    # cells with undamped period-two momentum (and pockets) would keep the
    # step-to-step residual from ever reaching the tolerance
    solid = inputs.fill_trapped_cells(solid)
    return solid, gx, float(solid.mean())


def make_lattice(gx, solid, stream, precision="f32", dims=DIMS):
    lat = lbm.Lattice(dims, walls=(False, False, True), tau=TAU, rho0=RHO0, force=(gx, 0, 0),
                      precision=precision, stream=stream)
    lat.set_schedule(graph_steps=20)
    lat.set_geometry(solid)
    return lat


def run_to_steady(lats, check_every=100, max_steps=400_000, tol=TOL):
    """Step several lattices (each on its own stream) until each one's
    steady-state residual ||u^n - u^(n-2)|| / (2 ||u^n||) is below TOL;
    returns per-lattice (steps, seconds, residual).  The two-step difference
    per step is the rate of change with the period-two cycles of trapped
    bounce-back cells filtered out."""
    import torch
    n = len(lats)
    done = [None] * n
    t0 = [time.perf_counter()] * n
    steps = [0] * n
    while any(d is None for d in done):
        for k, lat in enumerate(lats):
            if done[k] is None:
                lat.step(check_every - 2)
                lat.residual_mark()
                lat.step(2)
                steps[k] += check_every
        for k, lat in enumerate(lats):
            if done[k] is None:
                r2, m = lat.residual_since_mark()
                r = r2 / m
                if r < tol or steps[k] >= max_steps or not math.isfinite(r):
                    done[k] = (steps[k], time.perf_counter() - t0[k], r)
    torch.cuda.synchronize()
    return done


def generate(seeds, concurrent=8, log=print, dims=DIMS):
    """Steady states for `seeds`; returns list of dicts with device tensors."""
    import torch
    from paper_1007_1388_amd import surrogate as S
    L = S.lib()
    out = []
    streams = [torch.cuda.Stream() for _ in range(concurrent)]
    for i0 in range(0, len(seeds), concurrent):
        chunk = seeds[i0:i0 + concurrent]
        geo = [sample(s, dims) for s in chunk]
        lats = [make_lattice(gx, solid, streams[k].cuda_stream, dims=dims) for k, (solid, gx, _) in enumerate(geo)]
        res = run_to_steady(lats)
        for k, lat in enumerate(lats):
            solid, gx, frac = geo[k]
            rho, u = lat.macroscopic_device()
            sol = torch.from_numpy(solid.reshape(-1)).cuda()
            out.append(dict(seed=chunk[k], gx=gx, frac=frac, solid=sol, rho=rho, u=u, steps=res[k][0],
                            secs=res[k][1], resid=res[k][2], fluid=int((solid == 0).sum())))
            lat.close()
        log("generated %d/%d (steps %s)" % (len(out), len(seeds), [r[0] for r in res]))
    return out


class Trainer:
    def __init__(self, batch=4, seed=0, scale=None, dims=DIMS):
        from paper_1007_1388_amd import surrogate as S
        self.S = S
        self.batch = batch
        self.dims = tuple(dims)
        nx, ny, nz = self.dims
        self.net = S.UNet(batch, nz, ny, nx, seed=seed)
        self.infer = None
        self.scale = scale
        self.V = nx * ny * nz

    def prepare(self, data):
        """Network inputs and normalised targets of every sample (kernels)."""
        import torch
        S = self.S
        L = S.lib()
        nx, ny, nz = self.dims
        if self.scale is None:
            # targets u / (g_x scale) of order one: scale by the largest |u|/g_x
            m = max(float(d["u"][0].abs().max().item()) / d["gx"] for d in data[:16])
            self.scale = m
        for d in data:
            x = S.Act(1, nz, ny, nx, 8)
            st = L.lbm_surrogate_input(d["solid"].data_ptr(), d["gx"], x.ref, None)
            assert st == 0
            t = torch.empty((self.V, 4), dtype=torch.float32, device="cuda")
            w = torch.empty(self.V, dtype=torch.uint8, device="cuda")
            st = L.lbm_surrogate_target(d["rho"].data_ptr(), d["u"].data_ptr(), d["solid"].data_ptr(), RHO0,
                                        d["gx"], self.scale, self.V, t.data_ptr(), w.data_ptr(), None)
            assert st == 0
            d["x"], d["t"], d["w"] = x, t, w
        torch.cuda.synchronize()

    def train(self, data, epochs=10, lr=1e-3, log=print):
        import torch
        S = self.S
        L = S.lib()
        net, B = self.net, self.batch
        nx, ny, nz = self.dims
        tb = torch.empty((B * self.V, 4), dtype=torch.float32, device="cuda")
        wb = torch.empty(B * self.V, dtype=torch.uint8, device="cuda")
        dpred = S.Act(B, nz, ny, nx, 8)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        rng = np.random.default_rng(0)
        hist = []
        steps_per_epoch = len(data) // B
        total = epochs * steps_per_epoch
        flops = 3.0 * net.flops_forward()
        t_start = time.perf_counter()
        it = 0
        for ep in range(epochs):
            order = rng.permutation(len(data))
            loss.zero_()
            for sidx in range(steps_per_epoch):
                idx = order[sidx * B:(sidx + 1) * B]
                for b, j in enumerate(idx):
                    net.x.buf[b].copy_(data[j]["x"].buf[0])
                    tb[b * self.V:(b + 1) * self.V].copy_(data[j]["t"])
                    wb[b * self.V:(b + 1) * self.V].copy_(data[j]["w"])
                cnt = float(sum(int(data[j]["fluid"]) for j in idx)) * 4
                pred = net.forward()
                st = L.lbm_mse_loss(pred.ref, tb.data_ptr(), wb.data_ptr(), 4, 1.0 / cnt, dpred.ref,
                                    loss.data_ptr(), None)
                assert st == 0
                net.zero_grad()
                net.backward(dpred)
                # linear warm-up over the first 5 % of the steps (Adam's
                # first updates at the full rate can throw the network into a
                # poor region), then cosine decay
                warm = max(100, total // 20)
                lr_t = lr * min(1.0, (it + 1) / warm) * 0.5 * (1 + math.cos(math.pi * it / max(1, total)))
                net.adam(lr_t)
                it += 1
            torch.cuda.synchronize()
            l = loss.item() / steps_per_epoch
            hist.append(l)
            log("epoch %d loss %.4e" % (ep, l))
        secs = time.perf_counter() - t_start
        return dict(loss=hist, seconds=secs, tflops=flops * total / secs / 1e12 if secs > 0 else 0.0)

    def predict(self, d):
        """(rho, u) device FP64 fields predicted for one sample."""
        import torch
        S = self.S
        L = S.lib()
        if self.infer is None:
            nx, ny, nz = self.dims
            self.infer = S.UNet(1, nz, ny, nx, seed=0)
            for a, b in zip(self.infer.layers, self.net.layers):
                a.w.copy_(b.w)
                a.b.copy_(b.b)
                a.refresh()
        net = self.infer
        st = L.lbm_surrogate_input(d["solid"].data_ptr(), d["gx"], net.x.ref, None)
        assert st == 0
        pred = net.forward()
        rho = torch.empty(self.V, dtype=torch.float64, device="cuda")
        u = torch.empty(3 * self.V, dtype=torch.float64, device="cuda")
        st = L.lbm_surrogate_fields(pred.ref, d["solid"].data_ptr(), RHO0, d["gx"], self.scale, rho.data_ptr(),
                                    u.data_ptr(), None)
        assert st == 0
        return rho, u


def start_from(lat, rho, u):
    """Initial state from predicted fields: their equilibrium, one step, then
    the mean of the two states (lbm_average_two_steps).  An equilibrium of
    fields that do not solve the discrete equations excites period-two
    components that some pore geometries hardly damp (the velocity then keeps
    a step-to-step oscillation while its two-step mean converges); the mean
    removes them.  Returns the steps taken (1)."""
    lat.set_equilibrium(rho, u)
    lat.step(1)
    lat.average_two_steps()
    return 1


def solve(gx, solid, trainer=None, tol=TOL, dims=DIMS, check_every=100, max_steps=400_000):
    """One run to the residual criterion, from rest or (trainer given) from
    the network's prediction, timed end to end: inference, initial state,
    stepping and residual checks, bracketed by device synchronisation.
    Returns (steps, wall seconds, residual)."""
    import torch
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = make_lattice(gx, solid, None, dims=dims)
    n0 = 0
    if trainer is not None:
        d = dict(solid=torch.from_numpy(np.ascontiguousarray(solid).reshape(-1)).cuda(), gx=gx)
        rho_p, u_p = trainer.predict(d)
        n0 = start_from(lat, rho_p.cpu().numpy().reshape(shape), u_p.cpu().numpy().reshape((3,) + shape))
    (n, _, r), = run_to_steady([lat], check_every=check_every, max_steps=max_steps, tol=tol)
    n += n0
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    lat.close()
    return n, secs, r
