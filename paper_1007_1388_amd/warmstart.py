"""Learned warm start of the porous-channel solver: data, training, evaluation.

  python -m paper_1007_1388_amd.warmstart [--train N] [--test M] [--epochs E] [--out report.json]

1. Data: N porous channels 64 x 64 x 128 (x, y periodic, walls in z), solid
   fraction uniform in [5 %, 20 %], sphere radii 3..8 (trapped cells and
   isolated pores filled, see inputs.fill_trapped_cells), g_x log-uniform in
   [5e-7, 5e-6], tau 0.7, each run from rest by the lattice Boltzmann solver
   until the residual ||u^n - u^(n-2)|| / (2 ||u^n||) drops below 1e-6.
2. Training: the U-Net of surrogate.py on (mask, g_x) -> (u, rho - rho0)/g_x,
   BF16 MFMA kernels, FP32 master weights, Adam, masked MSE on fluid cells.
3. Evaluation on M held-out seeds: steps and wall time to residual 1e-6 from
   rest and from the network's prediction (inference included), the
   difference of the two converged fields, and the distance of each from a
   tightly converged FP64 reference (two-step residual 1e-10).

The solver judges the network: a prediction only sets the initial state, and
both runs stop on the same residual criterion of the same solver.
"""
import argparse
import json
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


def sample(seed):
    """Geometry and force of one sample (seeded)."""
    rng = np.random.default_rng(1_000_003 + seed)
    frac = float(rng.uniform(0.05, 0.20))
    gx = float(10 ** rng.uniform(np.log10(5e-7), np.log10(5e-6)))
    solid = inputs.porous_spheres(DIMS, target_fraction=frac, radius=(3, 8), seed=seed)
    # cells with undamped period-two momentum (and pockets) would keep the
    # step-to-step residual from ever reaching the tolerance
    solid = inputs.fill_trapped_cells(solid)
    return solid, gx, float(solid.mean())


def make_lattice(gx, solid, stream, precision="f32"):
    lat = lbm.Lattice(DIMS, walls=(False, False, True), tau=TAU, rho0=RHO0, force=(gx, 0, 0),
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


def generate(seeds, concurrent=8, log=print):
    """Steady states for `seeds`; returns list of dicts with device tensors."""
    import torch
    from paper_1007_1388_amd import surrogate as S
    L = S.lib()
    out = []
    streams = [torch.cuda.Stream() for _ in range(concurrent)]
    V = DIMS[0] * DIMS[1] * DIMS[2]
    for i0 in range(0, len(seeds), concurrent):
        chunk = seeds[i0:i0 + concurrent]
        geo = [sample(s) for s in chunk]
        lats = [make_lattice(gx, solid, streams[k].cuda_stream) for k, (solid, gx, _) in enumerate(geo)]
        res = run_to_steady(lats)
        for k, lat in enumerate(lats):
            solid, gx, frac = geo[k]
            rho, u = lat.macroscopic_device()
            sol = torch.from_numpy(solid.reshape(-1)).cuda()
            out.append(dict(seed=chunk[k], gx=gx, frac=frac, solid=sol, rho=rho, u=u, steps=res[k][0],
                            secs=res[k][1], resid=res[k][2]))
            lat.close()
        log("generated %d/%d (steps %s)" % (len(out), len(seeds), [r[0] for r in res]))
    return out


class Trainer:
    def __init__(self, batch=4, seed=0, scale=None):
        from paper_1007_1388_amd import surrogate as S
        self.S = S
        self.batch = batch
        nx, ny, nz = DIMS
        self.net = S.UNet(batch, nz, ny, nx, seed=seed)
        self.infer = None
        self.scale = scale
        self.V = nx * ny * nz

    def prepare(self, data):
        """Network inputs and normalised targets of every sample (kernels)."""
        import torch
        S = self.S
        L = S.lib()
        nx, ny, nz = DIMS
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
        nx, ny, nz = DIMS
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
                # cosine learning-rate decay
                lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / max(1, total)))
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
            nx, ny, nz = DIMS
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


def evaluate(trainer, seeds, log=print):
    """Time to residual 1e-6 from rest and from the prediction, per seed."""
    import torch
    rows = []
    nx, ny, nz = DIMS
    shape = (nz, ny, nx)
    for s in seeds:
        solid, gx, frac = sample(s)
        d = dict(solid=torch.from_numpy(solid.reshape(-1)).cuda(), gx=gx)
        # from rest
        torch.cuda.synchronize()
        lat = make_lattice(gx, solid, None)
        (n0, t0, r0), = run_to_steady([lat])
        rho0_, u0_ = lat.macroscopic()
        lat.close()
        # warm start: inference + initial state + solve, all timed
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        rho_p, u_p = trainer.predict(d)
        lat = make_lattice(gx, solid, None)
        lat.set_equilibrium(rho_p.cpu().numpy().reshape(shape), u_p.cpu().numpy().reshape((3,) + shape))
        t_inf = time.perf_counter() - t_a
        (n1, t1, r1), = run_to_steady([lat])
        rho1_, u1_ = lat.macroscopic()
        lat.close()
        t1 += t_inf
        # tightly converged reference: FP64 storage, continued from the
        # rest solution to a two-step residual of 1e-10
        lat = make_lattice(gx, solid, None, precision="f64")
        lat.set_equilibrium(rho0_, u0_)
        (n2, _, r2), = run_to_steady([lat], max_steps=200_000, tol=1e-10)
        _, u2_ = lat.macroscopic()
        lat.close()
        fluid = solid == 0
        ref = u0_[:, fluid]
        tight = u2_[:, fluid]
        nt = np.linalg.norm(tight)
        diff = np.linalg.norm(u1_[:, fluid] - ref) / np.linalg.norm(ref)
        pred_err = np.linalg.norm(u_p.cpu().numpy().reshape((3,) + shape)[:, fluid] - ref) / np.linalg.norm(ref)
        rows.append(dict(seed=s, gx=gx, solid_frac=frac, steps_rest=n0, secs_rest=t0, steps_warm=n1, secs_warm=t1,
                         infer_secs=t_inf, final_diff=diff, pred_err=pred_err, ref_steps=n2, ref_resid=r2,
                         dist_rest=float(np.linalg.norm(ref - tight) / nt),
                         dist_warm=float(np.linalg.norm(u1_[:, fluid] - tight) / nt)))
        log("seed %d: rest %d steps %.3fs, warm %d steps %.3fs (pred err %.3e, final diff %.2e, to the tight "
            "reference: rest %.2e warm %.2e)" % (s, n0, t0, n1, t1, pred_err, diff, rows[-1]["dist_rest"],
                                                rows[-1]["dist_warm"]))
    return rows


def summarize(rows):
    def q(key):
        v = np.array([r[key] for r in rows], dtype=float)
        return dict(median=float(np.median(v)), q25=float(np.percentile(v, 25)), q75=float(np.percentile(v, 75)))
    return dict(n=len(rows), steps_rest=q("steps_rest"), steps_warm=q("steps_warm"), secs_rest=q("secs_rest"),
                secs_warm=q("secs_warm"), pred_err=q("pred_err"), final_diff=q("final_diff"),
                dist_rest=q("dist_rest"), dist_warm=q("dist_warm"), ref_steps=q("ref_steps"),
                speedup_median=float(np.median([r["secs_rest"] / r["secs_warm"] for r in rows])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--concurrent", type=int, default=8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    data = generate(list(range(args.train)), concurrent=args.concurrent, log=log)
    t_gen = time.perf_counter() - t0
    log("generation %.1f s" % t_gen)
    for d in data:
        d["fluid"] = int((d["solid"] == 0).sum().item())
    tr = Trainer(batch=args.batch)
    tr.prepare(data)
    info = tr.train(data, epochs=args.epochs, lr=args.lr, log=log)
    for d in data:
        d.clear()
    rows = evaluate(tr, list(range(10000, 10000 + args.test)), log=log)
    rep = dict(train_samples=args.train, test_samples=args.test, epochs=args.epochs, batch=args.batch,
               generation_seconds=t_gen, training=info, scale=tr.scale, summary=summarize(rows), rows=rows,
               forward_gflop_per_sample=tr.net.flops_forward() / args.batch / 1e9)
    log(json.dumps(rep["summary"]))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)


if __name__ == "__main__":
    main()
