"""Learned warm start of the porous-channel solver: data, training, evaluation.

  python -m paper_1007_1388_amd.warmstart [--train N] [--test M] [--epochs E] [--out report.json]

1. Data: N porous channels 64 x 64 x 128 (x, y periodic, walls in z), solid
   fraction uniform in [5 %, 20 %], sphere radii 3..8 (trapped cells and
   isolated pores filled, see inputs.fill_trapped_cells), g_x log-uniform in
   [5e-7, 5e-6], tau 0.7, each run from rest by the lattice Boltzmann solver
   until the residual ||u^n - u^(n-2)|| / (2 ||u^n||) drops below 1e-6.
2. Training: the U-Net of surrogate.py on (mask, g_x) -> (u, rho - rho0)/g_x,
   BF16 MFMA kernels, FP32 master weights, Adam, masked MSE on fluid cells.
3. Evaluation on M held-out seeds against a tightly converged FP64 reference
   (two-step residual 1e-10): steps and time from rest and from the network's
   prediction (inference included) to the residual criterion 1e-6, and to
   velocity errors of 1e-2, 3e-3, 1e-3 and 3e-4 against the reference.  The
   residual criterion alone flatters the warm start: it stops a run whose
   remaining error decays slowly, and a warm-started run can stop farther
   from the steady state than one from rest.

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


TARGETS = (1e-2, 3e-3, 1e-3, 3e-4)


def reference(gx, solid, tol=1e-10, max_steps=400_000):
    """Tightly converged steady velocity (device, FP64 storage): from rest to
    a two-step residual of `tol`, averaged over two consecutive steps (which
    removes any period-two part); returns (u, steps, residual)."""
    lat = make_lattice(gx, solid, None, precision="f64")
    (n, _, r), = run_to_steady([lat], max_steps=max_steps, tol=tol)
    _, ua = lat.macroscopic_device()
    lat.step(1)
    _, ub = lat.macroscopic_device()
    import torch
    torch.cuda.synchronize()
    lat.close()
    return 0.5 * (ua + ub), n, r


def converge_tracked(lat, u_ref, fluid, check_every=100, max_steps=60_000):
    """Step `lat` until its two-step residual is below TOL and its velocity is
    within the smallest of TARGETS of u_ref (relative 2-norm over fluid
    cells), checking every `check_every` steps.  The error is taken both of
    the velocity itself and of its average over the last two steps: a
    period-two oscillation that bounce-back sustains in some pore geometries
    (and that the two-step residual cannot see) shows only in the first.
    Returns (steps to residual TOL, {target: steps} for the velocity,
    {target: steps} for the two-step average, seconds per step of the
    stepping and residual work alone, final errors (velocity, average))."""
    import torch
    nref = torch.linalg.vector_norm(u_ref[:, fluid])
    hit, hit2, n_res, steps, t_steps = {}, {}, None, 0, 0.0
    err = err2 = float("nan")
    while steps < max_steps:
        t = time.perf_counter()
        lat.step(check_every - 3)
        lat.residual_mark()
        lat.step(2)
        r2, m = lat.residual_since_mark()
        t_steps += time.perf_counter() - t
        _, ua = lat.macroscopic_device()
        t = time.perf_counter()
        lat.step(1)
        torch.cuda.synchronize()
        t_steps += time.perf_counter() - t
        _, u = lat.macroscopic_device()
        torch.cuda.synchronize()
        steps += check_every
        r = r2 / m
        if n_res is None and r < TOL:
            n_res = steps
        err = float(torch.linalg.vector_norm((u - u_ref)[:, fluid]) / nref)
        err2 = float(torch.linalg.vector_norm((0.5 * (u + ua) - u_ref)[:, fluid]) / nref)
        for tg in TARGETS:
            if tg not in hit and err < tg:
                hit[tg] = steps
            if tg not in hit2 and err2 < tg:
                hit2[tg] = steps
        if (n_res is not None and len(hit) == len(TARGETS) and len(hit2) == len(TARGETS)) or not math.isfinite(r):
            break
    return n_res, hit, hit2, t_steps / max(steps, 1), (err, err2)


def evaluate(trainer, seeds, log=print):
    """Per held-out seed: steps and time from rest and from the network's
    prediction (inference included) to the residual criterion, and to each
    accuracy target against a tightly converged FP64 reference."""
    import torch
    rows = []
    nx, ny, nz = DIMS
    shape = (nz, ny, nx)
    for s in seeds:
        solid, gx, frac = sample(s)
        d = dict(solid=torch.from_numpy(solid.reshape(-1)).cuda(), gx=gx)
        fluid = torch.from_numpy(solid == 0).cuda()
        u_ref, n_ref, r_ref = reference(gx, solid)
        # from rest
        torch.cuda.synchronize()
        lat = make_lattice(gx, solid, None)
        n0, hit0, avg0, sps0, e0 = converge_tracked(lat, u_ref, fluid)
        lat.close()
        # warm start: inference and initial state timed
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        rho_p, u_p = trainer.predict(d)
        lat = make_lattice(gx, solid, None)
        lat.set_equilibrium(rho_p.cpu().numpy().reshape(shape), u_p.cpu().numpy().reshape((3,) + shape))
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t_a
        n1, hit1, avg1, sps1, e1 = converge_tracked(lat, u_ref, fluid)
        lat.close()
        nref = torch.linalg.vector_norm(u_ref[:, fluid])
        pred_err = float(torch.linalg.vector_norm((u_p.reshape((3,) + shape) - u_ref)[:, fluid]) / nref)
        row = dict(seed=s, gx=gx, solid_frac=frac, ref_steps=n_ref, ref_resid=r_ref, infer_secs=t_inf,
                   pred_err=pred_err, sps_rest=sps0, sps_warm=sps1, err_end_rest=e0[0], err_end_warm=e1[0],
                   avgerr_end_rest=e0[1], avgerr_end_warm=e1[1],
                   steps_rest=n0, steps_warm=n1,
                   secs_rest=None if n0 is None else n0 * sps0,
                   secs_warm=None if n1 is None else t_inf + n1 * sps1)
        for tg in TARGETS:
            k = "%.0e" % tg
            row["steps_rest_" + k] = hit0.get(tg)
            row["steps_warm_" + k] = hit1.get(tg)
            row["secs_rest_" + k] = None if tg not in hit0 else hit0[tg] * sps0
            row["secs_warm_" + k] = None if tg not in hit1 else t_inf + hit1[tg] * sps1
            row["steps_rest_avg_" + k] = avg0.get(tg)
            row["steps_warm_avg_" + k] = avg1.get(tg)
            row["secs_rest_avg_" + k] = None if tg not in avg0 else avg0[tg] * sps0
            row["secs_warm_avg_" + k] = None if tg not in avg1 else t_inf + avg1[tg] * sps1
        rows.append(row)
        log("seed %d: pred err %.3f; residual 1e-6: rest %s warm %s steps; to error 1e-3: rest %s warm %s steps "
            "(two-step average: rest %s warm %s); final errors rest %.1e/%.1e warm %.1e/%.1e; inference %.1f ms"
            % (s, pred_err, n0, n1, hit0.get(1e-3), hit1.get(1e-3), avg0.get(1e-3), avg1.get(1e-3), e0[0], e0[1],
               e1[0], e1[1], 1e3 * t_inf))
    return rows


def summarize(rows):
    def q(key):
        v = np.array([r[key] for r in rows if r[key] is not None], dtype=float)
        if v.size == 0:
            return None
        return dict(median=float(np.median(v)), q25=float(np.percentile(v, 25)),
                    q75=float(np.percentile(v, 75)), n=int(v.size))

    def speedup(kr, kw):
        v = [r[kr] / r[kw] for r in rows if r[kr] is not None and r[kw] is not None]
        return float(np.median(v)) if v else None
    out = dict(n=len(rows), pred_err=q("pred_err"), ref_steps=q("ref_steps"), infer_secs=q("infer_secs"),
               steps_rest=q("steps_rest"), steps_warm=q("steps_warm"), secs_rest=q("secs_rest"),
               secs_warm=q("secs_warm"), speedup_residual=speedup("secs_rest", "secs_warm"))
    for tg in TARGETS:
        k = "%.0e" % tg
        out["steps_rest_" + k] = q("steps_rest_" + k)
        out["steps_warm_" + k] = q("steps_warm_" + k)
        out["speedup_" + k] = speedup("secs_rest_" + k, "secs_warm_" + k)
        out["steps_rest_avg_" + k] = q("steps_rest_avg_" + k)
        out["steps_warm_avg_" + k] = q("steps_warm_avg_" + k)
        out["speedup_avg_" + k] = speedup("secs_rest_avg_" + k, "secs_warm_avg_" + k)
    out["err_end_warm"] = q("err_end_warm")
    out["avgerr_end_warm"] = q("avgerr_end_warm")
    out["err_end_rest"] = q("err_end_rest")
    return out


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
