"""Storage-precision study of the lid-driven cavity (shifted FP16/BF16 vs FP32/FP64).

  python -m paper_1007_1388_amd.precision [--n 384] [--steps 5000] [--small 96] [--out report.json]

Runs the n^3 cavity (tau 0.55, lid 0.1 on +z) for `steps` steps in every
storage precision on the GPU, times each, and reports the normwise velocity
error of each run against (a) the GPU FP64 run of the same size and (b) for
the small instance, the CPU FP64 oracle.  Shifted storage keeps f~ = f - w_i
rho0 (Sec. 2.1), so the stored values are centred on zero.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1007_1388_amd import lbm  # noqa: E402

PRECS = ["f64", "f32", "f16s", "bf16s"]


def run(n, steps, prec, tau, lid):
    import torch
    lat = lbm.Lattice((n, n, n), walls=(True, True, True), wall_u={"+z": (lid, 0, 0)}, tau=tau,
                      precision=prec)
    lat.set_schedule(graph_steps=10)
    lat.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps - 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rho, u = lat.macroscopic()
    m, _ = lat.sums()
    lat.close()
    return dict(u=u, rho=rho, mlups=n ** 3 * (steps - 10) / dt / 1e6, seconds=dt, mass=m)


def err(u, ref):
    d = u - ref
    return dict(linf=float(np.abs(d).max() / np.abs(ref).max()),
                l2=float(np.sqrt((d ** 2).sum() / (ref ** 2).sum())))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=384)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--small", type=int, default=96)
    ap.add_argument("--tau", type=float, default=0.55)
    ap.add_argument("--lid", type=float, default=0.1)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    rep = dict(n=args.n, steps=args.steps, tau=args.tau, lid=args.lid, large={}, small={})
    # small instance against the CPU oracle
    import oracle
    o = oracle.OracleLBM((args.small,) * 3, walls=(True, True, True), wall_u={"+z": (args.lid, 0, 0)},
                         tau=args.tau)
    t0 = time.perf_counter()
    o.step(args.steps)
    rep["small"]["oracle_seconds"] = time.perf_counter() - t0
    _, u_o = o.macroscopic()
    o.close()
    for p in PRECS:
        r = run(args.small, args.steps, p, args.tau, args.lid)
        rep["small"][p] = dict(err_vs_oracle=err(r["u"], u_o), mlups=r["mlups"])
        print(p, "small", rep["small"][p], flush=True)
    # large instance against the GPU FP64 run
    ref = None
    for p in PRECS:
        r = run(args.n, args.steps, p, args.tau, args.lid)
        if not np.isfinite(r["mass"]):
            rep["large"][p] = dict(unstable=True)
            continue
        if p == "f64":
            ref = r["u"]
        rep["large"][p] = dict(mlups=r["mlups"], seconds=r["seconds"],
                               err_vs_gpu_f64=err(r["u"], ref) if ref is not None else None,
                               umax=float(np.abs(r["u"]).max()))
        print(p, "large", rep["large"][p], flush=True)
        del r
    f32 = rep["large"].get("f32", {}).get("mlups")
    for p in ("f16s", "bf16s"):
        if f32 and "mlups" in rep["large"].get(p, {}):
            rep["large"][p]["speedup_vs_f32"] = rep["large"][p]["mlups"] / f32
    print(json.dumps({k: v for k, v in rep.items() if k != "rows"}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)


if __name__ == "__main__":
    main()
