"""Benchmark: D3Q19 BGK stream-collide throughput on one MI355X.

Default workload: the force-driven plane Poiseuille channel, 256^3 cells,
periodic in x and y, half-way bounce-back walls in z, g_x = 1e-6, tau = 0.8,
started from rest, FP32 storage (and FP64 beside it).  One step = one sweep of
every Block (pull, bounce-back, collision) over the whole domain plus the
ghost-layer exchange.  Median of 3 timed repeats.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--seed S]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    """Hash of the sources that decide what the sweep moves through HBM: the
    kernels, the data layout, and the runtime (work-item order and launch
    shapes)."""
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_internal.h", "lbm_runtime.hip"):
        with open(os.path.join(ROOT, "paper_1007_1388_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(name, src_hash, seed=0):
    """HBM bytes per sweep launch from committed rocprofv3 counter summaries,
    or None when absent, taken on a different kernel source or on another
    seed of the workload."""
    path = os.path.join(PROFILE_DIR, name)
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != src_hash or d.get("seed", 0) != seed:
        return None
    return d.get("hbm_bytes_per_launch")


def workload(name, seed=0):
    from paper_1007_1388_amd import inputs
    p = inputs.preset(name)
    blocks = None
    solid = None
    if name == "porous512":
        blocks = inputs.uneven_blocks(p["dims"], p["block_edges"], seed=seed)
        solid = inputs.porous_spheres(p["dims"], p["solid_fraction"], p["radius"], seed=seed)
    return p, blocks, solid


def time_gpu(p, blocks, solid, precision, fp64_math, steps, warmup, schedule=None, autotune=None,
             timed_launches=200, repeats=3):
    """Timed region: `steps` steps (HIP-graph replays) bracketed by a
    synchronize and HIP events on the context's stream, `repeats` times in a
    row; the median repeat counts.  Then `timed_launches` further steps
    launched one by one with an event pair around every kernel give the
    sweep kernel's own mean duration."""
    import torch
    from paper_1007_1388_amd import lbm
    lat = lbm.Lattice(p["dims"], blocks=blocks, walls=p["walls"], wall_u=p["wall_u"], tau=p["tau"],
                      force=p["force"], precision=precision, fp64_math=fp64_math)
    if solid is not None:
        lat.set_geometry(solid)
    if schedule:
        lat.set_schedule(**schedule)
    if autotune:
        lat.autotune(autotune, trial_steps=10)
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    walls, gpus = [], []
    for _ in range(max(1, repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        lat.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        gpus.append(e0.elapsed_time(e1))
    order = sorted(range(len(walls)), key=lambda k: walls[k])
    mid = order[len(order) // 2]
    wall, gpu_ms = walls[mid], gpus[mid]
    sweep_ms, exch_ms = lat.step_timed(timed_launches) if timed_launches else (None, None)
    info = lat.info()
    sched = lat.schedule
    mass, _ = lat.sums()   # finite-check of the run (raises on instability)
    lat.close()
    return dict(wall=wall, walls=walls, step_ms=gpu_ms / steps, sweep_ms=sweep_ms, exchange_ms=exch_ms,
                info=info, schedule=sched, mass=mass)


def copy_probe(nbytes=1 << 30, reps=10):
    """Attainable HBM bandwidth of the library's 16-byte copy kernel (the
    paper's own benchmark method, Sec. 3.1): GB/s counting read + write."""
    import torch
    from paper_1007_1388_amd import lbm
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    ms = lbm.lbm_bw_probe(b.data_ptr(), a.data_ptr(), nbytes, reps, torch.cuda.current_stream().cuda_stream)
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


# copy-type patterns of lbm_hbm_probe whose best rate is the ceiling the
# sweep (every stored value read once and written once) is read against:
# (kind, unroll, nontemporal, grid)
CEILING_PROBES = [(2, u, 1, g) for u in (1, 2) for g in (256, 512, 1024, 4096)] + \
                 [(3, u, 1, g) for u in (4, 8) for g in (1024, 8192, 16384)] + \
                 [(5, u, 1, g) for u in (1, 2, 4) for g in (256, 512, 1024, 4096)] + [(6, 1, 1, 0)]


def copy_ceiling(nbytes=2 << 30, reps=4):
    """Best copy-type bandwidth (GB/s, read + write) over CEILING_PROBES on
    `nbytes` buffers, and the pattern that reached it."""
    import torch
    from paper_1007_1388_amd import lbm
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream().cuda_stream
    best = (0.0, None)
    for kind, unroll, nt, grid in CEILING_PROBES:
        ms = lbm.lbm_hbm_probe(kind, unroll, nt, a.data_ptr(), b.data_ptr(), nbytes, grid, reps, st)
        moved = 2 * nbytes
        if kind == 5:
            per = nbytes // 19 // 4096 * 4096
            while 19 * per + 18 * 768 > nbytes:
                per -= 4096
            moved = 2 * 19 * per
        gbs = moved / (ms * 1e-3) / 1e9
        if gbs > best[0]:
            best = (gbs, dict(kind=kind, unroll=unroll, nontemporal=nt, grid=grid))
    del a, b
    return best


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, solid, seconds=12.0, single_steps=3):
    """The CPU FP64 oracle on the host cores, on a bounded sample of the same
    workload: the full domain for as many steps as fit in ~seconds on all
    OpenMP threads, then `single_steps` steps on one thread."""
    import oracle
    o = oracle.OracleLBM(p["dims"], walls=p["walls"], wall_u=p["wall_u"], tau=p["tau"], force=p["force"])
    if solid is not None:
        o.set_geometry(solid)
    cores = oracle.max_threads()
    o.step(1)  # touch memory
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        n += 1
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    t1 = time.perf_counter()
    o.step(single_steps)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    cells = o.ncell if solid is None else int((solid == 0).sum())
    o.close()
    return dict(value=round(cells * n / dt / 1e6, 3), unit="MLUPS", cores=cores, kind="oracle",
                sample="%s full domain%s: %d steps after 1 warm-up on %d OpenMP threads, then %d steps on 1 "
                       "thread; FP64" % ("x".join(map(str, p["dims"])), " (porous)" if solid is not None else "",
                                         n, cores, single_steps),
                single_thread_value=round(cells * single_steps / dt1 / 1e6, 3), cpu_model=cpu_model())


def porous_leg(seed=0, steps=1000, warmup=100):
    """The porous channel 512x256x256 in its seeded uneven Blocks with
    spheres (FP32 storage): MLUPS and the sweep's roofline fraction."""
    p, blocks, solid = workload("porous512", seed)
    r = time_gpu(p, blocks, solid, "f32", False, steps, warmup, {"graph_steps": 10}, None, repeats=1)
    info = r["info"]
    nf = info["n_fluid"]
    achieved = nf * info["bytes_per_update"] / (r["sweep_ms"] * 1e-3) / 1e9
    tr = traffic_from_profile("sweep_f32_porous512_pmc.json", kernel_source_hash(), seed)
    return {"workload": "porous512 512x256x256, seed %d, %d uneven Blocks, solid fraction %.4f"
                        % (seed, info["n_blocks"], float(solid.mean())),
            "value": round(nf * steps / r["wall"] / 1e6, 1), "unit": "MLUPS", "steps": steps,
            "ms_per_step": round(r["wall"] * 1e3 / steps, 5), "kernel_ms": round(r["sweep_ms"], 5),
            "exchange_ms": round(r["exchange_ms"], 5), "bytes_per_update": info["bytes_per_update"],
            "achieved_gbs": round(achieved, 1), "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic_gbs": (round(tr / (r["sweep_ms"] * 1e-3) / 1e9, 1) if tr else None),
            "schedule": r["schedule"]}


def precision_leg(n=384, steps=5000, tau=0.55, lid=0.1):
    """The n^3 lid-driven cavity in FP64, FP32, shifted FP16 and shifted BF16
    storage for `steps` steps: MLUPS, the 16-bit speedup over FP32, and the
    normwise velocity error of each run against the FP64 run."""
    import numpy as np
    import torch
    from paper_1007_1388_amd import lbm
    out, ref = {}, None
    for prec in ("f64", "f32", "f16s", "bf16s"):
        lat = lbm.Lattice((n, n, n), walls=(True, True, True), wall_u={"+z": (lid, 0, 0)}, tau=tau,
                          precision=prec)
        lat.set_schedule(graph_steps=10)
        lat.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps - 10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # per-launch sweep times while the GPU is still busy (after the idle
        # time of a host copy its first launches run at a lower clock)
        sweep_ms, _ = lat.step_timed(100)
        _, u = lat.macroscopic()
        info = lat.info()
        lat.close()
        achieved = n ** 3 * info["bytes_per_update"] / (sweep_ms * 1e-3) / 1e9
        row = {"value": round(n ** 3 * (steps - 10) / dt / 1e6, 1), "kernel_ms": round(sweep_ms, 5),
               "bytes_per_update": info["bytes_per_update"], "roofline_frac": round(achieved / HBM_PEAK_GBS, 4)}
        if prec == "f64":
            ref = u
        else:
            d = u - ref
            row["err_vs_f64_inf"] = float(np.abs(d).max() / np.abs(ref).max())
            row["err_vs_f64_l2"] = float(np.sqrt((d ** 2).sum() / (ref ** 2).sum()))
        out[prec] = row
        del u
    for prec in ("f16s", "bf16s"):
        out[prec]["speedup_vs_f32"] = round(out[prec]["value"] / out["f32"]["value"], 3)
    return {"workload": "cavity384 %d^3 lid-driven cavity, tau %g, lid %g, %d steps (+100 timed per launch)"
                        % (n, tau, lid, steps),
            "unit": "MLUPS", "storage": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=3, help="timed repeats of --steps steps; the median counts")
    ap.add_argument("--workload", default="poiseuille256",
                    choices=["poiseuille256", "porous512", "cavity384", "cavity32"])
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16s", "bf16s"])
    ap.add_argument("--seed", type=int, default=0, help="geometry and tiling seed of porous512")
    ap.add_argument("--fp64-math", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--graph-steps", type=int, default=10, help="time steps per captured HIP graph")
    ap.add_argument("--fused", type=int, default=None,
                    help="ghost exchange: 0 copy kernel, 1 fused into the sweep, 2 x faces by the sweep and "
                         "the rest by the copy kernel (default: the library's, 0 for one Block, 2 for several)")
    ap.add_argument("--autotune", default=None, help="autotune cache file (runs the schedule autotuner)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the porous-channel and storage-precision legs of the default workload")
    ap.add_argument("--copy-only", type=int, default=0,
                    help="only run the copy probe on this many bytes (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (the Block exchange between GPUs is a "
              "design, not code); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.init()
    if args.copy_only:
        gbs = copy_probe(args.copy_only, reps=1)
        print(json.dumps({"copy_probe_bytes": args.copy_only, "copy_gbs": round(gbs, 1)}), flush=True)
        return
    copy_gbs = copy_probe()
    ceil_gbs, ceil_pattern = copy_ceiling()
    p, blocks, solid = workload(args.workload, args.seed)
    prec = args.precision
    f64m = bool(args.fp64_math) and prec in ("f32", "f64")
    sched = {"graph_steps": args.graph_steps}
    if args.fused is not None:
        sched["fused_exchange"] = args.fused
    r = time_gpu(p, blocks, solid, prec, f64m, args.steps, args.warmup, sched, args.autotune,
                 repeats=args.repeats)
    info = r["info"]
    nf = info["n_fluid"]
    mlups = nf * args.steps / r["wall"] / 1e6
    bpu = info["bytes_per_update"]
    # algorithmic bytes of one sweep launch over its measured mean duration
    achieved = nf * bpu / (r["sweep_ms"] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    tr = traffic_from_profile("sweep_%s_%s_pmc.json" % (prec, args.workload), src_hash,
                              args.seed if solid is not None else 0)
    if prec == "f64" or (prec == "f32" and f64m):
        arith = "f64"
    elif prec == "f32":
        arith = "f32 even part of feq/F; f64 velocity, odd part and update"
    else:
        arith = "f32 (storage %s, shifted)" % prec
    if solid is not None:
        extra = {"seed": args.seed, "solid_fraction": round(float(solid.mean()), 5)}
    else:
        extra = {}
    out = {
        "metric": "D3Q19 MLUPS (fluid lattice-cell updates per second, millions)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] * 1e3 / args.steps, 5),
        "repeats_ms_per_step": [round(w * 1e3 / args.steps, 5) for w in r["walls"]],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if arith == "f64" else "f32"),
        "data": "synthetic",
        "config": {"workload": "%s %s" % (args.workload, "x".join(map(str, p["dims"]))),
                   "storage": prec, "arithmetic": arith,
                   "tau": p["tau"], "force": list(p["force"]), "blocks": info["n_blocks"],
                   "fluid_cells": nf, "schedule": r["schedule"], "parallelism": "1 GPU", **extra},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (round(tr / (r["sweep_ms"] * 1e-3) / 1e9, 1) if tr else None),
                     "kernel": "k_sweep", "kernel_ms": round(r["sweep_ms"], 5),
                     "exchange_ms": round(r["exchange_ms"], 5), "step_ms_events": round(r["step_ms"], 5),
                     "bytes_per_update": bpu, "copy_probe_gbs": round(copy_gbs, 1),
                     "copy_ceiling_gbs": round(ceil_gbs, 1), "copy_ceiling_pattern": ceil_pattern,
                     "frac_of_copy": round(achieved / ceil_gbs, 4), "kernel_hash": src_hash},
    }
    if not args.no_f64 and prec == "f32":
        n64 = max(1, args.steps // 2)
        r64 = time_gpu(p, blocks, solid, "f64", False, n64, args.warmup, sched, args.autotune, repeats=1)
        i64 = r64["info"]
        m64 = i64["n_fluid"] * n64 / r64["wall"] / 1e6
        a64 = i64["n_fluid"] * i64["bytes_per_update"] / (r64["sweep_ms"] * 1e-3) / 1e9
        out["f64_storage"] = {"value": round(m64, 1), "unit": "MLUPS", "steps": n64,
                              "roofline_frac": round(a64 / HBM_PEAK_GBS, 4), "achieved_gbs": round(a64, 1),
                              "kernel_ms": round(r64["sweep_ms"], 5)}
    if not args.no_legs and args.workload == "poiseuille256" and prec == "f32":
        out["porous512"] = porous_leg(seed=0)
        out["cavity384_precision"] = precision_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, solid)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
