"""Size and Block-count sweeps of the D3Q19 sweep on one GPU.

  python -m paper_1007_1388_amd.sweeps size   [--steps 200]   # single-Block periodic cubes
  python -m paper_1007_1388_amd.sweeps blocks [--steps 200]   # 384^3 split into 1..216 Blocks, porous
  python -m paper_1007_1388_amd.sweeps open   [--steps 200]   # open x faces against periodic x
  python -m paper_1007_1388_amd.sweeps pad    [--steps 200]   # odd Block sizes and row padding
  python -m paper_1007_1388_amd.sweeps hbm                    # HBM ceilings of read, write, copy
  python -m paper_1007_1388_amd.sweeps hetero [--steps 50]    # host-CPU Blocks next to the GPU's

size:   periodic cube N^3 (N = 64..512 step 32) as one Block, FP32 and FP64
        storage, started from rest with g_x = 1e-6, tau 0.8: MLUPS against N,
        the single-Block scaling study of Sec. 5.1.
blocks: the 384^3 periodic cube as 1, 8, 27, 64 and 216 equal Blocks, and
        the 512x256x256 porous channel as its uneven Blocks; per-launch times
        of the sweep and of the separate ghost exchange (HIP events) for the
        three exchange schedules (0 copy kernel, 2 x faces written by the
        sweep, 1 fully fused), for the porous channel in its uneven Blocks and
        for 64 uneven Blocks (4x4x4, edges from {32, 48, 64}): the cost of
        Blocks and of their on-GPU copies, Sec. 5.1.
pad:    single-Block periodic cubes of odd and even edge around 64, 70,
        128 and 256 (the paper's odd-size effects, Sec. 5.1) with rows
        aligned to 128-byte lines and no extra padding (row_pad -1) or one
        or two extra lines per row, with streaming stores, and without
        padding with ordinary stores, FP32 and FP64: MLUPS against the edge.
hbm:    read-only, write-only and copy streams over 2 GiB buffers (well past
        the 256 MB Infinity Cache) with 1-8 accesses in flight per thread,
        streaming or ordinary, several grid sizes: the attainable bandwidth
        of each pattern (lbm_hbm_probe), against which the sweep (one read
        and one write of every value, the copy pattern) is read.
hetero: the porous 512x256x256 channel in its uneven Blocks, FP32 (Sec. 5.3's
        heterogeneous study on one node): the GPU alone, then the last k
        Blocks on the host CPU (k = 1, 2, 4, 8, 16, 16 threads) with the GPU
        sweep, host sweep, exchange and whole-step times of phase-timed steps
        and the step time of lbm_step's pipelined steps; the host sweep's
        rate against its thread count on the last Block; and the static load
        balance (lbm_balance_host_blocks).
open:   a 512x256x256 duct (y periodic, z walls), FP32: x periodic with a
        body force against a velocity inlet and a pressure outlet on the x
        faces, as one Block and as 4 Blocks along x; the second column of
        times is then the post-sweep work (exchange and the boundary nodes of
        the open faces).

Prints one JSON line per case.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1007_1388_amd import inputs, lbm  # noqa: E402

HBM_PEAK_GBS = 8000.0


def measure(dims, precision, steps, blocks=None, solid=None, walls=(False, False, False), tau=0.8,
            force=(1e-6, 0.0, 0.0), fused=0, graph_steps=10, open_x=None, row_pad=0, nontemporal=1):
    import torch
    lat = lbm.Lattice(dims, blocks=blocks, walls=walls, tau=tau, force=force, precision=precision,
                      open_x=open_x, row_pad=row_pad)
    if solid is not None:
        lat.set_geometry(solid)
    lat.set_schedule(fused_exchange=fused, graph_steps=graph_steps, nontemporal=nontemporal)
    lat.step(20)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    sweep_ms, exch_ms = lat.step_timed(min(steps, 100))
    info = lat.info()
    lat.sums()
    lat.close()
    nf = info["n_fluid"]
    return dict(step_ms=round(step_ms, 5), sweep_ms=round(sweep_ms, 5), exchange_ms=round(exch_ms, 5),
                mlups=round(nf / step_ms / 1e3, 1),
                sweep_gbs=round(nf * info["bytes_per_update"] / (sweep_ms * 1e-3) / 1e9, 1),
                frac=round(nf * info["bytes_per_update"] / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                blocks=info["n_blocks"], fluid_cells=nf)


def size_sweep(steps, sizes):
    for n in sizes:
        for prec in ("f32", "f64"):
            r = measure((n, n, n), prec, steps)
            print(json.dumps(dict(study="size", n=n, precision=prec, **r)), flush=True)


def block_sweep(steps):
    n = 384
    for k in (1, 2, 3, 4, 6):
        blocks = inputs.uniform_blocks((n, n, n), (k, k, k))
        for fused in (0, 2, 1):
            r = measure((n, n, n), "f32", steps, blocks=blocks, fused=fused)
            print(json.dumps(dict(study="blocks", domain="384^3 periodic", split="%dx%dx%d" % (k, k, k),
                                  precision="f32", fused=fused, **r)), flush=True)
    p = inputs.preset("porous512")
    blocks = inputs.uneven_blocks(p["dims"], p["block_edges"], seed=0)
    solid = inputs.porous_spheres(p["dims"], p["solid_fraction"], p["radius"], seed=0)
    for fused in (0, 2, 1):
        r = measure(p["dims"], "f32", steps, blocks=blocks, solid=solid, walls=p["walls"], tau=p["tau"],
                    force=p["force"], fused=fused)
        print(json.dumps(dict(study="blocks", domain="porous 512x256x256", split="uneven {32,48,64}",
                              precision="f32", fused=fused, **r)), flush=True)
    # the literal 64 uneven Blocks: a 4x4x4 grid with edges from {32, 48, 64},
    # the domain being whatever the edges sum to
    dims, blocks = inputs.uneven_blocks_grid((4, 4, 4), p["block_edges"], seed=0)
    solid = inputs.porous_spheres(dims, p["solid_fraction"], p["radius"], seed=0)
    for fused in (0, 2, 1):
        r = measure(dims, "f32", steps, blocks=blocks, solid=solid, walls=p["walls"], tau=p["tau"],
                    force=p["force"], fused=fused)
        print(json.dumps(dict(study="blocks", domain="porous %s" % "x".join(map(str, dims)),
                              split="4x4x4 uneven {32,48,64}", precision="f32", fused=fused, **r)), flush=True)


def pad_sweep(steps):
    for n in (63, 64, 65, 69, 70, 71, 72, 127, 128, 129, 255, 256, 257):
        for prec in ("f32", "f64"):
            for rp, nt in ((-1, 1), (1, 1), (2, 1), (-1, 0)):
                r = measure((n, n, n), prec, steps, row_pad=rp, nontemporal=nt)
                print(json.dumps(dict(study="pad", n=n, precision=prec, row_pad=rp, nontemporal=nt, **r)),
                      flush=True)


def hbm_sweep(reps=10):
    import torch
    nbytes = 2 << 30
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for kind, name, moved in ((0, "read", 1), (1, "write", 1), (2, "copy", 2)):
        for unroll in (1, 2, 4, 8):
            for nt in (1, 0):
                for grid in (1024, 4096, 16384, 65536):
                    ms = lbm.lbm_hbm_probe(kind, unroll, nt, a.data_ptr(), b.data_ptr(), nbytes, grid, reps, st)
                    gbs = moved * nbytes / (ms * 1e-3) / 1e9
                    print(json.dumps(dict(study="hbm", pattern=name, unroll=unroll, nontemporal=nt, grid=grid,
                                          ms=round(ms, 5), gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))),
                          flush=True)


def hetero_sweep(steps, threads=16):
    import torch
    p = inputs.preset("porous512")
    blocks = inputs.uneven_blocks(p["dims"], p["block_edges"], seed=0)
    solid = inputs.porous_spheres(p["dims"], p["solid_fraction"], p["radius"], seed=0)
    lat = lbm.Lattice(p["dims"], blocks=blocks, walls=p["walls"], tau=p["tau"], force=p["force"], precision="f32")
    lat.set_geometry(solid)
    nb = len(blocks)
    nf = lat.info()["n_fluid"]
    lat.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    print(json.dumps(dict(study="hetero", case="gpu alone", blocks=nb, host_blocks=0, step_ms=round(ms, 4),
                          mlups=round(nf / ms / 1e3, 1))), flush=True)
    # host sweep rate against threads, last Block
    for th in (1, 2, 4, 8, 16):
        lat.set_host_blocks([nb - 1], threads=th)
        lat.step(2)
        g, c, x, s = lat.step_host_timed(max(5, steps // 5))
        fh = _fluid(solid, blocks[nb - 1:])
        print(json.dumps(dict(study="hetero", case="host rate", threads=th, host_fluid=fh, cpu_ms=round(c, 4),
                              host_mlups=round(fh / c / 1e3, 1))), flush=True)
    for k in (1, 2, 4, 8, 16):
        ids = list(range(nb - k, nb))
        lat.set_host_blocks(ids, threads=threads)
        lat.step(2)
        g, c, x, s = lat.step_host_timed(steps)
        # the same split stepped as lbm_step runs it (the next GPU sweep
        # queued behind the exchange)
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        sp = (time.perf_counter() - t0) * 1e3 / steps
        fh = _fluid(solid, blocks[nb - k:])
        print(json.dumps(dict(study="hetero", case="split", threads=threads, host_blocks=k, host_fluid=fh,
                              gpu_sweep_ms=round(g, 4), cpu_sweep_ms=round(c, 4), exchange_ms=round(x, 4),
                              step_ms=round(s, 4), pipelined_step_ms=round(sp, 4),
                              mlups=round(nf / sp / 1e3, 1))), flush=True)
    lat.set_host_blocks([])
    k, tg, th = lat.balance_host_blocks(threads=threads, trial_steps=steps)
    print(json.dumps(dict(study="hetero", case="balance", threads=threads, host_blocks=k, gpu_alone_ms=round(tg, 4),
                          split_ms=round(th, 4))), flush=True)
    lat.close()


def _fluid(solid, blocks):
    n = 0
    for lo, hi in blocks:
        # solid is [z][y][x]
        n += int((solid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] == 0).sum())
    return n


def open_sweep(steps):
    dims = (512, 256, 256)
    opn = {"-x": ("velocity", (0.02, 0.0, 0.0)), "+x": ("pressure", 1.0)}
    for label, walls, force, ox in (("x periodic, g_x = 1e-6", (False, False, True), (1e-6, 0, 0), None),
                                    ("x velocity inlet / pressure outlet", (True, False, True), (0, 0, 0), opn)):
        for nb in (1, 4):
            blocks = inputs.uniform_blocks(dims, (nb, 1, 1))
            for fused in ((0,) if nb == 1 else (0, 2)):
                r = measure(dims, "f32", steps, blocks=blocks, walls=walls, force=force, fused=fused, open_x=ox)
                print(json.dumps(dict(study="open", domain="512x256x256 duct", x=label, split="%dx1x1" % nb,
                                      precision="f32", fused=fused, **r)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["size", "blocks", "open", "pad", "hbm", "hetero"])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--sizes", default="64-512:32")
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    if args.study == "size":
        lo, rest = args.sizes.split("-")
        hi, st = rest.split(":")
        size_sweep(args.steps, range(int(lo), int(hi) + 1, int(st)))
    elif args.study == "open":
        open_sweep(args.steps)
    elif args.study == "pad":
        pad_sweep(args.steps)
    elif args.study == "hbm":
        hbm_sweep()
    elif args.study == "hetero":
        hetero_sweep(args.steps)
    else:
        block_sweep(args.steps)


if __name__ == "__main__":
    main()
