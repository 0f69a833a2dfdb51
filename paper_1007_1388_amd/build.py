"""Build the gfx950 HIP library in-tree: paper_1007_1388_amd/liblbm_hip.so.

Usage: python -m paper_1007_1388_amd.build   (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["lbm_kernels.hip", "lbm_runtime.hip", "conv3d.hip", "hbm_probe.hip", "lbm_host.cpp"]

# Packed FP32 instructions are kept off: the code is plain scalar float/double.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wno-unused-result"]
# per-source extras: the convolution kernels keep MFMA accumulators in
# VGPRs, which spares the AGPR copies the K loop otherwise carries
EXTRA = {"conv3d.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         # the host sweep of heterogeneous runs: x86-64 FMA for the fused
         # multiply-adds the GPU arithmetic prescribes
         "lbm_host.cpp": ["-mavx2", "-mfma", "-pthread"]}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=3):
    """Compile every HIP source for gfx950 and link liblbm_hip.so (always rebuilds)."""
    objs, procs = [], []
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    for s in srcs:
        obj = os.path.join(CSRC, "_" + os.path.splitext(s)[0] + ".o")
        cmd = [hipcc(), *HIPFLAGS, *EXTRA.get(s, []), "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        objs.append(obj)
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    for s, p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed on %s" % s)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
