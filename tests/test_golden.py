"""Pins against values the paper prints (tests/golden/, each file citing its
passage): the bytes-per-update model of Sec. 3.1, which sets the algorithmic
bytes every roofline figure here divides by."""
import os

import numpy as np

from paper_1007_1388_amd import lbm

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    out = {}
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = (t.strip() for t in line.split("="))
            out[k] = float(v)
    return out


def test_bytes_per_update_model_reproduces_the_printed_figures():
    g = golden("bytes_per_update.txt")
    q = int(g["n_stencil"])
    assert q == 19
    # GPU: one load and one store of every population; CPU: plus the
    # read-for-ownership of each store
    for prec, s in (("sp", 4), ("dp", 8)):
        assert q * (1 + 1) * s == g["gpu_bytes_" + prec]
        assert q * (1 + 1 + 1) * s == g["cpu_bytes_" + prec]
    # the estimates are bandwidth / bytes, to the rounding of the print
    # (78 GB/s / 152 B = 513 MFLUPS against the printed 516)
    for side, bw in (("cpu_node", g["cpu_node_bandwidth_gbs"]), ("gpu", g["gpu_bandwidth_gbs"])):
        pre = "cpu" if side == "cpu_node" else "gpu"
        for prec in ("sp", "dp"):
            est = bw * 1e3 / g["%s_bytes_%s" % (pre, prec)]
            printed = g["%s_estimate_%s_mflups" % (side, prec)]
            assert abs(est - printed) / printed < 0.01, (side, prec, est, printed)


def test_storage_types_match_the_model():
    """The binding's storage types give the printed GPU bytes per update
    (19 loads + 19 stores), and the 16-bit formats half of SP."""
    g = golden("bytes_per_update.txt")
    size = {p: np.dtype(lbm.STORAGE_DTYPE[lbm.PRECISIONS[p]]).itemsize for p in ("f32", "f64", "f16s", "bf16s")}
    assert 19 * 2 * size["f32"] == g["gpu_bytes_sp"]
    assert 19 * 2 * size["f64"] == g["gpu_bytes_dp"]
    assert 19 * 2 * size["f16s"] == g["gpu_bytes_sp"] / 2 == 19 * 2 * size["bf16s"]
