"""Storage precision on the 96^3 instance of the 384^3 lid-driven cavity
(tau 0.55, lid u_x = 0.1 on +z, 5000 steps): every storage precision of the
HIP library against the CPU FP64 oracle, normwise velocity error over the
whole cavity.  Shifted storage keeps f~ = f - w_i rho0 (Sec. 2.1), so the
16-bit values are centred on zero; arithmetic is FP32 and the reductions FP64.

Bars: FP64 1e-12 and FP32 1e-5 (the parity bars); shifted FP16 5e-3 and
shifted BF16 5e-2 in the infinity norm (measured on gfx950: 1.3e-3 and
1.7e-2), and the L2 norm below the infinity norm.
"""
import numpy as np
import pytest

from tests.helpers import gpu_lattice, run_oracle

pytestmark = pytest.mark.gpu

CASE = dict(dims=(96, 96, 96), walls=(True, True, True), wall_u={"+z": (0.1, 0.0, 0.0)}, tau=0.55)
STEPS = 5000
BARS = {"f64": 1e-12, "f32": 1e-5, "f16s": 5e-3, "bf16s": 5e-2}


@pytest.fixture(scope="module")
def oracle_u():
    o = run_oracle(CASE, STEPS)
    _, u = o.macroscopic()
    o.close()
    return u


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s", "bf16s"])
def test_cavity96_5000_steps_against_oracle(oracle_u, precision):
    lat = gpu_lattice(CASE, precision=precision)
    lat.set_schedule(graph_steps=10)
    lat.step(STEPS)
    _, u = lat.macroscopic()
    mass, _ = lat.sums()
    lat.close()
    assert np.isfinite(mass)
    d = u - oracle_u
    linf = np.abs(d).max() / np.abs(oracle_u).max()
    l2 = np.sqrt((d ** 2).sum() / (oracle_u ** 2).sum())
    print("cavity 96^3, %d steps, %s storage: velocity error inf %.3e, L2 %.3e" % (STEPS, precision, linf, l2))
    assert linf <= BARS[precision] and l2 <= linf, (precision, linf, l2)
