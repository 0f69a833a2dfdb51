"""The allocation-free reduction entry point lbm_sums_noalloc against
lbm_sums, through the C ABI: bit for bit, on two calls in a row (the second
on a smaller lattice), and with a schedule whose reduction spreads over the
most workgroup partials."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs, lbm
from tests.helpers import gpu_lattice, prepare

pytestmark = pytest.mark.gpu


def _case(dims, seed):
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=1e-2)
    solid = inputs.porous_spheres(dims, target_fraction=0.08, radius=(2, 3), seed=seed)
    u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(False, False, True), tau=0.7, force=(1e-5, 0.0, 0.0), init=(rho, u), solid=solid)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_sums_noalloc_matches_sums_on_two_calls_in_a_row(precision):
    big = _case((96, 64, 48), 11)
    small = _case((20, 12, 10), 12)
    for case, blocks in ((big, inputs.uniform_blocks(big["dims"], (2, 2, 2))), (small, None)):
        lat = gpu_lattice(case, blocks=blocks, precision=precision)
        prepare(lat, case)
        lat.step(5)
        m0, p0 = lat.sums()
        m1, p1 = lbm.lbm_sums_noalloc(lat.ctx)
        assert m1 == m0 and np.array_equal(p1, p0), (m0, m1, p0, p1)
        lat.close()


def test_sums_noalloc_with_many_workgroups():
    # small work items: the reduction runs the most workgroup partials
    case = _case((64, 64, 64), 13)
    lat = gpu_lattice(case, precision="f64")
    prepare(lat, case)
    lat.set_schedule(item_cells=64)
    lat.step(3)
    m0, p0 = lat.sums()
    m1, p1 = lbm.lbm_sums_noalloc(lat.ctx)
    assert m1 == m0 and np.array_equal(p1, p0)
    lat.close()
