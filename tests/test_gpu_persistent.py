"""The persistent multi-step sweep (lbm_step_persistent: one cooperative
launch per run of steps, the block list walked step after step with the
ghost exchange fused into the sweep and a grid-wide barrier between steps)
against lbm_step, bit for bit, through the C ABI."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs, lbm
from tests.helpers import gpu_lattice, prepare

pytestmark = pytest.mark.gpu


def porous(dims=(48, 40, 36), seed=21):
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(2, 4), seed=seed)
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=1e-2)
    u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(False, False, True), tau=0.7, force=(1e-5, 0.0, 0.0), init=(rho, u), solid=solid)


def cavity(dims=(20, 18, 17)):
    return dict(dims=dims, walls=(True, True, True), wall_u={"+z": (0.05, 0.0, 0.0)}, tau=0.6)


def periodic(dims=(33, 17, 12), seed=4):
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=2e-2)
    return dict(dims=dims, walls=(False, False, False), tau=0.7, force=(3e-5, -1e-5, 2e-5), init=(rho, u))


def _pair(case, blocks, precision):
    a = gpu_lattice(case, blocks=blocks, precision=precision)
    b = gpu_lattice(case, blocks=blocks, precision=precision)
    prepare(a, case)
    prepare(b, case)
    return a, b


@pytest.mark.parametrize("name,precision", [("porous", "f32"), ("porous", "f64"), ("cavity", "f64"),
                                            ("periodic", "f32"), ("porous", "f16s"), ("cavity", "bf16s")])
@pytest.mark.parametrize("split", [(1, 1, 1), (2, 2, 3)])
def test_persistent_steps_equal_lbm_step(name, precision, split):
    case = {"porous": porous, "cavity": cavity, "periodic": periodic}[name]()
    blocks = inputs.uniform_blocks(case["dims"], split)
    a, b = _pair(case, blocks, precision)
    a.step(23)
    b.step_persistent(23, steps_per_launch=10)     # 10 + 10 + 3 steps
    assert a.info()["steps"] == b.info()["steps"] == 23
    assert np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))
    ra, ua = a.macroscopic()
    rb, ub = b.macroscopic()
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    # and the two continue alike, mixing both kinds of stepping
    a.step(4)
    b.step_persistent(1, steps_per_launch=1)
    b.step(3)
    assert np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))
    (ma, qa), (mb, qb) = a.sums(), b.sums()
    assert ma == mb and np.array_equal(qa, qb)
    a.close()
    b.close()


def test_persistent_uneven_blocks_many():
    dims, blocks = inputs.uneven_blocks_grid((3, 3, 2), (16, 24, 32), seed=2)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(2, 4), seed=3)
    case = dict(dims=dims, walls=(False, False, True), tau=0.7, force=(1e-5, 0.0, 0.0), solid=solid)
    a, b = _pair(case, blocks, "f32")
    a.step(30)
    b.step_persistent(30, steps_per_launch=30)
    assert np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))
    a.close()
    b.close()


def test_persistent_refusals():
    duct = dict(dims=(20, 6, 5), walls=(True, False, True), tau=0.7,
                open_x={"-x": ("velocity", (0.02, 0.0, 0.0)), "+x": ("pressure", 1.0)})
    lat = gpu_lattice(duct, precision="f64")
    with pytest.raises(lbm.LBMError):
        lat.step_persistent(2)
    lat.close()
    lat = gpu_lattice(cavity(), precision="f64")
    with pytest.raises(lbm.LBMError):
        lat.step_persistent(2, steps_per_launch=0)
    lat.set_host_blocks([0])
    with pytest.raises(lbm.LBMError):
        lat.step_persistent(2)
    lat.close()
