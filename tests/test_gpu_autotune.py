"""The schedule autotuner (per-context kernel and schedule selection by
measurement, after the paper's per-Block kernel selection by metadata,
Sec. 4.1): it leaves the simulation unchanged, its choice reproduces the
default schedule's results bit for bit, a cache hit runs no trials, and a
cached line the context refuses is skipped."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs
from tests.helpers import gpu_lattice, prepare

pytestmark = pytest.mark.gpu


def porous_case():
    dims = (48, 40, 36)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(2, 4), seed=5)
    rho, u = inputs.perturbed_fields(dims, seed=5, drho=1e-3, du=1e-2)
    u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(False, False, True), tau=0.7, force=(1e-5, 0.0, 0.0), init=(rho, u), solid=solid)


def duct_case():
    dims = (40, 12, 10)
    rho, u = inputs.perturbed_fields(dims, seed=6, drho=1e-3, du=1e-2)
    return dict(dims=dims, walls=(True, False, True), tau=0.7, force=(0.0, 2e-6, 0.0), init=(rho, u),
                open_x={"-x": ("velocity", (0.02, 0.0, 0.0)), "+x": ("pressure", 1.0)})


def lattice(case, blocks=None, precision="f32"):
    lat = gpu_lattice(case, blocks=blocks, precision=precision)
    prepare(lat, case)
    return lat


def cache_lines(path):
    with open(path) as fh:
        return [l for l in fh.read().splitlines() if l.strip()]


@pytest.mark.parametrize("name", ["porous", "duct"])
def test_autotune_keeps_state_and_choice_reproduces_default(tmp_path, name):
    case = porous_case() if name == "porous" else duct_case()
    blocks = inputs.uniform_blocks(case["dims"], (2, 2, 3)) if name == "porous" else \
        inputs.uniform_blocks(case["dims"], (4, 1, 1))
    cache = str(tmp_path / "tune.txt")
    ref = lattice(case, blocks)
    ref.step(7)
    tuned = lattice(case, blocks)
    tuned.step(7)
    f0 = tuned.get_state(as_fp64=False)
    steps0 = tuned.info()["steps"]
    chosen = tuned.autotune(cache, trial_steps=2)
    # the simulation is unchanged (both grids restored, step count kept)
    assert np.array_equal(tuned.get_state(as_fp64=False), f0)
    assert tuned.info()["steps"] == steps0
    assert tuned.schedule == chosen
    # the chosen schedule continues the run exactly as the default does
    tuned.step(9)
    ref.step(9)
    assert np.array_equal(tuned.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    r1, r2 = tuned.macroscopic(), ref.macroscopic()
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    assert len(cache_lines(cache)) == 1
    # a second context of the same problem takes the cached choice without
    # trials (a tuning run would append a line)
    again = lattice(case, blocks)
    c2 = again.autotune(cache, trial_steps=2)
    assert c2 == chosen
    assert len(cache_lines(cache)) == 1
    again.step(16)
    assert np.array_equal(again.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    for lat in (ref, tuned, again):
        lat.close()


def test_autotune_skips_refused_and_malformed_cache_lines(tmp_path):
    # open faces allow one cell per lane only: a cached line asking for two
    # (and a malformed one) must not stop the tuner
    case = duct_case()
    cache = str(tmp_path / "tune.txt")
    a = lattice(case)
    a.autotune(cache, trial_steps=2)
    key = cache_lines(cache)[0].split()[0]
    with open(cache, "w") as fh:
        fh.write("%s 0 512 256 0 10 1 2\n" % key)        # two cells per lane: refused here
        fh.write("%s 0 512 100 0 10 1 0\n" % key)        # workgroup of 100 threads: invalid
        fh.write("%s garbage\n" % key)
    b = lattice(case)
    b.step(3)
    f0 = b.get_state(as_fp64=False)
    chosen = b.autotune(cache, trial_steps=2)
    assert chosen["cells_per_lane"] != 2 and chosen["wg_size"] in (64, 128, 256)
    assert len(cache_lines(cache)) == 4       # tuned again and appended
    assert np.array_equal(b.get_state(as_fp64=False), f0)
    a.step(3)
    b.step(5)
    a.step(5)
    assert np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))
    a.close()
    b.close()
