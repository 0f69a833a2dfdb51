"""lbm_average_two_steps: the state replaced by the mean of the last two
post-collision states, against the oracle stepped to the same two states and
restarted from their mean (numpy mean of the oracle's own FP64 states), and
bit for bit across tilings, exchange modes and precisions; its error cases;
and what it is for: a start from a perturbed equilibrium keeps a period-two
velocity oscillation that the mean removes."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs
from tests.helpers import gpu_lattice, prepare, run_oracle
from tests.test_gpu_parity import TOL, cavity, channel, check_vs_oracle, duct

pytestmark = pytest.mark.gpu


def porous_channel(dims=(24, 12, 10)):
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 3), seed=6)
    return channel(dims=dims, solid=solid, force=(2e-5, 1e-6, 0.0), tau=0.7, seed=6)


CASES = {"cavity": (cavity, None), "porous_2x2x1": (porous_channel, (2, 2, 1)), "duct": (duct, (2, 1, 1))}


def oracle_averaged(case, before, after):
    """Oracle: `before` steps, the mean of the states after steps before - 1
    and before, then `after` more steps."""
    o = run_oracle(case, before - 1)
    fa = o.get_state()
    o.step(1)
    fb = o.get_state()
    o.set_state(0.5 * (fa + fb))
    o.step(after)
    return o


@pytest.mark.parametrize("name", list(CASES))
def test_mean_of_two_steps_matches_oracle_f64(name):
    make, split = CASES[name]
    case = make()
    blocks = inputs.uniform_blocks(case["dims"], split) if split else None
    lat = gpu_lattice(case, blocks=blocks)
    prepare(lat, case)
    lat.step(3)
    lat.average_two_steps()
    o = oracle_averaged(case, 3, 0)
    fg, fo = lat.get_state(), o.get_state()
    scale = max(np.abs(fo).max(), o.rho0 * np.abs(np.asarray(o.force)).max())
    assert np.abs(fg - fo).max() / scale <= TOL["f64"]
    lat.step(6)
    o.step(6)
    check_vs_oracle(lat, o, TOL["f64"])
    lat.close()


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_mean_of_two_steps_is_bitwise_across_tilings(precision):
    case = porous_channel()
    states = []
    for split, sched in [(None, None), ((2, 2, 1), None), ((2, 2, 1), dict(fused_exchange=0)),
                         ((3, 1, 2), dict(fused_exchange=1))]:
        blocks = inputs.uniform_blocks(case["dims"], split) if split else None
        lat = gpu_lattice(case, blocks=blocks, precision=precision)
        if sched:
            lat.set_schedule(**sched)
        prepare(lat, case)
        lat.step(4)
        lat.average_two_steps()
        lat.step(5)
        states.append(lat.get_state(as_fp64=False))
        lat.close()
    for s in states[1:]:
        assert np.array_equal(s, states[0])


def test_mean_of_two_steps_f32_tracks_oracle():
    case = porous_channel()
    lat = gpu_lattice(case, blocks=inputs.uniform_blocks(case["dims"], (2, 2, 1)), precision="f32")
    prepare(lat, case)
    lat.step(5)
    lat.average_two_steps()
    lat.step(10)
    check_vs_oracle(lat, oracle_averaged(case, 5, 10), TOL["f32"])
    lat.close()


def test_mean_of_two_steps_needs_a_step_and_gpu_blocks():
    from paper_1007_1388_amd.lbm import LBMError
    case = porous_channel()
    lat = gpu_lattice(case, blocks=inputs.uniform_blocks(case["dims"], (2, 2, 1)))
    with pytest.raises(LBMError):            # nothing stepped since creation
        lat.average_two_steps()
    prepare(lat, case)
    with pytest.raises(LBMError):            # nor since the equilibrium was set
        lat.average_two_steps()
    lat.step(2)
    lat.average_two_steps()
    with pytest.raises(LBMError):            # nor since the last mean
        lat.average_two_steps()
    with pytest.raises(LBMError):            # the previous step's state is gone
        lat.residual()
    lat.step(1)
    assert np.isfinite(lat.residual())
    f = lat.get_state()
    lat.set_state(f)
    with pytest.raises(LBMError):            # nor since a state was set
        lat.average_two_steps()
    lat.step(1)
    lat.set_host_blocks([1], threads=2)
    with pytest.raises(LBMError):            # host Blocks hold their own state
        lat.average_two_steps()
    lat.close()


def test_mean_removes_the_period_two_oscillation_of_a_perturbed_start():
    """A porous channel (seeded geometry of the warm-start data) started from
    an equilibrium of its converged velocity with 20 % smooth error: after
    6000 steps the one-step change of the velocity stays far above the
    two-step change (a period-two component that this geometry hardly
    damps); with one mean after the first step the one-step change is below
    twice the two-step change, as in a monotone approach, and the velocity is
    closer to the converged one."""
    from paper_1007_1388_amd import warmstart as ws
    dims = (32, 32, 64)
    solid, gx, _ = ws.sample(900000, dims)
    fluid = solid == 0

    def lattice():
        lat = ws.make_lattice(gx, solid, None, precision="f64", dims=dims)
        lat.set_schedule(graph_steps=0)
        return lat

    ref = lattice()
    ref.step(40000)
    rho_ref, u_ref = ref.macroscopic()
    ref.close()
    rng = np.random.default_rng(0)
    noise = rng.standard_normal(u_ref.shape)
    for ax in (1, 2, 3):
        for _ in range(4):
            noise = (noise + np.roll(noise, 1, ax) + np.roll(noise, -1, ax)) / 3
    noise /= noise.std()
    u0 = u_ref * (1 + 0.2 * noise)
    u0[:, ~fluid] = 0.0

    def run(average):
        lat = lattice()
        lat.set_equilibrium(rho_ref, u0)
        lat.step(1)
        if average:
            lat.average_two_steps()
        lat.step(6000)
        lat.residual_mark()
        lat.step(1)
        _, u1 = lat.macroscopic()
        r1 = lat.residual()
        lat.step(1)
        r2, _ = lat.residual_since_mark()
        err = np.linalg.norm((u1 - u_ref)[:, fluid]) / np.linalg.norm(u_ref[:, fluid])
        lat.close()
        return r1, r2, err

    r1, r2, e = run(False)
    q1, q2, f = run(True)
    print("one-step / two-step change and error: plain %.2e %.2e %.2e, mean %.2e %.2e %.2e" % (r1, r2, e, q1, q2, f))
    assert r1 > 10 * r2
    assert q1 < 2 * q2
    assert f < 0.1 * e
