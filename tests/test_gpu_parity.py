"""GPU parity: the HIP library against the CPU FP64 oracle, element by element,
on seeded inputs, through the C ABI (ctypes binding).

Bars: FP64 storage and arithmetic 1e-12 (normwise relative, infinity norm);
FP32 storage 1e-5; partition, schedule and exchange variants bit-exact
against each other (same per-cell arithmetic, only data movement differs).
"""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs
from tests.helpers import field_errors, gpu_lattice, prepare, rel_inf, run_oracle

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def cavity(dims=(20, 18, 17), lid=(0.05, 0.0, 0.0), tau=0.6):
    return dict(dims=dims, walls=(True, True, True), wall_u={"+z": lid}, tau=tau)


def channel(dims=(24, 10, 13), force=(1e-5, 2e-6, 0.0), tau=0.8, seed=0, solid=None):
    nx, ny, nz = dims
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=1e-2)
    if solid is not None:
        u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(False, False, True), tau=tau, force=force, init=(rho, u), solid=solid)


def periodic_box(dims=(11, 9, 7), seed=1, force=(3e-5, -1e-5, 2e-5), tau=0.7):
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=2e-2)
    return dict(dims=dims, walls=(False, False, False), tau=tau, force=force, init=(rho, u))


def duct(dims=(29, 10, 9), tau=0.7, force=(0.0, 3e-6, 0.0), seed=3, obstacles=True):
    """Open x faces: velocity inlet with a tangential part at -x, pressure
    outlet at +x, walls in z (the -z wall moving), periodic y, spheres off the
    open faces, a perturbed warm start."""
    solid = None
    if obstacles:
        solid = inputs.porous_spheres(dims, target_fraction=0.08, radius=(2, 3), seed=seed)
        solid[:, :, 0] = 0
        solid[:, :, -1] = 0
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=1e-2)
    if solid is not None:
        u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(True, False, True), wall_u={"-z": (0.01, 0.0, 0.0)}, tau=tau, force=force,
                open_x={"-x": ("velocity", (0.03, 0.005, 0.0)), "+x": ("pressure", 1.001)},
                init=(rho, u), solid=solid)


def run_gpu(case, steps, blocks=None, precision="f64", fp64_math=False, schedule=None):
    lat = gpu_lattice(case, blocks=blocks, precision=precision, fp64_math=fp64_math)
    if schedule:
        lat.set_schedule(**schedule)
    prepare(lat, case)
    lat.step(steps)
    return lat


def check_vs_oracle(lat, o, tol):
    rho_g, u_g = lat.macroscopic()
    rho_o, u_o = o.macroscopic()
    err = field_errors(rho_g, u_g, rho_o, u_o)
    assert err["u_inf"] <= tol and err["drho_inf"] <= tol, err
    # Populations: a post-collision value sums terms as large as the force
    # source 3 w rho0 |g| even when the result is much smaller, so rounding is
    # measured against max(|f|, rho0 |g|).
    fg, fo = lat.get_state(), o.get_state()
    scale = max(np.abs(fo).max(), o.rho0 * np.abs(np.asarray(o.force)).max())
    fs = np.abs(fg - fo).max() / scale
    assert fs <= tol, fs
    return err


# ------------------------------------------------------------ vs oracle ----

@pytest.mark.parametrize("steps", [0, 1, 60])
def test_cavity_f64_matches_oracle(steps):
    case = cavity()
    lat = run_gpu(case, steps)
    o = run_oracle(case, steps)
    if steps == 0:
        rho, u = lat.macroscopic()
        assert np.all(rho == 1.0) and np.all(u == 0.0)
        return
    check_vs_oracle(lat, o, TOL["f64"])


def test_channel_with_force_and_warm_start_f64():
    case = channel()
    lat = run_gpu(case, 0)
    o = run_oracle(case, 0)
    check_vs_oracle(lat, o, TOL["f64"])  # warm start itself
    lat.step(50)
    o.step(50)
    check_vs_oracle(lat, o, TOL["f64"])


def test_periodic_box_all_axes_f64():
    case = periodic_box()
    lat = run_gpu(case, 40)
    o = run_oracle(case, 40)
    check_vs_oracle(lat, o, TOL["f64"])


@pytest.mark.parametrize("fp64_math", [False, True])
def test_channel_f32_storage(fp64_math):
    case = channel(force=(2e-5, 0, 0))
    lat = run_gpu(case, 60, precision="f32", fp64_math=fp64_math)
    o = run_oracle(case, 60)
    check_vs_oracle(lat, o, TOL["f32"])


@pytest.mark.parametrize("precision,tol", [("f16s", 1e-2), ("bf16s", 5e-2)])
@pytest.mark.parametrize("dims", [(24, 12, 10), (13, 12, 10)])
def test_shifted_half_storage_tracks_oracle(precision, tol, dims):
    # Storage rounding of 2^-11 (FP16) / 2^-8 (BF16) of |f~| ~ w 3|u| per step
    # accumulates to ~1e-3 / ~1e-2 relative velocity error over 100 steps.
    case = cavity(dims=dims, lid=(0.05, 0.0, 0.0))
    case["solid"] = inputs.porous_spheres(dims, target_fraction=0.05, radius=(1, 2), seed=9,
                                          periodic=(False, False, False))
    lat = run_gpu(case, 100, precision=precision)
    o = run_oracle(case, 100)
    err = field_errors(*lat.macroscopic(), *o.macroscopic())
    assert err["u_inf"] < tol, err


@pytest.mark.parametrize("precision", ["f16s", "bf16s"])
def test_force_free_half_storage_bitwise_across_tilings(precision):
    """Without a body force the 16-bit sweeps leave the (zero) force terms
    out of the collision (the test above checks them against the oracle):
    tilings, exchange modes and two cells per lane give the one-Block result
    bit for bit."""
    dims = (24, 12, 10)
    case = cavity(dims=dims, lid=(0.05, 0.0, 0.0))
    case["solid"] = inputs.porous_spheres(dims, target_fraction=0.05, radius=(1, 2), seed=9,
                                          periodic=(False, False, False))
    ref = run_gpu(case, 30, precision=precision).get_state(as_fp64=False)
    for split, sched in [((2, 2, 1), None), ((3, 1, 2), dict(fused_exchange=1)), (None, dict(cells_per_lane=2)),
                         ((2, 2, 1), dict(cells_per_lane=2, fused_exchange=0))]:
        blocks = inputs.uniform_blocks(dims, split) if split else None
        lat = run_gpu(case, 30, blocks=blocks, precision=precision, schedule=sched)
        assert np.array_equal(lat.get_state(as_fp64=False), ref)
        lat.close()


def test_porous_multiblock_f64_matches_oracle():
    dims = (40, 24, 20)
    solid = inputs.porous_spheres(dims, target_fraction=0.15, radius=(2, 4), seed=5)
    case = channel(dims=dims, solid=solid, force=(1e-5, 0, 0), tau=0.7)
    blocks = inputs.random_tiling(dims, max_blocks_per_axis=3, seed=11, min_edge=1)
    lat = run_gpu(case, 40, blocks=blocks)
    o = run_oracle(case, 40)
    check_vs_oracle(lat, o, TOL["f64"])
    rho_g, _ = lat.macroscopic()
    assert np.all(rho_g[solid == 1] == 1.0)


def test_lid_on_every_face_f64():
    # moving walls on several faces at once: exercises the face-precedence rule
    case = dict(dims=(9, 10, 11), walls=(True, True, True), tau=0.65,
                wall_u={"-x": (0, 0.02, 0.01), "+y": (0.03, 0, -0.01), "+z": (0.05, 0.02, 0),
                        "-z": (-0.01, 0, 0)})
    lat = run_gpu(case, 30, blocks=inputs.uniform_blocks(case["dims"], (2, 2, 3)))
    o = run_oracle(case, 30)
    check_vs_oracle(lat, o, TOL["f64"])


# ------------------------------------------------- partition invariance ---

TILINGS = {
    "uniform222": lambda d: inputs.uniform_blocks(d, (2, 2, 2)),
    "slabs": lambda d: inputs.uniform_blocks(d, (1, 1, 4)),
    "random": lambda d: inputs.random_tiling(d, max_blocks_per_axis=4, seed=3, min_edge=1),
    "thin": lambda d: inputs.uniform_blocks(d, (d[0], 1, 1)),
    "vec": lambda d: inputs.uniform_blocks(d, (max(1, d[0] // 8), 2, 3)),
}


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("tiling", sorted(TILINGS))
@pytest.mark.parametrize("dims", [(13, 12, 10), (24, 12, 10)])
def test_partition_invariance_bitwise(precision, tiling, dims):
    # With x = 24 the single-Block reference of the 16-bit formats runs two
    # cells per lane; the tilings run one: both must round alike.
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 3), seed=2)
    case = channel(dims=dims, solid=solid, force=(1e-5, 0, 3e-6), tau=0.75, seed=4)
    two = precision in ("f16s", "bf16s") and dims[0] % 2 == 0
    ref = run_gpu(case, 25, precision=precision, schedule=dict(cells_per_lane=2) if two else None)
    lat = run_gpu(case, 25, blocks=TILINGS[tiling](dims), precision=precision)
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_self_wrapping_block_matches_tiling(precision):
    """A Block that is its own neighbour along x and y (x extent > 64) reads
    across those axes from itself instead of its ghost layers: bitwise equal
    to tilings that exchange, with obstacles straddling the periodic faces and
    walls in z."""
    dims = (80, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.12, radius=(1, 3), seed=5)
    case = channel(dims=dims, solid=solid, force=(1e-5, 3e-6, 0.0), tau=0.75, seed=2)
    ref = run_gpu(case, 20, blocks=inputs.uniform_blocks(dims, (2, 2, 1)), precision=precision)
    for blocks in (None, inputs.uniform_blocks(dims, (1, 2, 1)), inputs.uniform_blocks(dims, (2, 1, 1))):
        lat = run_gpu(case, 20, blocks=blocks, precision=precision)
        assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))
        lat.close()


@pytest.mark.parametrize("precision,f64m", [("f32", False), ("f64", False), ("f32", True), ("f16s", False)])
def test_rows_of_64_cells_bitwise_across_tilings(precision, f64m):
    """One Block with rows of exactly 64 cells wraps onto itself in y when the
    sweep runs one cell per lane (FP32 mixed, FP64), and takes the exchange
    where two cells per lane are possible (FP32 with FP64 math, 16-bit): every
    case equals a tiling that exchanges, bit for bit, with two cells per lane
    as well where allowed."""
    dims = (64, 12, 9)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 3), seed=9)
    case = channel(dims=dims, solid=solid, force=(1e-5, 3e-6, 0.0), tau=0.75, seed=4)
    ref = run_gpu(case, 17, blocks=inputs.uniform_blocks(dims, (2, 2, 1)), precision=precision, fp64_math=f64m)
    scheds = [None] + ([dict(cells_per_lane=2)] if precision == "f16s" or f64m else [])
    for sched in scheds:
        lat = run_gpu(case, 17, precision=precision, fp64_math=f64m, schedule=sched)
        assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))
        lat.close()


def test_self_wrapping_periodic_box_matches_oracle():
    """Fully periodic box as one Block (wraps on all three axes) against the
    oracle, and against a two-Block tiling bit for bit."""
    case = periodic_box(dims=(70, 9, 7))
    lat = run_gpu(case, 30)
    o = run_oracle(case, 30)
    check_vs_oracle(lat, o, TOL["f64"])
    two = run_gpu(case, 30, blocks=inputs.uniform_blocks((70, 9, 7), (2, 1, 1)))
    assert np.array_equal(lat.get_state(as_fp64=False), two.get_state(as_fp64=False))


# ------------------------------------------------- open faces (NEXT) -------

@pytest.mark.parametrize("steps", [0, 1, 150])
def test_open_faces_f64_match_oracle(steps):
    """Velocity inlet and pressure outlet (non-equilibrium extrapolation) with
    a moving wall, a body force, obstacles and a warm start, against the
    oracle; steps = 1 checks the boundary nodes filled from a loaded state."""
    case = duct()
    lat = run_gpu(case, steps)
    o = run_oracle(case, steps)
    check_vs_oracle(lat, o, TOL["f64"])


@pytest.mark.parametrize("fp64_math", [False, True])
def test_open_faces_f32_storage(fp64_math):
    case = duct()
    lat = run_gpu(case, 150, precision="f32", fp64_math=fp64_math)
    o = run_oracle(case, 150)
    rho_g, u_g = lat.macroscopic()
    rho_o, u_o = o.macroscopic()
    err = field_errors(rho_g, u_g, rho_o, u_o)
    assert err["u_inf"] <= TOL["f32"] and err["drho_inf"] <= TOL["f32"], err


@pytest.mark.parametrize("variant", range(5))
def test_open_faces_tilings_and_schedules_bitwise(variant):
    """Blocks cut along x, every exchange mode and graph capture give the
    one-Block result bit for bit; a row longer than a wave (y wraps on the
    Block itself) with the open faces."""
    dims = (70, 6, 5) if variant == 4 else (29, 10, 9)
    case = duct(dims=dims, obstacles=variant != 4)
    blocks = [None, inputs.uniform_blocks(dims, (3, 1, 1)),
              [((0, 0, 0), (5, dims[1], dims[2])), ((5, 0, 0), (23, dims[1], dims[2])),
               ((23, 0, 0), (dims[0], dims[1], dims[2]))],
              inputs.uniform_blocks(dims, (2, 1, 1)), None][variant]
    sched = [dict(fused_exchange=1), dict(fused_exchange=0), dict(fused_exchange=2),
             dict(fused_exchange=1, graph_steps=4), dict(graph_steps=5)][variant]
    ref = run_gpu(case, 37, precision="f32")
    lat = run_gpu(case, 37, blocks=blocks, precision="f32", schedule=sched)
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    if variant == 4:
        o = run_oracle(case, 37)
        f64 = run_gpu(case, 37)
        check_vs_oracle(f64, o, TOL["f64"])


@pytest.mark.parametrize("variant", range(6))
def test_open_faces_on_blocks_cut_across_y_and_z(variant):
    """Open x faces on tilings cut across y and z: a boundary node feeds the
    face cells of the Blocks next to it through their x-ghost planes' ghost
    rows.  Bit for bit against the one-Block run (every exchange mode, graph
    capture, uneven cuts, a periodic z axis), and FP64 against the oracle."""
    dims = (29, 10, 9)
    case = duct(dims=dims)
    if variant == 5:
        # periodic z and y: the boundary nodes' periodic images sit in ghost
        # rows of the Blocks at the far side
        case = duct(dims=dims)
        case["walls"] = (True, False, False)
        case.pop("wall_u")
    blocks = [inputs.uniform_blocks(dims, (1, 2, 1)), inputs.uniform_blocks(dims, (1, 1, 3)),
              inputs.uniform_blocks(dims, (3, 2, 3)),
              [((x0, y0, z0), (x1, y1, z1)) for (x0, x1) in ((0, 11), (11, 29)) for (y0, y1) in ((0, 3), (3, 10))
               for (z0, z1) in ((0, 4), (4, 9))],
              inputs.uniform_blocks(dims, (2, 2, 2)), inputs.uniform_blocks(dims, (1, 2, 3))][variant]
    sched = [dict(fused_exchange=0), dict(fused_exchange=1), dict(fused_exchange=2),
             dict(fused_exchange=2, graph_steps=4), dict(fused_exchange=1, graph_steps=5), dict()][variant]
    ref = run_gpu(case, 41, precision="f32")
    lat = run_gpu(case, 41, blocks=blocks, precision="f32", schedule=sched)
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    f64 = run_gpu(case, 41, blocks=blocks, schedule=sched)
    o = run_oracle(case, 41)
    check_vs_oracle(f64, o, TOL["f64"])


def test_open_faces_cut_tiling_checkpoint_restart():
    """A state loaded into a cut tiling with open faces (set_state fills the
    boundary nodes from the face cells' stored populations, whose moments
    equal those of their last collision up to rounding) continues as the
    uninterrupted run, to FP64 rounding."""
    dims = (29, 10, 9)
    case = duct(dims=dims)
    blocks = inputs.uniform_blocks(dims, (2, 2, 3))
    a = run_gpu(case, 30, blocks=blocks)
    f = a.get_state(as_fp64=True)
    b = gpu_lattice(case, blocks=inputs.uniform_blocks(dims, (1, 3, 1)))
    prepare(b, case)
    b.set_state(f, as_fp64=True)
    a.step(20)
    b.step(20)
    fa, fb = a.get_state(as_fp64=True), b.get_state(as_fp64=True)
    assert np.abs(fa - fb).max() <= 1e-12 * np.abs(fa).max()


def test_open_faces_reject_solid_on_the_face():
    case = duct(obstacles=False)
    lat = gpu_lattice(case)
    solid = np.zeros(lat.shape, np.uint8)
    solid[3, 4, 0] = 1
    from paper_1007_1388_amd import lbm
    with pytest.raises(lbm.LBMError):
        lat.set_geometry(solid)
    solid[3, 4, 0] = 0
    solid[3, 4, 5] = 1
    lat.set_geometry(solid)


SCHEDULES = [
    dict(fused_exchange=0),
    dict(fused_exchange=2),
    dict(fused_exchange=2, wg_size=64, item_cells=96, nontemporal=0),
    dict(fused_exchange=1, persistent=2, wg_size=128, item_cells=64),
    dict(fused_exchange=0, persistent=1, wg_size=64, item_cells=4096, nontemporal=0),
    dict(graph_steps=4),
    dict(graph_steps=3, fused_exchange=0),
]


@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_schedules_are_bitwise_identical(sched):
    dims = (30, 17, 12)
    case = cavity(dims=dims)
    blocks = inputs.random_tiling(dims, max_blocks_per_axis=3, seed=7, min_edge=2)
    ref = run_gpu(case, 21, blocks=blocks, precision="f32")
    lat = run_gpu(case, 21, blocks=blocks, precision="f32", schedule=SCHEDULES[sched])
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))


def test_graph_steps_split_across_calls():
    case = periodic_box()
    ref = run_gpu(case, 0)
    ref.step(7)
    lat = run_gpu(case, 0, schedule=dict(graph_steps=3))
    for n in (1, 2, 0, 4):
        lat.step(n)
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))


@pytest.mark.parametrize("precision,f64m", [("f16s", False), ("bf16s", False), ("f32", True)])
def test_cells_per_lane_bitwise(precision, f64m):
    """One or two cells per lane: identical rounding, identical states."""
    dims = (24, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 2), seed=9)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7)
    blocks = inputs.uniform_blocks(dims, (2, 2, 1))
    out = []
    for cpl in (1, 2, 0):
        lat = run_gpu(case, 0, blocks=blocks, precision=precision, fp64_math=f64m,
                      schedule=dict(cells_per_lane=cpl, fused_exchange=cpl % 2))
        lat.step(15)
        out.append(lat.get_state(as_fp64=False))
        lat.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_cells_per_lane_two_rejected_where_unsupported():
    from paper_1007_1388_amd.lbm import LBMError
    lat = gpu_lattice(channel(dims=(23, 8, 6)), precision="f16s")  # odd x extent
    with pytest.raises(LBMError):
        lat.set_schedule(cells_per_lane=2)
    lat.close()
    lat = gpu_lattice(channel(dims=(24, 8, 6)), precision="f32")  # mixed FP32 math: one cell per lane
    with pytest.raises(LBMError):
        lat.set_schedule(cells_per_lane=2)
    lat.set_schedule(cells_per_lane=1)
    lat.close()


@pytest.mark.parametrize("fused", [0, 1, 2])
def test_step_timed_matches_step(fused):
    """The per-launch timed stepping advances the state exactly as lbm_step."""
    dims = (16, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 2), seed=3)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7)
    blocks = inputs.uniform_blocks(dims, (2, 2, 1))
    ref = run_gpu(case, 0, blocks=blocks, schedule=dict(fused_exchange=fused))
    ref.step(9)
    lat = run_gpu(case, 0, blocks=blocks, schedule=dict(fused_exchange=fused))
    lat.step(2)
    ts, te = lat.step_timed(5)
    lat.step(2)
    assert ts > 0 and (te == 0 if fused == 1 else te > 0)
    assert lat.info()["steps"] == 9
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_row_padding_is_layout_only(precision):
    """Extra x-row padding changes addresses only: bitwise equal states."""
    dims = (24, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 2), seed=6)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7)
    blocks = inputs.uniform_blocks(dims, (2, 2, 1))
    states = []
    for pad in (-1, 1, 3):
        lat = gpu_lattice(case, blocks=blocks, precision=precision, row_pad=pad)
        prepare(lat, case)
        lat.step(12)
        states.append(lat.get_state(as_fp64=False))
        lat.close()
    assert np.array_equal(states[0], states[1]) and np.array_equal(states[0], states[2])


@pytest.mark.parametrize("precision,dims,split", [("f32", (96, 20, 14), (2, 2, 1)), ("f64", (48, 20, 14), (2, 2, 1)),
                                                   ("f32", (80, 16, 9), (1, 2, 1))])
def test_packed_rows_are_layout_only(precision, dims, split):
    """Rows of an odd number of half lines (FP32 rows of 48 or 80 cells) are
    packed two to three lines by default (row_pad 0), and rows stored back to
    back (packed, or FP32 96 and FP64 48 cells) run as flat runs of 64 cells
    across row ends: bitwise equal to rows rounded to whole lines (row_pad -1)
    and to padded rows (row segments), and FP64 against the oracle; obstacles,
    walls, a body force and a warm start, Blocks of packed and unpacked rows
    side by side."""
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 3), seed=8)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7, seed=8)
    blocks = inputs.uniform_blocks(dims, split)
    if split == (1, 2, 1):
        blocks = [((0, 0, 0), (48, 8, 9)), ((48, 0, 0), (80, 8, 9)), ((0, 8, 0), (48, 16, 9)), ((48, 8, 0), (80, 16, 9))]
    states = []
    for pad in (0, -1, 2):
        lat = gpu_lattice(case, blocks=blocks, precision=precision, row_pad=pad)
        prepare(lat, case)
        lat.step(19)
        states.append(lat.get_state(as_fp64=False))
        if pad == 0 and precision == "f64":
            check_vs_oracle(lat, run_oracle(case, 19), TOL["f64"])
        lat.close()
    assert np.array_equal(states[0], states[1]) and np.array_equal(states[0], states[2])


def _pad_case(kind):
    dims = (104, 12, 10)
    if kind == "open":
        return duct(dims=dims, seed=4)
    solid = inputs.porous_spheres(dims, target_fraction=0.08, radius=(2, 3), seed=4)
    rho, u = inputs.perturbed_fields(dims, seed=4, drho=1e-3, du=1e-2)
    u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(True, False, True), wall_u={"+x": (0.0, 0.01, 0.0), "-z": (0.01, 0.0, 0.0)},
                tau=0.7, force=(2e-6, 1e-6, 0.0), init=(rho, u), solid=solid)


# a Block of 100 cells along x next to one of 4: padding lanes of the first
# (x = 100 .. 103 in FP64, .. 111 in FP32, .. 127 in F16S) lie at global x up
# to and past the far x face of the 104-cell domain
PAD_SPLIT = [((0, 0, 0), (100, 6, 10)), ((100, 0, 0), (104, 6, 10)), ((0, 6, 0), (100, 12, 10)),
             ((100, 6, 0), (104, 12, 10))]


@pytest.mark.parametrize("kind", ["walls", "open"])
def test_padding_lanes_write_only_padding(kind):
    """The lanes past a row's end that complete its last 64-byte sector
    write only row padding, and the wall, open-face and exchange rules never
    fire for them although their global x reaches the far x face (x walls
    with a moving +x wall, or a velocity inlet and pressure outlet):
    obstacles (padding lanes take the solid-cell path) and a body force.
    FP64 against the oracle; FP32 and F16S bit for bit across tilings, every
    exchange mode, row paddings and (closed faces) the persistent sweep."""
    case = _pad_case(kind)
    check_vs_oracle(run_gpu(case, 25, blocks=PAD_SPLIT), run_oracle(case, 25), TOL["f64"])
    for precision in ("f32", "f16s"):
        runs = [(None, 0, {}), (PAD_SPLIT, 0, dict(fused_exchange=0)), (PAD_SPLIT, 0, dict(fused_exchange=1)),
                (PAD_SPLIT, 0, dict(fused_exchange=2, graph_steps=5)), (PAD_SPLIT, -1, {}), (PAD_SPLIT, 2, {})]
        if kind == "walls":
            runs.append((PAD_SPLIT, 0, "persistent"))
        states = []
        for blocks, row_pad, sched in runs:
            lat = gpu_lattice(case, blocks=blocks, precision=precision, row_pad=row_pad)
            prepare(lat, case)
            if sched == "persistent":
                lat.step_persistent(25, steps_per_launch=10)
            else:
                lat.set_schedule(**sched)
                lat.step(25)
            states.append(lat.get_state(as_fp64=False))
            lat.close()
        for st in states[1:]:
            assert np.array_equal(st, states[0])


def test_block_size_limits():
    """A Block one of whose FP64 population arrays would reach 4 GiB is
    refused before anything is allocated; a 512^3 FP64 Block (1.1 GB per
    array) runs, and refuses obstacles, whose addressing spans six arrays."""
    import torch
    from paper_1007_1388_amd import lbm
    with pytest.raises(lbm.LBMError):
        lbm.Lattice((1100, 1100, 1100), precision="f64", tau=0.7)
    lat = lbm.Lattice((512, 512, 512), walls=(False, False, True), precision="f64", tau=0.7,
                      force=(1e-6, 0.0, 0.0))
    solid = np.zeros(lat.shape, np.uint8)
    solid[5, 6, 7] = 1
    with pytest.raises(lbm.LBMError):
        lat.set_geometry(solid)
    lat.step(3)
    mass, mom = lat.sums()
    assert abs(mass - 512 ** 3) < 1e-6 * 512 ** 3 and mom[0] > 0
    lat.close()
    del lat
    torch.cuda.empty_cache()


# ------------------------------------------------------ sums, residual ----

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_residual_since_mark(precision):
    """One step after the mark it is the one-step residual, bit for bit; two
    steps after, it matches the oracle's ||u^n - u^(n-2)|| / ||u^n||."""
    dims = (16, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.15, radius=(1, 2), seed=4)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7)
    lat = run_gpu(case, 0, blocks=inputs.uniform_blocks(dims, (2, 1, 2)), precision=precision)
    from paper_1007_1388_amd.lbm import LBMError
    with pytest.raises(LBMError):
        lat.residual_since_mark()
    lat.step(6)
    lat.residual_mark()
    lat.step(1)
    r1, n1 = lat.residual_since_mark()
    assert n1 == 1 and r1 == lat.residual()
    o = run_oracle(case, 0)
    o.step(5)
    _, u_a = o.macroscopic()
    o.step(2)
    _, u_b = o.macroscopic()
    fl = solid == 0
    r_ref = np.linalg.norm((u_b - u_a)[:, fl]) / np.linalg.norm(u_b[:, fl])
    lat2 = run_gpu(case, 0, blocks=inputs.uniform_blocks(dims, (2, 1, 2)), precision=precision)
    lat2.step(5)
    lat2.residual_mark()
    lat2.step(2)
    r2, n2 = lat2.residual_since_mark()
    assert n2 == 2
    assert abs(r2 - r_ref) <= (1e-10 if precision == "f64" else 1e-4) * r_ref, (r2, r_ref)
    lat2.set_geometry(solid)  # re-initialisation discards the snapshot
    with pytest.raises(LBMError):
        lat2.residual_since_mark()


def test_sums_and_residual_match_oracle():
    dims = (16, 12, 10)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 2), seed=8)
    case = channel(dims=dims, solid=solid, force=(2e-5, 0, 0), tau=0.7)
    lat = run_gpu(case, 0, blocks=inputs.uniform_blocks(dims, (2, 2, 1)))
    o = run_oracle(case, 0)
    from paper_1007_1388_amd.lbm import LBMError
    with pytest.raises(LBMError):
        lat.residual()
    for n in (2, 5):
        lat.step(n)
        o.step(n)
        mg, pg = lat.sums()
        mo, po = o.sums()
        assert abs(mg - mo) <= 1e-12 * abs(mo)
        assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
        rg, ro = lat.residual(), o.residual()
        assert abs(rg - ro) <= 1e-11 * ro


def test_periodic_mass_and_force_momentum_on_gpu():
    case = periodic_box(force=(1e-5, 2e-5, -1e-5))
    lat = run_gpu(case, 1, blocks=inputs.uniform_blocks(case["dims"], (2, 1, 2)))
    n = np.prod(case["dims"])
    m0, p0 = lat.sums()
    for _ in range(5):
        lat.step(1)
        m, p = lat.sums()
        assert abs(m - m0) <= 1e-13 * n
        assert np.abs(p - p0 - n * np.array(case["force"])).max() <= 1e-14 * n
        p0 = p


# --------------------------------------------------------- checkpoint -----

@pytest.mark.parametrize("precision", ["f64", "f32", "bf16s"])
def test_checkpoint_resume_is_bitwise(precision):
    dims = (14, 10, 9)
    case = channel(dims=dims)
    blocks = inputs.uniform_blocks(dims, (2, 1, 3))
    ref = run_gpu(case, 20, blocks=blocks, precision=precision)
    a = run_gpu(case, 10, blocks=blocks, precision=precision)
    saved = a.get_state(as_fp64=False)
    b = run_gpu(case, 0, blocks=inputs.uniform_blocks(dims, (1, 2, 1)), precision=precision)
    b.set_state(saved, as_fp64=False)
    b.step(10)
    assert np.array_equal(b.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    r1, u1 = b.macroscopic()
    r2, u2 = ref.macroscopic()
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2)


def test_macroscopic_device_output_matches_host():
    case = channel()
    lat = run_gpu(case, 5)
    rho_h, u_h = lat.macroscopic()
    rho_d, u_d = lat.macroscopic_device()
    assert np.array_equal(rho_d.cpu().numpy(), rho_h) and np.array_equal(u_d.cpu().numpy(), u_h)


# ---------------------------------------------------- degenerate cases ----

def test_single_cell_periodic_box():
    case = periodic_box(dims=(1, 1, 1), force=(1e-4, 0, 0))
    lat = run_gpu(case, 10)
    o = run_oracle(case, 10)
    check_vs_oracle(lat, o, TOL["f64"])


def test_one_cell_thick_blocks_and_walls():
    dims = (5, 4, 3)
    case = dict(dims=dims, walls=(True, False, True), tau=0.9, wall_u={"+x": (0, 0.02, 0.01)},
                force=(0, 1e-5, 0))
    blocks = inputs.uniform_blocks(dims, (5, 4, 3))
    lat = run_gpu(case, 15, blocks=blocks)
    o = run_oracle(case, 15)
    check_vs_oracle(lat, o, TOL["f64"])


def test_all_solid_but_one_cell():
    dims = (6, 5, 4)
    solid = np.ones((4, 5, 6), np.uint8)
    solid[2, 2, 3] = 0
    case = dict(dims=dims, walls=(False, False, False), tau=0.8, force=(1e-3, 0, 0), solid=solid)
    lat = run_gpu(case, 12, blocks=inputs.uniform_blocks(dims, (2, 1, 2)))
    o = run_oracle(case, 12)
    check_vs_oracle(lat, o, TOL["f64"])
    assert lat.info()["n_fluid"] == 1


def test_zero_steps_and_errors():
    from paper_1007_1388_amd.lbm import LBMError
    lat = run_gpu(cavity(), 0)
    lat.step(0)
    assert lat.info()["steps"] == 0
    with pytest.raises(LBMError):
        lat.step(-1)
    with pytest.raises(LBMError):
        lat.set_schedule(wg_size=96)
    assert lat.schedule["wg_size"] == 256


def test_unstable_run_is_reported():
    # tau just above 1/2 with a fast lid blows up; the FP64 sums must say so
    from paper_1007_1388_amd.lbm import LBMError, LBM_EUNSTABLE
    case = cavity(dims=(12, 12, 12), lid=(0.9, 0, 0), tau=0.5 + 1e-6)
    lat = run_gpu(case, 3000, precision="f32")
    with pytest.raises(LBMError) as e:
        lat.sums()
    assert e.value.status == LBM_EUNSTABLE


def test_repeated_create_destroy_returns_device_memory():
    """Contexts of 128^3 (about 0.35 GB of grids each) created and destroyed
    in a row, with geometry, a velocity snapshot and, on every other one,
    a host Block: the device memory comes back every time."""
    import torch
    dims = (128, 128, 128)
    solid = inputs.porous_spheres(dims, target_fraction=0.05, radius=(2, 4), seed=1)
    case = channel(dims=dims, solid=solid, force=(1e-6, 0, 0), tau=0.8)
    blocks = inputs.uniform_blocks(dims, (2, 1, 1))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    for k in range(8):
        lat = run_gpu(case, 2, blocks=blocks, precision="f32")
        lat.residual_mark()
        if k % 2 == 0:
            lat.set_host_blocks([1], threads=2)
            lat.step(1)
        lat.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (256 << 20), (free0 - free1) / 2**20


@pytest.mark.parametrize("precision,key", [("f32", "gpu_bytes_sp"), ("f64", "gpu_bytes_dp")])
def test_reported_bytes_per_update_is_the_papers_model(precision, key):
    """lbm_info's bytes per fluid-cell update (the roofline's algorithmic
    bytes) is the model printed in Sec. 3.1 without obstacles, and adds the
    4-byte link mask with them."""
    from tests.test_golden import golden
    g = golden("bytes_per_update.txt")
    lat = run_gpu(channel(dims=(16, 8, 6)), 0, precision=precision)
    assert lat.info()["bytes_per_update"] == g[key]
    dims = (16, 8, 6)
    solid = inputs.porous_spheres(dims, target_fraction=0.1, radius=(1, 2), seed=3)
    lat2 = run_gpu(channel(dims=dims, solid=solid), 0, precision=precision)
    i = lat2.info()
    assert i["bytes_per_update"] == g[key] + 4.0 * i["n_cells"] / i["n_fluid"]
