"""Heterogeneous runs (Sec. 4.5, Sec. 5.3): Blocks on the host CPU next to
Blocks on the GPU, through the C ABI.

The host sweep repeats the GPU arithmetic operation for operation and the
exchange between the two memories only moves values, so a run with host
Blocks must equal the all-GPU run of the same tiling bit for bit (FP64, FP32
mixed and FP32 with FP64 arithmetic), and the FP64 run must meet the oracle
at 1e-12 like every other tiling."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs, lbm
from tests.helpers import field_errors, gpu_lattice, prepare, run_oracle

pytestmark = pytest.mark.gpu


def porous(dims=(30, 16, 14), seed=5, tau=0.7):
    solid = inputs.porous_spheres(dims, target_fraction=0.12, radius=(1, 3), seed=seed)
    rho, u = inputs.perturbed_fields(dims, seed=seed, drho=1e-3, du=1e-2)
    u[:, solid == 1] = 0.0
    return dict(dims=dims, walls=(False, False, True), tau=tau, force=(1e-5, 2e-6, 0.0), init=(rho, u),
                solid=solid)


def cavity(dims=(14, 12, 13)):
    return dict(dims=dims, walls=(True, True, True), wall_u={"+z": (0.05, 0.01, 0.0), "-x": (0.0, 0.02, 0.0)},
                tau=0.6)


def run(case, steps, blocks, host=(), precision="f64", fp64_math=False, threads=3, fused=None):
    lat = gpu_lattice(case, blocks=blocks, precision=precision, fp64_math=fp64_math)
    if fused is not None:
        lat.set_schedule(fused_exchange=fused)
    prepare(lat, case)
    if host:
        lat.set_host_blocks(list(host), threads=threads)
    lat.step(steps)
    return lat


def same_state(a, b):
    return np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))


@pytest.mark.parametrize("precision,f64m", [("f64", False), ("f32", False), ("f32", True)])
@pytest.mark.parametrize("host", [(0,), (1, 4, 11), (0, 2, 3, 5, 6, 8, 9)])
def test_host_blocks_bitwise_equal_gpu(precision, f64m, host):
    """Porous channel (periodic x, y; walls z; obstacles on Block faces;
    body force) in 3x2x2 uneven Blocks: host Blocks next to GPU Blocks, along
    faces, edges and corners, bit-identical to the all-GPU run."""
    case = porous()
    blocks = inputs.random_tiling(case["dims"], max_blocks_per_axis=3, seed=7, min_edge=2)
    nb = len(blocks)
    host = tuple(j for j in host if j < nb)
    ref = run(case, 23, blocks, precision=precision, fp64_math=f64m)
    lat = run(case, 23, blocks, host, precision=precision, fp64_math=f64m)
    assert same_state(lat, ref)
    ra, ua = lat.macroscopic()
    rb, ub = ref.macroscopic()
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)


@pytest.mark.parametrize("fused", [0, 1, 2])
def test_host_blocks_with_every_exchange_mode(fused):
    """GPU pairs exchange as the schedule says (copy kernel, sweep-written x
    faces plus rim, fully fused sweep) while host pairs use the buffers."""
    case = porous(dims=(36, 18, 16), seed=9)
    blocks = inputs.uniform_blocks(case["dims"], (3, 2, 2))
    ref = run(case, 19, blocks, precision="f32", fused=0)
    lat = run(case, 19, blocks, host=(1, 6, 10), precision="f32", fused=fused)
    assert same_state(lat, ref)


def test_moving_walls_on_the_host_match_oracle():
    """Lid-driven cavity with two moving faces, 2x2x2 Blocks, the Blocks on
    both moving faces on the host: FP64 against the oracle at 1e-12, and
    bitwise against the all-GPU run."""
    case = cavity()
    blocks = inputs.uniform_blocks(case["dims"], (2, 2, 2))
    lat = run(case, 40, blocks, host=(0, 4, 5, 6))
    ref = run(case, 40, blocks)
    assert same_state(lat, ref)
    o = run_oracle(case, 40)
    rho_g, u_g = lat.macroscopic()
    rho_o, u_o = o.macroscopic()
    e = field_errors(rho_g, u_g, rho_o, u_o)
    assert e["u_inf"] < 1e-12 and e["drho_inf"] < 1e-12, e


def test_every_block_on_the_host():
    case = porous(dims=(20, 12, 10), seed=3)
    blocks = inputs.uniform_blocks(case["dims"], (2, 2, 1))
    ref = run(case, 15, blocks)
    lat = run(case, 15, blocks, host=(0, 1, 2, 3), threads=4)
    assert same_state(lat, ref)


def test_self_wrapping_host_block():
    """A host Block that is its own neighbour in y (x extent > 64) and the
    single Block across x on the host: reads across its own faces."""
    dims = (80, 10, 9)
    case = porous(dims=dims, seed=2)
    for blocks, host in ((inputs.uniform_blocks(dims, (2, 1, 1)), (1,)), (None, (0,))):
        ref = run(case, 17, blocks, precision="f32")
        lat = run(case, 17, blocks, host, precision="f32")
        assert same_state(lat, ref)
        lat.close()
        ref.close()


@pytest.mark.parametrize("fused", [0, 2])
def test_host_blocks_with_faces_of_many_cells(fused):
    """Faces of 960 cells (40 x 24), so that every lane of the copy kernel
    moves four ghost cells of a task, on the GPU side of a host/GPU pair
    (pack and unpack through the exchange buffer) and between GPU Blocks;
    FP32 bit for bit against the all-GPU run, FP64 against the oracle."""
    dims = (96, 40, 24)
    case = porous(dims=dims, seed=8)
    blocks = inputs.uniform_blocks(dims, (3, 1, 1))
    ref = run(case, 9, blocks, precision="f32", fused=fused)
    lat = run(case, 9, blocks, (1,), precision="f32", fused=fused)
    assert same_state(lat, ref)
    f64 = run(case, 9, blocks, (2,), fused=fused)
    o = run_oracle(case, 9)
    rho_g, u_g = f64.macroscopic()
    rho_o, u_o = o.macroscopic()
    err = field_errors(rho_g, u_g, rho_o, u_o)
    assert err["u_inf"] <= 1e-12 and err["drho_inf"] <= 1e-12, err


def test_moving_blocks_between_host_and_gpu_midrun():
    """The split can change between steps: state carried over exactly,
    diagnostics (sums, residual) equal to the all-GPU run at each stage."""
    case = porous()
    blocks = inputs.uniform_blocks(case["dims"], (3, 2, 2))
    ref = run(case, 0, blocks, precision="f32")
    lat = run(case, 0, blocks, precision="f32")
    for host in ((2, 7), (0, 1, 2, 3, 4, 5), (), (11,)):
        lat.set_host_blocks(list(host), threads=2)
        lat.step(9)
        ref.step(9)
        assert same_state(lat, ref)
        m1, p1 = lat.sums()
        m2, p2 = ref.sums()
        assert m1 == m2 and np.array_equal(p1, p2)
        assert lat.residual() == ref.residual()


def test_checkpoint_and_residual_snapshot_with_host_blocks():
    """A checkpoint taken and restored while Blocks run on the host resumes
    bit for bit; the velocity snapshot residual sees the host Blocks."""
    case = porous(dims=(32, 16, 12), seed=4)
    blocks = inputs.uniform_blocks(case["dims"], (2, 2, 1))
    ref = run(case, 11, blocks, precision="f32")
    lat = run(case, 11, blocks, host=(1, 2), precision="f32")
    f = lat.get_state(as_fp64=False)
    lat.step(5)
    lat.set_state(f, as_fp64=False)
    ref.set_state(ref.get_state(as_fp64=False), as_fp64=False)
    lat.residual_mark()
    ref.residual_mark()
    lat.step(8)
    ref.step(8)
    assert same_state(lat, ref)
    assert lat.residual_since_mark() == ref.residual_since_mark()


def test_host_timing_and_balance_keep_the_state():
    case = porous(dims=(64, 32, 32), seed=1)
    blocks = inputs.uniform_blocks(case["dims"], (2, 2, 2))
    ref = run(case, 12, blocks, precision="f32")
    lat = run(case, 12, blocks, precision="f32")
    with pytest.raises(lbm.LBMError):
        lat.step_host_timed(1)           # no host Blocks yet
    k, t_gpu, t_split = lat.balance_host_blocks(threads=4, trial_steps=5)
    assert 0 <= k < 8 and t_gpu > 0 and t_split > 0
    lat.step(6)
    ref.step(6)
    assert same_state(lat, ref)
    lat.set_host_blocks([7], threads=4)
    g, c, x, s = lat.step_host_timed(3)
    ref.step(3)
    assert c > 0 and x >= 0 and s >= max(g, c)
    assert same_state(lat, ref)


def test_host_block_rules():
    case = porous(dims=(20, 12, 10))
    blocks = inputs.uniform_blocks(case["dims"], (2, 1, 1))
    lat = run(case, 1, blocks)
    for ids in ([2], [-1], [0, 0]):
        with pytest.raises(lbm.LBMError):
            lat.set_host_blocks(ids)
    with pytest.raises(lbm.LBMError):
        lat.set_host_blocks([0], threads=-1)
    lat.set_host_blocks([1])
    with pytest.raises(lbm.LBMError):
        lat.autotune(trial_steps=2)
    half = gpu_lattice(case, blocks=blocks, precision="f16s")
    with pytest.raises(lbm.LBMError):
        half.set_host_blocks([0])
