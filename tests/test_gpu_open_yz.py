"""Open faces on y or on z: the duct of the open-x tests (velocity inlet with
a tangential part, pressure outlet, a moving wall, a body force, spheres off
the open faces, a perturbed warm start) with its axes renamed so that the
open faces are y faces or z faces.  FP64 against the oracle (1e-12), FP32
against it (1e-5), bit for bit across tilings cut along and across the open
axis, exchange modes, graphs and cells per lane; checkpoint restart; solid
cells on the face rejected."""
import numpy as np
import pytest

from paper_1007_1388_amd import inputs
from tests.helpers import field_errors, gpu_lattice, prepare, run_oracle
from tests.test_gpu_parity import TOL, check_vs_oracle, duct, run_gpu

pytestmark = pytest.mark.gpu

# spatial axis k of the x duct becomes axis PERM[k]: x -> y, or x -> z
PERMS = {"y": (1, 2, 0), "z": (2, 0, 1)}


def permuted(case, perm):
    names = "xyz"
    inv = [perm.index(j) for j in range(3)]
    axes = [2 - inv[2 - t] for t in range(3)]   # arrays are [z][y][x]

    def vec(v):
        return tuple(v[inv[j]] for j in range(3))

    def face(f):
        return f[0] + names[perm[names.index(f[1])]]

    def spec(sp):
        return (sp[0], vec(sp[1])) if sp[0] == "velocity" else sp

    out = dict(dims=vec(case["dims"]), walls=vec(case["walls"]), tau=case["tau"], force=vec(case["force"]),
               wall_u={face(f): vec(v) for f, v in case.get("wall_u", {}).items()},
               open_faces={face(f): spec(sp) for f, sp in case["open_x"].items()})
    if case.get("solid") is not None:
        out["solid"] = np.ascontiguousarray(np.transpose(case["solid"], axes))
    rho, u = case["init"]
    rho2 = np.ascontiguousarray(np.transpose(rho, axes))
    u2 = np.empty((3,) + rho2.shape)
    for k in range(3):
        u2[perm[k]] = np.transpose(u[k], axes)
    out["init"] = (rho2, u2)
    return out


def yz_duct(axis, **kw):
    return permuted(duct(**kw), PERMS[axis])


@pytest.mark.parametrize("axis", ["y", "z"])
@pytest.mark.parametrize("steps", [0, 1, 150])
def test_open_faces_on_y_and_z_f64_match_oracle(axis, steps):
    case = yz_duct(axis)
    lat = run_gpu(case, steps)
    o = run_oracle(case, steps)
    check_vs_oracle(lat, o, TOL["f64"])


@pytest.mark.parametrize("axis", ["y", "z"])
def test_open_faces_on_y_and_z_f32_storage(axis):
    case = yz_duct(axis)
    lat = run_gpu(case, 150, precision="f32")
    o = run_oracle(case, 150)
    rho_g, u_g = lat.macroscopic()
    rho_o, u_o = o.macroscopic()
    err = field_errors(rho_g, u_g, rho_o, u_o)
    assert err["u_inf"] <= TOL["f32"] and err["drho_inf"] <= TOL["f32"], err


def _tilings(dims, a):
    """Blocks cut along the open axis a, across it, both, and unevenly."""
    along = [1, 1, 1]
    along[a] = 3
    across = [2, 2, 2]
    across[a] = 1
    t1, t2 = [k for k in range(3) if k != a]
    cut = lambda k, f: [0, int(dims[k] * f), dims[k]]
    uneven = []
    ca, c1, c2 = cut(a, 0.3), cut(t1, 0.6), cut(t2, 0.45)
    for i in range(2):
        for j in range(2):
            for k in range(2):
                lo, hi = [0, 0, 0], [0, 0, 0]
                lo[a], hi[a] = ca[i], ca[i + 1]
                lo[t1], hi[t1] = c1[j], c1[j + 1]
                lo[t2], hi[t2] = c2[k], c2[k + 1]
                uneven.append((tuple(lo), tuple(hi)))
    return [inputs.uniform_blocks(dims, tuple(along)), inputs.uniform_blocks(dims, tuple(across)),
            inputs.uniform_blocks(dims, (2, 2, 2)), uneven]


@pytest.mark.parametrize("axis", ["y", "z"])
@pytest.mark.parametrize("variant", range(5))
def test_open_faces_on_y_and_z_bitwise_across_tilings(axis, variant):
    """Bit for bit against the one-Block run (every exchange mode, graph
    capture, uneven cuts, a periodic tangential axis whose boundary-node
    images sit in ghost cells of the far Blocks), and FP64 against the
    oracle."""
    case = yz_duct(axis)
    a = "xyz".index(axis)
    dims = case["dims"]
    tl = _tilings(dims, a)
    blocks = [tl[0], tl[1], tl[2], tl[3], tl[2]][variant]
    sched = [dict(fused_exchange=0), dict(fused_exchange=1), dict(fused_exchange=2),
             dict(fused_exchange=2, graph_steps=4), dict(fused_exchange=1, graph_steps=5)][variant]
    ref = run_gpu(case, 41, precision="f32")
    lat = run_gpu(case, 41, blocks=blocks, precision="f32", schedule=sched)
    assert np.array_equal(lat.get_state(as_fp64=False), ref.get_state(as_fp64=False))
    f64 = run_gpu(case, 41, blocks=blocks, schedule=sched)
    o = run_oracle(case, 41)
    check_vs_oracle(f64, o, TOL["f64"])


def test_open_z_faces_two_cells_per_lane_bitwise():
    """Open z faces leave the sweep untouched: FP16S and BF16S with two cells
    per lane give the one-cell-per-lane result bit for bit (x extent even)."""
    case = yz_duct("z")
    assert case["dims"][0] % 2 == 0
    for prec in ("f16s", "bf16s"):
        a = run_gpu(case, 33, precision=prec, schedule=dict(cells_per_lane=1))
        b = run_gpu(case, 33, precision=prec, schedule=dict(cells_per_lane=2),
                    blocks=inputs.uniform_blocks(case["dims"], (1, 2, 2)))
        assert np.array_equal(a.get_state(as_fp64=False), b.get_state(as_fp64=False))


@pytest.mark.parametrize("axis", ["y", "z"])
def test_open_faces_on_y_and_z_checkpoint_restart(axis):
    case = yz_duct(axis)
    a_ = "xyz".index(axis)
    dims = case["dims"]
    a = run_gpu(case, 30, blocks=_tilings(dims, a_)[2])
    f = a.get_state(as_fp64=True)
    b = gpu_lattice(case, blocks=_tilings(dims, a_)[0])
    prepare(b, case)
    b.set_state(f, as_fp64=True)
    a.step(20)
    b.step(20)
    fa, fb = a.get_state(as_fp64=True), b.get_state(as_fp64=True)
    assert np.abs(fa - fb).max() <= 1e-12 * np.abs(fa).max()


@pytest.mark.parametrize("axis", ["y", "z"])
def test_open_faces_on_y_and_z_reject_solid_on_the_face(axis):
    from paper_1007_1388_amd import lbm
    case = yz_duct(axis, obstacles=False)
    lat = gpu_lattice(case)
    a = "xyz".index(axis)
    solid = np.zeros(lat.shape, np.uint8)
    idx = [2, 3, 4]
    idx[2 - a] = lat.shape[2 - a] - 1
    solid[tuple(idx)] = 1
    with pytest.raises(lbm.LBMError):
        lat.set_geometry(solid)
    solid[tuple(idx)] = 0
    idx[2 - a] = 3
    solid[tuple(idx)] = 1
    lat.set_geometry(solid)
