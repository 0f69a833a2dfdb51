"""Parity at the benchmark sizes: the full workloads, checked on outputs the
oracle can produce one by one (a 1x1xN column for a translation-invariant
channel, light-cone windows of a porous domain) and on properties that hold
at any size (translation invariance, partition invariance, conservation)."""
import numpy as np
import pytest

import oracle
from paper_1007_1388_amd import inputs
from tests.helpers import field_errors, gpu_lattice

pytestmark = pytest.mark.gpu


def test_cavity32_full_fp64():
    p = inputs.preset("cavity32")
    lat = gpu_lattice(p, precision="f64")
    lat.step(p["steps"])
    o = oracle.OracleLBM(p["dims"], walls=p["walls"], wall_u=p["wall_u"], tau=p["tau"])
    o.step(p["steps"])
    err = field_errors(*lat.macroscopic(), *o.macroscopic())
    assert err["u_inf"] < 1e-12 and err["drho_inf"] < 1e-12, err
    m0 = 32 ** 3
    m, _ = lat.sums()
    assert abs(m - m0) < 1e-11 * m0


def _column_oracle(p, steps):
    nz = p["dims"][2]
    o = oracle.OracleLBM((1, 1, nz), walls=p["walls"], tau=p["tau"], force=p["force"])
    o.step(steps)
    rho, u = o.macroscopic()
    return rho[:, 0, 0], u[:, :, 0, 0]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_poiseuille256_full_against_oracle_column(precision, tol):
    # x, y periodic and a uniform force: the 256^3 field equals the 1x1x256
    # column everywhere (same recurrence per cell), so the oracle column is
    # the exact reference for every column of the GPU field.
    p = inputs.preset("poiseuille256")
    steps = p["steps"]
    lat = gpu_lattice(p, precision=precision)
    lat.step(steps)
    rho, u = lat.macroscopic()
    rho_c, u_c = _column_oracle(p, steps)
    rng = np.random.default_rng(0)
    cols = [(0, 0), (255, 255), (17, 200)] + [tuple(rng.integers(0, 256, 2)) for _ in range(5)]
    for (x, y) in cols:
        e = field_errors(rho[:, y, x][:, None, None], u[:, :, y, x][:, :, None, None],
                         rho_c[:, None, None], u_c[:, :, None, None])
        assert e["u_inf"] < tol and e["drho_inf"] < tol, (x, y, e)
    # translation invariance over the whole field (bitwise: same per-cell code)
    assert np.array_equal(u[0], np.broadcast_to(u[0][:, :1, :1], u[0].shape))
    # start-up against the continuum series (discretisation error ~3e-4)
    nu = (p["tau"] - 0.5) / 3
    H = 256
    zeta = np.arange(H) + 0.5
    g = p["force"][0]
    steady = g / (2 * nu) * zeta * (H - zeta)
    series = steady.copy()
    for n in range(1, 400, 2):
        series -= 4 * g * H * H / (nu * np.pi ** 3 * n ** 3) * np.sin(n * np.pi * zeta / H) * \
            np.exp(-n * n * np.pi ** 2 * nu * steps / H ** 2)
    dev = np.linalg.norm(u[0, :, 0, 0] - series) / np.linalg.norm(series)
    assert dev < 1e-3, dev


def _window_oracle(p, solid, center, steps, h):
    """Oracle on a periodic/walled window around `center`: after `steps`
    steps the centre cell only depends on cells within distance `steps`, so a
    window of half-width h > steps reproduces it exactly."""
    nx, ny, nz = p["dims"]
    cx, cy, cz = center
    xs = np.arange(cx - h, cx + h + 1) % nx
    ys = np.arange(cy - h, cy + h + 1) % ny
    z0, z1 = max(0, cz - h), min(nz, cz + h + 1)
    sub = solid[z0:z1][:, ys][:, :, xs]
    dims = (len(xs), len(ys), z1 - z0)
    o = oracle.OracleLBM(dims, walls=(False, False, True), tau=p["tau"], force=p["force"])
    o.set_geometry(sub)
    o.step(steps)
    rho, u = o.macroscopic()
    return rho[cz - z0, h, h], u[:, cz - z0, h, h]


def test_porous512_full_partition_invariance_and_windows():
    p = inputs.preset("porous512")
    solid = inputs.porous_spheres(p["dims"], p["solid_fraction"], p["radius"], seed=0)
    blocks = inputs.uneven_blocks(p["dims"], p["block_edges"], seed=0)
    steps = 12
    a = gpu_lattice(p, blocks=blocks, precision="f32")
    a.set_geometry(solid)
    a.set_schedule(fused_exchange=2)  # x faces written by the sweep, the rest by the copy kernel
    a.step(steps)
    fa = a.get_state(as_fp64=False)
    ra, ua = a.macroscopic()
    a.close()
    b = gpu_lattice(p, precision="f32")
    b.set_geometry(solid)
    b.step(steps)
    assert np.array_equal(b.get_state(as_fp64=False), fa)
    b.close()
    del fa
    rng = np.random.default_rng(1)
    fluid = np.argwhere(solid == 0)
    picks = fluid[rng.choice(len(fluid), 6, replace=False)]
    picks = np.vstack([picks, [[0, 5, 7], [255, 100, 511]]])  # next to both walls
    for z, y, x in picks:
        if solid[z, y, x]:
            continue
        r_o, u_o = _window_oracle(p, solid, (x, y, z), steps, steps + 2)
        scale = max(np.abs(u_o).max(), 1e-12)
        assert np.abs(ua[:, z, y, x] - u_o).max() <= 1e-5 * scale + 1e-12, (x, y, z)
        # density by the same normwise bar (drho errors over max(|drho|,
        # |u|)), plus the FP64 rounding of rho0 + drho
        assert abs(ra[z, y, x] - r_o) <= 1e-5 * max(abs(r_o - 1.0), scale) + 1e-12, (x, y, z)


@pytest.mark.slow
def test_porous512_full_domain_against_oracle_100_steps():
    """The whole 512x256x256 porous channel in its 250 uneven Blocks (default
    schedule: x faces written by the sweep, the rest by the copy kernel)
    against the FP64 oracle of the whole domain after 100 steps: velocity and
    every population, FP64 storage to 1e-12, FP32 storage to 1e-5.  (The
    density itself is compared through the populations: rho = rho0 + drho in
    FP64 resolves drho only to ~1e-16, which at this flow scale, |u| ~ 1e-4,
    is already 1e-12 relative.)"""
    p = inputs.preset("porous512")
    solid = inputs.porous_spheres(p["dims"], p["solid_fraction"], p["radius"], seed=0)
    blocks = inputs.uneven_blocks(p["dims"], p["block_edges"], seed=0)
    steps = 100
    o = oracle.OracleLBM(p["dims"], walls=p["walls"], tau=p["tau"], force=p["force"])
    o.set_geometry(solid)
    o.step(steps)
    _, u_o = o.macroscopic()
    f_o = o.get_state()
    o.close()
    fluid = solid == 0
    scale = max(np.abs(f_o).max(), np.abs(np.asarray(p["force"])).max())
    for precision, tol in (("f64", 1e-12), ("f32", 1e-5)):
        lat = gpu_lattice(p, blocks=blocks, precision=precision)
        lat.set_geometry(solid)
        lat.step(steps)
        _, u_g = lat.macroscopic()
        du = u_g[:, fluid] - u_o[:, fluid]
        u_inf = np.abs(du).max() / np.abs(u_o[:, fluid]).max()
        f_g = lat.get_state()
        lat.close()
        f_err = np.abs(f_g - f_o).max() / scale
        del f_g
        assert u_inf <= tol and f_err <= tol, (precision, u_inf, f_err)
