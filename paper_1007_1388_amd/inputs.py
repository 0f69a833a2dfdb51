"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no lattice Boltzmann arithmetic: it only draws geometries
(solid masks), block tilings and random perturbation fields from numpy's
PCG64 generator, so the GPU library and the CPU oracle can be fed the very
same data.

Workload shapes follow the paper's synthetic scenarios: lid-driven cavities
(Sec. 5), single-Block cubes and domains split into a Cartesian grid of
Blocks (Sec. 4.2, Sec. 5.1), extended with the channel, porous-channel and
precision presets the benchmark uses.
"""
import numpy as np


# ----------------------------------------------------------- geometries -----

def porous_spheres(dims, target_fraction=0.10, radius=(3, 8), seed=0,
                   periodic=(True, True, False)):
    """Random spheres until the solid fraction reaches ``target_fraction``.

    dims = (nx, ny, nz); returns uint8 [nz, ny, nx], 1 = solid.  Centres are
    uniform in the domain, radii are integers uniform in [radius[0],
    radius[1]]; a cell is solid when its centre lies within the radius of a
    sphere, taking periodic images on the axes flagged ``periodic``.  Each
    sphere only touches its bounding box.
    """
    nx, ny, nz = (int(d) for d in dims)
    n = [nx, ny, nz]
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), dtype=bool)
    target = float(target_fraction) * solid.size
    if target <= 0:
        return solid.astype(np.uint8)
    count = 0
    for _ in range(1_000_000):
        c = rng.uniform(0, 1, 3) * np.array(n)
        r = int(rng.integers(radius[0], radius[1] + 1))
        idx, d2 = [], []
        for axis in range(3):
            lo = int(np.floor(c[axis] - r)) - 1
            hi = int(np.ceil(c[axis] + r)) + 2
            cells = np.arange(lo, hi)
            if periodic[axis]:
                cells = cells[(cells - lo) < n[axis]] if hi - lo > n[axis] else cells
                wrapped = cells % n[axis]
                # distance to the nearest periodic image of the centre
                dd = np.abs(wrapped - c[axis])
                diff = np.minimum(dd, n[axis] - dd)
                order = np.unique(wrapped, return_index=True)[1]
                wrapped, diff = wrapped[order], diff[order]
                idx.append(wrapped)
                d2.append(diff * diff)
            else:
                keep = (cells >= 0) & (cells < n[axis])
                cells = cells[keep]
                idx.append(cells)
                d2.append((cells - c[axis]) ** 2)
        if any(len(v) == 0 for v in idx):
            continue
        ball = (d2[2][:, None, None] + d2[1][None, :, None] + d2[0][None, None, :]) <= r * r
        box = np.ix_(idx[2], idx[1], idx[0])
        before = solid[box]
        count += int((ball & ~before).sum())
        solid[box] = before | ball
        if count >= target:
            break
    return solid.astype(np.uint8)


def fill_isolated_pores(solid, periodic=(True, True, False)):
    """Make solid every fluid cell outside the largest connected pore space.

    solid: uint8 [nz, ny, nx].  Two fluid cells are connected when one of
    the 18 D3Q19 links joins them (across the faces flagged ``periodic``,
    taken as (x, y, z)).  A pocket that no link joins to the main pore space
    carries no flow, and with a body force it keeps a population cycle of
    period two (bounce-back reverses its momentum every step), so it is
    filled.  Returns a new uint8 array.
    """
    from scipy import ndimage
    sol = np.asarray(solid, dtype=bool)
    fluid = ~sol
    struct = np.ones((3, 3, 3), dtype=bool)
    for c in [(0, 0, 0), (0, 0, 2), (0, 2, 0), (0, 2, 2), (2, 0, 0), (2, 0, 2), (2, 2, 0), (2, 2, 2)]:
        struct[c] = False
    pz, py, px = (1 if periodic[2] else 0), (1 if periodic[1] else 0), (1 if periodic[0] else 0)
    padded = np.pad(fluid, ((pz, pz), (py, py), (px, px)), mode="wrap")
    lab, n = ndimage.label(padded, structure=struct)
    if n == 0:
        return sol.astype(np.uint8)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    # a padded cell is the periodic image of an interior cell: join their labels
    nz, ny, nx = fluid.shape
    zz, yy, xx = np.nonzero(lab)
    inner = lab[pz:pz + nz, py:py + ny, px:px + nx]
    img = inner[(zz - pz) % nz, (yy - py) % ny, (xx - px) % nx]
    for a, b in set(zip(lab[zz, yy, xx].tolist(), img.tolist())):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    roots = np.array([find(k) for k in range(n + 1)])
    comp = roots[inner]
    comp[~fluid] = 0
    counts = np.bincount(comp.ravel())
    counts[0] = 0
    keep = int(np.argmax(counts))
    out = sol | (comp != keep)
    return out.astype(np.uint8)


_LINKS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
          (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def fill_trapped_cells(solid, periodic=(True, True, False)):
    """Fill fluid cells whose open links do not span 3-D space, repeatedly,
    then the pores outside the main pore space (``fill_isolated_pores``).

    solid: uint8 [nz, ny, nx]; non-periodic faces count as walls.  In a cell
    whose open link directions e (neighbour x + e fluid) all lie in one plane,
    the momentum component normal to that plane is conserved by the
    collision and reversed by bounce-back on every step, so it oscillates
    with period two and never decays; a body force feeds it.  The test is
    det(sum over open links of e e^T) == 0, exact in integers.  Returns a new
    uint8 array.
    """
    sol = np.asarray(solid, dtype=bool).copy()
    nz, ny, nx = sol.shape
    while True:
        fluid = ~sol
        G = np.zeros((6,) + sol.shape, dtype=np.int64)  # xx, yy, zz, xy, xz, yz
        for ex, ey, ez in _LINKS:
            nb = fluid
            for axis, e in ((2, ex), (1, ey), (0, ez)):
                if e == 0:
                    continue
                per = periodic[2 - axis]
                nb = np.roll(nb, -e, axis=axis)   # nb[c] = fluid[c + e]
                if not per:
                    idx = [slice(None)] * 3
                    idx[axis] = slice(-1, None) if e > 0 else slice(0, 1)
                    nb = nb.copy()
                    nb[tuple(idx)] = False
            o = nb.astype(np.int64)
            G[0] += o * ex * ex
            G[1] += o * ey * ey
            G[2] += o * ez * ez
            G[3] += o * ex * ey
            G[4] += o * ex * ez
            G[5] += o * ey * ez
        xx, yy, zz, xy, xz, yz = G
        det = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz)
        bad = fluid & (det == 0)
        if not bad.any():
            break
        sol |= bad
    return fill_isolated_pores(sol.astype(np.uint8), periodic)


def channel_obstacle(dims, center=None, radius=3):
    """One sphere obstacle in a channel (deterministic), uint8 [nz, ny, nx]."""
    nx, ny, nz = dims
    c = center if center is not None else (nx / 2 - 0.5, ny / 2 - 0.5, nz / 2 - 0.5)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
    return (d2 <= radius * radius).astype(np.uint8)


# --------------------------------------------------------------- tilings ----

def uniform_blocks(dims, counts):
    """Cartesian grid of near-equal Blocks: counts = (bx, by, bz).

    Returns a list of (lo, hi) half-open cell boxes in BlockID order (x
    fastest), like the paper's Patch split into a Cartesian grid of Blocks
    (Sec. 4.2).
    """
    cuts = []
    for n, k in zip(dims, counts):
        edges = [round(j * n / k) for j in range(k + 1)]
        cuts.append(edges)
    return _product(cuts)


def segments(length, choices, rng, max_tries=10000):
    """Split ``length`` into segments drawn uniformly from ``choices``.

    Draws until the running sum reaches ``length``; accepts if it is exact,
    otherwise redraws from scratch.
    """
    for _ in range(max_tries):
        out, s = [], 0
        while s < length:
            v = int(rng.choice(choices))
            out.append(v)
            s += v
        if s == length:
            return out
    raise ValueError("no exact split of %d from %s" % (length, choices))


def uneven_blocks(dims, choices=(32, 48, 64), seed=0):
    """Seeded uneven Cartesian tiling: per axis, segments from ``choices``.

    The Blocks are the Cartesian product of the three axis splits, so every
    face and edge neighbour is unique (a rectilinear grid of Blocks).
    """
    rng = np.random.default_rng(seed)
    cuts = []
    for n in dims:
        seg = segments(n, choices, rng)
        cuts.append([0] + list(np.cumsum(seg)))
    return _product(cuts)


def uneven_blocks_grid(counts=(4, 4, 4), choices=(32, 48, 64), seed=0):
    """Exactly bx*by*bz Blocks with per-axis edge lengths drawn from ``choices``;
    the domain is whatever the lengths sum to.  Returns (dims, blocks)."""
    rng = np.random.default_rng(seed)
    cuts, dims = [], []
    for k in counts:
        seg = [int(rng.choice(choices)) for _ in range(k)]
        cuts.append([0] + list(np.cumsum(seg)))
        dims.append(int(sum(seg)))
    return tuple(dims), _product(cuts)


def _product(cuts):
    blocks = []
    cx, cy, cz = cuts
    for k in range(len(cz) - 1):
        for j in range(len(cy) - 1):
            for i in range(len(cx) - 1):
                blocks.append(((int(cx[i]), int(cy[j]), int(cz[k])),
                               (int(cx[i + 1]), int(cy[j + 1]), int(cz[k + 1]))))
    return blocks


def random_tiling(dims, max_blocks_per_axis=3, seed=0, min_edge=1):
    """Random rectilinear tiling with arbitrary (possibly tiny) edges."""
    rng = np.random.default_rng(seed)
    cuts = []
    for n in dims:
        k = int(rng.integers(1, max_blocks_per_axis + 1))
        k = min(k, n // min_edge)
        inner = sorted(rng.choice(np.arange(min_edge, n - min_edge + 1), size=k - 1,
                                  replace=False).tolist()) if k > 1 else []
        edges = [0] + inner + [n]
        # enforce the minimum edge
        ok = all(b - a >= min_edge for a, b in zip(edges[:-1], edges[1:]))
        cuts.append(edges if ok else [0, n])
    return _product(cuts)


# ------------------------------------------------------- random fields ------

def perturbed_fields(dims, seed=0, drho=1e-3, du=1e-2, rho0=1.0):
    """Random (rho, u) fields: rho [nz,ny,nx], u [3,nz,ny,nx], FP64."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    rho = rho0 + drho * rng.standard_normal((nz, ny, nx))
    u = du * rng.standard_normal((3, nz, ny, nx))
    return rho, u


# ---------------------------------------------------------------- presets ---

def preset(name):
    """Named workloads (dicts of plain parameters, no arithmetic).

    cavity32      32^3 lid-driven cavity, FP64, tau 0.6, lid (0.05,0,0) on +z
    poiseuille256 256^3 channel, periodic x,y, walls z, g_x 1e-6, tau 0.8
    porous512     512x256x256 porous channel, uneven {32,48,64} Blocks,
                  spheres r 3..8 to 10 % solid, tau 0.7, g_x 1e-6
    cavity384     384^3 cavity, tau 0.55, lid (0.1,0,0)
    warmstart     64x64x128 porous channel, tau 0.7 (surrogate data)
    """
    p = {
        "cavity32": dict(dims=(32, 32, 32), walls=(True, True, True), tau=0.6,
                         wall_u={"+z": (0.05, 0.0, 0.0)}, force=(0.0, 0.0, 0.0), steps=100),
        "poiseuille256": dict(dims=(256, 256, 256), walls=(False, False, True), tau=0.8,
                              wall_u={}, force=(1e-6, 0.0, 0.0), steps=2000),
        "porous512": dict(dims=(512, 256, 256), walls=(False, False, True), tau=0.7,
                          wall_u={}, force=(1e-6, 0.0, 0.0), steps=1000,
                          solid_fraction=0.10, radius=(3, 8), block_edges=(32, 48, 64)),
        "cavity384": dict(dims=(384, 384, 384), walls=(True, True, True), tau=0.55,
                          wall_u={"+z": (0.1, 0.0, 0.0)}, force=(0.0, 0.0, 0.0), steps=5000),
        "warmstart": dict(dims=(64, 64, 128), walls=(False, False, True), tau=0.7,
                          wall_u={}, solid_fraction=(0.05, 0.20), force_range=(5e-7, 5e-6)),
    }
    return dict(p[name])
