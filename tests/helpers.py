"""Shared helpers of the GPU parity tests: run the same seeded case on the HIP
library and on the CPU oracle, and the normwise error measures."""
import numpy as np

import oracle


def has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def gpu_lattice(case, blocks=None, precision="f64", fp64_math=False, **kw):
    from paper_1007_1388_amd import lbm
    return lbm.Lattice(case["dims"], blocks=blocks, walls=case.get("walls", (False, False, False)),
                       wall_u=case.get("wall_u"), tau=case["tau"], force=case.get("force", (0, 0, 0)),
                       precision=precision, fp64_math=fp64_math, open_x=case.get("open_x"),
                       open_faces=case.get("open_faces"), **kw)


def oracle_lattice(case):
    return oracle.OracleLBM(case["dims"], walls=case.get("walls", (False, False, False)),
                            wall_u=case.get("wall_u"), tau=case["tau"], force=case.get("force", (0, 0, 0)),
                            open_x=case.get("open_x"), open_faces=case.get("open_faces"))


def prepare(sim, case):
    if case.get("solid") is not None:
        sim.set_geometry(case["solid"])
    if case.get("init") is not None:
        rho, u = case["init"]
        sim.set_equilibrium(rho, u)


def run_oracle(case, steps):
    o = oracle_lattice(case)
    prepare(o, case)
    o.step(steps)
    return o


def rel_inf(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)).max()
    s = np.abs(np.asarray(b)).max()
    return d / s if s > 0 else d


def field_errors(rho_a, u_a, rho_b, u_b, rho0=1.0, fluid=None):
    """Normwise errors of (rho, u) a against reference b over fluid cells:
    u: ||du||_inf/||u||_inf and ||du||_2/||u||_2; drho: ||d drho||_inf divided by
    max(||drho_ref||_inf, ||u_ref||_inf)."""
    if fluid is None:
        fluid = np.ones(rho_b.shape, bool)
    ua, ub = u_a[:, fluid], u_b[:, fluid]
    du = ua - ub
    u_inf = np.abs(du).max() / max(np.abs(ub).max(), 1e-300)
    u_l2 = np.sqrt((du ** 2).sum()) / max(np.sqrt((ub ** 2).sum()), 1e-300)
    dr = (rho_a - rho0)[fluid] - (rho_b - rho0)[fluid]
    scale = max(np.abs(rho_b[fluid] - rho0).max(), np.abs(ub).max(), 1e-300)
    return dict(u_inf=u_inf, u_l2=u_l2, drho_inf=np.abs(dr).max() / scale)
