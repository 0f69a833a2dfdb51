"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1007_1388_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1007_1388_amd import build
        build.build()
    return lbm.load()


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lbm_[a-z0-9_]+)\s*\(",
                                 text, flags=re.M)))


@pytest.mark.parametrize("header", [h for h in sorted(os.listdir(os.path.join(ROOT, "include")))
                                    if h.endswith(".h")])
def test_every_declared_symbol_is_exported(header):
    _lib()
    names = _declared(header)
    assert names, "no declarations parsed from %s" % header
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (\S+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_binding_lists_the_header_symbols():
    assert sorted(lbm.SYMBOLS) == _declared("lbm.h")


def test_strerror_and_last_error():
    lib = _lib()
    assert lbm.lbm_strerror(0) == "ok"
    assert "invalid" in lbm.lbm_strerror(1)
    assert lib.lbm_last_error() is not None


def _create(params, blocks):
    return lbm.lbm_create_blocks(params, blocks)


def _status(params, blocks):
    _lib()
    try:
        _create(params, blocks)
    except lbm.LBMError as e:
        return e.status
    return 0


BOX = [((0, 0, 0), (8, 8, 8))]


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.4), dict(tau=float("nan")), dict(rho0=0.0), dict(dims=(0, 8, 8)),
    dict(precision=7), dict(force=(float("inf"), 0, 0)), dict(row_pad=-2), dict(row_pad=65),
])
def test_invalid_parameters_are_rejected(bad):
    kw = dict(dims=(8, 8, 8), tau=0.7)
    kw.update(bad)
    p = lbm.make_params(**kw) if "precision" not in bad else lbm.make_params(dims=(8, 8, 8), tau=0.7)
    if "precision" in bad:
        p.precision = bad["precision"]
    assert _status(p, BOX) == lbm.LBM_EINVAL


def test_mismatched_faces_and_normal_wall_velocity_rejected():
    p = lbm.make_params((8, 8, 8), tau=0.7)
    p.face[0] = lbm.LBM_WALL  # -x wall, +x periodic
    assert _status(p, BOX) == lbm.LBM_EINVAL
    p = lbm.make_params((8, 8, 8), walls=(True, True, True), wall_u={"+z": (0, 0, 0.1)}, tau=0.7)
    assert _status(p, BOX) == lbm.LBM_EINVAL
    p = lbm.make_params((8, 8, 8), walls=(False, False, False), wall_u={"+z": (0.1, 0, 0)}, tau=0.7)
    assert _status(p, BOX) == lbm.LBM_EINVAL


def test_open_face_rules_rejected():
    ok = dict(open_x={"-x": ("velocity", (0.01, 0, 0)), "+x": ("pressure", 1.0)})
    p = lbm.make_params((8, 8, 8), walls=(True, False, True), tau=0.7, **ok)
    p.face[2] = p.face[3] = lbm.LBM_VELOCITY          # open faces lie on one axis
    assert _status(p, BOX) == lbm.LBM_EINVAL
    for ax, walls in (("y", (True, True, False)), ("z", (False, True, True))):
        p = lbm.make_params((8, 8, 8), walls=walls, tau=0.7,
                            open_faces={"-" + ax: ("velocity", (0.0, 0.01, 0.0)), "+" + ax: ("pressure", 1.0)})
        assert _status(p, BOX) != lbm.LBM_EINVAL        # the faces of one axis, any axis
        p = lbm.make_params((8, 1, 8), walls=walls, tau=0.7, open_faces={"-" + ax: ("pressure", 1.0)})
        if ax == "y":
            assert _status(p, [((0, 0, 0), (8, 1, 8))]) == lbm.LBM_EINVAL   # two cells across
    p = lbm.make_params((8, 8, 8), walls=(True, False, True), tau=0.7, open_x={"+x": ("pressure", 0.0)})
    assert _status(p, BOX) == lbm.LBM_EINVAL            # density must be > 0
    p = lbm.make_params((8, 8, 8), walls=(False, False, True), tau=0.7, open_x={"-x": ("pressure", 1.0)})
    assert _status(p, BOX) == lbm.LBM_EINVAL            # periodic faces come in pairs
    p = lbm.make_params((1, 8, 8), walls=(True, False, True), tau=0.7, **ok)
    assert _status(p, [((0, 0, 0), (1, 8, 8))]) == lbm.LBM_EINVAL   # nx >= 2

@pytest.mark.parametrize("blocks", [
    [((0, 0, 0), (8, 8, 4))],                                   # does not cover
    [((0, 0, 0), (8, 8, 8)), ((0, 0, 0), (8, 8, 8))],           # overlap
    [((0, 0, 0), (4, 8, 8)), ((4, 0, 0), (8, 4, 8)), ((4, 4, 0), (8, 8, 8))],  # not Cartesian
    [((0, 0, 0), (9, 8, 8))],                                   # outside
    [((0, 0, 0), (0, 8, 8))],                                   # empty
    [],
])
def test_bad_tilings_rejected(blocks):
    p = lbm.make_params((8, 8, 8), tau=0.7)
    assert _status(p, blocks) == lbm.LBM_EINVAL


def test_null_arguments_rejected():
    lib = _lib()
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_step_timed(None, 1, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_residual(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_residual_mark(None) == lbm.LBM_EINVAL
    assert lib.lbm_residual_since_mark(None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_destroy(None) == lbm.LBM_OK
    assert lib.lbm_set_host_blocks(None, None, 0, 0) == lbm.LBM_EINVAL
    d = ctypes.c_double()
    assert lib.lbm_step_host_timed(None, 1, *[ctypes.byref(d)] * 4) == lbm.LBM_EINVAL
    k = ctypes.c_int32()
    assert lib.lbm_balance_host_blocks(None, 0, 10, ctypes.byref(k), None, None) == lbm.LBM_EINVAL
    assert lib.lbm_bw_probe(None, None, 16, 1, None, None) == lbm.LBM_EINVAL
    for bad in [(3, 1, 1, None, 1, 16, 0, 1, None), (0, 3, 1, 1, 1, 16, 0, 1, None), (0, 1, 1, None, 1, 16, 0, 1, None),
                (2, 1, 1, 1, 1, 24, 0, 1, None), (1, 1, 1, None, 1, 16, 0, 0, None)]:
        ms = ctypes.c_double()
        assert lib.lbm_hbm_probe(*bad[:8], bad[8], ctypes.byref(ms)) == lbm.LBM_EINVAL
