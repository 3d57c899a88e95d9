"""The C-ABI library loads, exports every declared entry point, and rejects
bad arguments on the host before any device work (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1303_2470_amd import lbmp
    if not os.path.exists(lbmp.LIB_PATH):
        from paper_1303_2470_amd import build_lib
        build_lib.build()
    return lbmp.load_library()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "lbmp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z][a-z_0-9]*)\s*\(", txt)) - {"if", "sizeof"})


def test_every_declared_symbol_is_exported(lib):
    from paper_1303_2470_amd import lbmp
    names = declared_functions()
    assert "mp_step_n" in names and "lb_flow_solve" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lbmp.EXPORTS)


def test_version_and_error_string(lib):
    assert b"lbmp" in lib.lbmp_version()
    assert isinstance(lib.lbmp_last_error(), bytes)


def _geom(lbmp, mask, periodic=(1, 1, 1), nb=18):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = m.shape
    return lbmp.Geometry(nx, ny, nz, (ctypes.c_int * 3)(*periodic), ctypes.c_void_p(m.ctypes.data), nb), m


def test_host_validation_errors(lib):
    from paper_1303_2470_amd import inputs, lbmp
    f = (ctypes.c_double * 3)(0, 0, 0)
    out = ctypes.c_void_p()
    # tau <= 1/2
    g, m = _geom(lbmp, inputs.slit_mask(4, 4, 8))
    assert lib.lb_flow_solve(ctypes.byref(g), 0.5, f, 1e-10, 10, 100, None, 0, None, 0, None,
                             ctypes.byref(out), None, None) == -1
    # all solid
    g, m = _geom(lbmp, np.ones((4, 4, 4)))
    assert lib.lb_flow_solve(ctypes.byref(g), 1.0, f, 1e-10, 10, 100, None, 0, None, 0, None,
                             ctypes.byref(out), None, None) == -1
    assert b"no fluid" in lib.lbmp_last_error()
    # z not periodic but boundary planes fluid
    g, m = _geom(lbmp, np.zeros((6, 4, 4)), periodic=(1, 1, 0))
    assert lib.lb_flow_solve(ctypes.byref(g), 1.0, f, 1e-10, 10, 100, None, 0, None, 0, None,
                             ctypes.byref(out), None, None) == -1
    # a non-periodic slit axis with solid walls is accepted by the size query
    g, m = _geom(lbmp, inputs.slit_mask(4, 4, 8), periodic=(1, 1, 0))
    p, s = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lb_flow_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(s)) == 0
    assert p.value > 0 and s.value >= 19 * 8 * 2 * 4 * 4 * 8
    # workspace too small
    g, m = _geom(lbmp, inputs.slit_mask(4, 4, 8))
    assert lib.lb_flow_solve(ctypes.byref(g), 1.0, f, 1e-10, 10, 100, ctypes.c_void_p(256), 16,
                             ctypes.c_void_p(256), 16, None, ctypes.byref(out), None, None) == -3
    # bad handles
    assert lib.mp_step_n(None, 1) == -6
    assert lib.lb_flow_velocity(None, None) == -6
    assert lib.mp_uptake(None, 0, 0, 1, None, None) == -6
    assert lib.mp_uptake_init(None, None, 1, 32, 10, None, 0, None, None) == -1
    # invalid interface rule
    g, m = _geom(lbmp, inputs.slit_mask(4, 4, 8), nb=7)
    assert lib.lb_flow_solve(ctypes.byref(g), 1.0, f, 1e-10, 10, 100, None, 0, None, 0, None,
                             ctypes.byref(out), None, None) in (-1, -3)
