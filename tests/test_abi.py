"""CPU checks of the C ABI (no GPU): the library loads and exports every declared symbol, its FP64 host
tables equal the oracle's operators formed independently, and argument errors are reported before any
device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import pstd as opstd
from paper_2005_00322_amd import _lib
from paper_2005_00322_amd.pstd import axis_operator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N, D = opstd.NEUMANN, opstd.DIRICHLET


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pstd_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert names <= set(_lib.SIGNATURES), names - set(_lib.SIGNATURES)


def test_status_strings():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.pstd_status_string(code)
    assert lib.pstd_status_string(0) == b"ok"


@pytest.mark.parametrize("bc", [(N, N), (N, D), (D, N), (D, D)])
@pytest.mark.parametrize("n", [3, 4, 17, 64, 129, 384])
def test_host_tables_match_oracle(bc, n):
    dx = 1e-4
    ax = opstd.Axis(n, bc[0], bc[1], dx)
    G = axis_operator(n, bc[0], bc[1], dx, 0)
    Dm = axis_operator(n, bc[0], bc[1], dx, 1)
    scale = np.pi / dx
    assert np.max(np.abs(G - ax.grad_matrix())) < 2e-13 * scale
    assert np.max(np.abs(Dm - ax.div_matrix())) < 2e-13 * scale


def _grid(shape):
    g = _lib.Grid()
    g.ndim = len(shape)
    for a, s in enumerate(shape):
        g.n[a] = s
    return g


def _faces(*f):
    arr = (C.c_int32 * 6)()
    for i, v in enumerate(f):
        arr[i] = v
    return arr


def test_argument_errors_need_no_device():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.pstd_plan_create(C.byref(_grid((10, 10))), 1e-4, 1e-8, 1500.0, _faces(0, 0, 0, 0), None) == _lib.E_INVALID_ARG
    g0 = _lib.Grid()
    g0.ndim = 0
    assert lib.pstd_plan_create(C.byref(g0), 1e-4, 1e-8, 1500.0, _faces(), C.byref(h)) == _lib.E_INVALID_ARG
    assert lib.pstd_plan_create(C.byref(_grid((2, 10))), 1e-4, 1e-8, 1500.0, _faces(), C.byref(h)) == _lib.E_INVALID_ARG
    assert lib.pstd_plan_create(C.byref(_grid((10,))), -1e-4, 1e-8, 1500.0, _faces(), C.byref(h)) == _lib.E_INVALID_ARG
    assert lib.pstd_plan_create(C.byref(_grid((10,))), 1e-4, 1e-8, 1500.0, _faces(0, 7), C.byref(h)) == _lib.E_INVALID_ARG
    assert lib.pstd_plan_create(C.byref(_grid((5000,))), 1e-4, 1e-8, 1500.0, _faces(), C.byref(h)) == _lib.E_UNSUPPORTED
    assert b"nodes" in lib.pstd_last_error()


def test_periodic_axis_size_limits_need_no_device():
    # a periodic axis above 4097 points runs only on the FFT path: a power of two up to 8192 with a float
    # state; every other case is refused before any device work
    lib = _lib.load()
    h = C.c_void_p()
    P = opstd.PERIODIC
    dx, c0 = 1e-4, 1500.0
    dt = 0.1 * dx / c0
    for n, prec in ((8193, _lib.FP32), (12288, _lib.FP32), (16384, _lib.FP32), (8192, _lib.FP64)):
        st = lib.pstd_plan_create_ex(C.byref(_grid((n, 8))), dx, dt, c0, _faces(P, P, N, D), 1000.0, prec, None,
                                     None, C.byref(h))
        assert st == _lib.E_UNSUPPORTED, (n, prec)
        assert b"periodic" in lib.pstd_last_error()


@pytest.mark.parametrize("shape,bcs", [((65,), (N, N)), ((33, 40), (N, N, D, N)), ((20, 20, 20), (N, D, D, D, N, N))])
def test_stability_limit_enforced(shape, bcs):
    lib = _lib.load()
    dx, c0 = 1e-4, 1500.0
    prob = opstd.Problem(shape, tuple(zip(bcs[0::2], bcs[1::2])), dx, 1e-9, c0)
    limit = prob.cfl_limit()
    h = C.c_void_p()
    dt_bad = 1.001 * limit * dx / c0
    assert lib.pstd_plan_create(C.byref(_grid(shape)), dx, dt_bad, c0, _faces(*bcs), C.byref(h)) == _lib.E_UNSTABLE
    if len(shape) == 1:
        assert abs(limit - 2.0 / np.pi) < 1e-12     # §4.2's 1D limit for Neumann at both ends


def test_nop_predict_rejects_bad_arguments_before_device_work():
    lib = _lib.load()
    g = _lib.NopGate(0.1, 1400.0, 1600.0, 3.0, 10, 1e-3)
    pr = _lib.NopProblem()
    pr.dx, pr.dt, pr.rho0, pr.steps = 1e-4, 1e-8, 1000.0, 10
    nf = C.c_int32(-1)
    # null surrogate handle, null gate, null buffers
    assert lib.pstd_nop_predict(None, C.byref(g), C.byref(pr), 1, 1, 1, 4, 0.5, None, C.byref(nf)) == _lib.E_INVALID_ARG
    assert lib.pstd_nop_predict(None, None, C.byref(pr), 1, 1, 1, 4, 0.5, None, None) == _lib.E_INVALID_ARG
    assert nf.value == -1
    assert b"null" in lib.pstd_last_error()


def test_step_prepare_rejects_bad_arguments():
    lib = _lib.load()
    st = _lib.State()
    assert lib.pstd_step_prepare(None, C.byref(st), 10) == _lib.E_INVALID_ARG
    assert lib.pstd_step_prepare(None, None, 10) == _lib.E_INVALID_ARG
