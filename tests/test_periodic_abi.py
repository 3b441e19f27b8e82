"""Periodic axes in the library (CPU only): the host operator tables of a periodic pair equal the
oracle's periodic grad/div matrices, formed independently (FFT there, direct sine sums here); a plan
rejects an axis with one periodic face before any device work."""
import ctypes as C

import numpy as np
import pytest

from oracle import pstd as opstd
from paper_2005_00322_amd import PERIODIC, axis_operator
from paper_2005_00322_amd import _lib


@pytest.mark.parametrize("n", [3, 4, 16, 17, 64, 129])
def test_tables_match_oracle(n):
    dx = 1e-4
    ax = opstd.PeriodicAxis(n, dx)
    G = axis_operator(n, PERIODIC, PERIODIC, dx, 0)
    Dm = axis_operator(n, PERIODIC, PERIODIC, dx, 1)
    assert G.shape == Dm.shape == (n, n)
    scale = np.pi / dx
    assert np.max(np.abs(G - ax.grad_matrix())) < 1e-13 * scale
    assert np.max(np.abs(Dm - ax.div_matrix())) < 1e-13 * scale


def test_mixed_faces_rejected():
    lib = _lib.load()
    g = _lib.Grid()
    g.ndim = 2
    g.n[0], g.n[1], g.n[2] = 16, 16, 1
    bcs = (C.c_int32 * 6)(PERIODIC, 0, 0, 0, 0, 0)
    h = C.c_void_p()
    rc = lib.pstd_plan_create_ex(C.byref(g), 1e-4, 1e-8, 1500.0, bcs, 1000.0, 1, None, None, C.byref(h))
    assert rc == _lib.E_INVALID_ARG
    with pytest.raises(Exception):
        axis_operator(8, PERIODIC, 0, 1e-4, 0)
