"""Pins of the oracle's transform definitions (CPU only).

* Each matrix equals scipy.fft's unnormalised DCT/DST of the same type, whose sums are FFTW's
  REDFT/RODFT definitions adopted in §3.2.
* The inverse relations of Eq. (inverse_transforms) hold as identities.
* Periods and wavenumber ranges match Table DTT_wavenumber_groups (golden fixture).
* The worked gradient of Eq. (dtt_gradient_example_I), (1/M) S2{-k C3{f}} with M = 2N, differentiates
  WSWA modes exactly.
"""
import json
import os

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import dtt, pstd


@pytest.mark.parametrize("kind", ["C", "S"])
@pytest.mark.parametrize("typ", [1, 2, 3, 4])
@pytest.mark.parametrize("L", [2, 3, 8, 17, 64])
def test_matrix_matches_library(kind, typ, L):
    rng = np.random.default_rng(typ * 100 + L)
    x = rng.standard_normal((3, L))
    lib = (sfft.dct if kind == "C" else sfft.dst)(x, type=typ, norm=None, axis=-1)
    ours = x @ dtt.matrix(kind, typ, L).T
    assert np.max(np.abs(ours - lib)) <= 1e-12 * max(1.0, np.max(np.abs(lib)))


@pytest.mark.parametrize("kind", ["C", "S"])
@pytest.mark.parametrize("typ", [1, 2, 3, 4])
@pytest.mark.parametrize("L", [2, 5, 16, 33])
def test_inverse_relations(kind, typ, L):
    T = dtt.matrix(kind, typ, L)
    Ti = dtt.inverse_matrix(kind, typ, L)
    assert np.max(np.abs(Ti @ T - np.eye(L))) < 1e-12
    assert np.max(np.abs(T @ Ti - np.eye(L))) < 1e-12


def test_inverse_pairing_is_the_printed_one():
    # Eq. (inverse_transforms): j=3 -> T2, j=1,4 -> itself, j=2 -> T3
    assert dtt.inverse_pair("C", 1) == ("C", 1)
    assert dtt.inverse_pair("C", 2) == ("C", 3)
    assert dtt.inverse_pair("C", 3) == ("C", 2)
    assert dtt.inverse_pair("S", 4) == ("S", 4)
    # and it is the only pairing of the four types that inverts (a transposed operand would not)
    for kind in "CS":
        for j in (1, 2, 3, 4):
            ok = [t for t in (1, 2, 3, 4)
                  if np.allclose(dtt.matrix(kind, t, 9) @ dtt.matrix(kind, j, 9) / dtt.period(kind, j, 9), np.eye(9))]
            assert ok == [dtt.inverse_pair(kind, j)[1]]


def test_wavenumber_table(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "wavenumber_groups.json")))
    for row in g["rows"]:
        kind, typ = row["dtt"][0], int(row["dtt"][1])
        for N in (6, 9):
            M = dtt.period(kind, typ, N)
            assert M == {"2(N-1)": 2 * (N - 1), "2N": 2 * N, "2(N+1)": 2 * (N + 1)}[row["M"]]
            idx, periodic = pstd.wavenumber_indices(kind, typ, M)
            assert periodic == (row["group"] == "periodic")
            env = {"M": M}
            assert idx[0] == eval(row["n_first"], env)
            assert idx[-1] == eval(row["n_last"], env)
            # one coefficient per representative sample
            assert len(idx) == N


def test_worked_gradient_example():
    # d/dx f = (1/M) S2{-k C3{f}}, WSWA sample of length N, M = 2N, k = 2 pi (n + 1/2) / (M dx)
    N, dx = 24, 0.01
    M = 2 * N
    x = np.arange(N) * dx
    T = dtt.matrix("C", 3, N)
    Sinv = dtt.matrix("S", 2, N) / M
    n, periodic = pstd.wavenumber_indices("C", 3, M)
    k = pstd.wavenumbers(n, periodic, M, dx)
    for q in range(N):
        f = np.cos(k[q] * x)                 # a WSWA mode (cosine, zero half a period past the end)
        df = Sinv @ (-k * (T @ f))
        # the result is WAWS: its representative sample starts one node past the antisymmetric point
        assert np.max(np.abs(df - (-k[q] * np.sin(k[q] * (x + dx))))) < 1e-11 * k[q]
