"""Discrete trigonometric transforms of groups I and II as explicit FP64 matrices.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper adopts FFTW's unnormalised definitions (§3.2, the paragraph after Eq. (inverse_transforms)),
and groups I and II of Table DTT_wavenumber_groups are exactly FFTW's REDFT00/10/01/11 (DCT-I..IV) and
RODFT00/10/01/11 (DST-I..IV).  Each matrix below is the direct O(L^2) cosine/sine sum of that
definition for an input of length L; nothing is factorised.

Pins (tests/test_oracle_dtt.py): equality with ``scipy.fft.dct/dst(type=t, norm=None)``, which use the
same unnormalised sums, and the inverse relations of Eq. (inverse_transforms).
"""
from __future__ import annotations

import numpy as np

# Logical period M of each transform for a representative sample of length L
# (Table DTT_wavenumber_groups, columns "M=...").
_PERIOD = {
    ("C", 1): lambda L: 2 * (L - 1),
    ("C", 2): lambda L: 2 * L,
    ("C", 3): lambda L: 2 * L,
    ("C", 4): lambda L: 2 * L,
    ("S", 1): lambda L: 2 * (L + 1),
    ("S", 2): lambda L: 2 * L,
    ("S", 3): lambda L: 2 * L,
    ("S", 4): lambda L: 2 * L,
}


def period(kind: str, typ: int, L: int) -> int:
    """Implied period M of the symmetric periodic sequence of a length-L sample (Table DTT_wavenumber_groups)."""
    return _PERIOD[(kind, typ)](L)


def matrix(kind: str, typ: int, L: int) -> np.ndarray:
    """Forward transform matrix T (L x L) with y = T @ x, FFTW convention (§3.2).

    kind is "C" (cosine) or "S" (sine); typ is 1..4.  Row index = output index, column = input index.
    """
    if L < 1:
        raise ValueError("transform length must be >= 1")
    j = np.arange(L, dtype=np.float64)[None, :]  # input index
    k = np.arange(L, dtype=np.float64)[:, None]  # output index
    pi = np.pi
    if (kind, typ) == ("C", 1):
        if L < 2:
            raise ValueError("DCT-I needs L >= 2")
        T = 2.0 * np.cos(pi * j * k / (L - 1))
        T[:, 0] = 1.0
        T[:, L - 1] = (-1.0) ** k[:, 0]
    elif (kind, typ) == ("C", 2):
        T = 2.0 * np.cos(pi * (j + 0.5) * k / L)
    elif (kind, typ) == ("C", 3):
        T = 2.0 * np.cos(pi * j * (k + 0.5) / L)
        T[:, 0] = 1.0
    elif (kind, typ) == ("C", 4):
        T = 2.0 * np.cos(pi * (j + 0.5) * (k + 0.5) / L)
    elif (kind, typ) == ("S", 1):
        T = 2.0 * np.sin(pi * (j + 1.0) * (k + 1.0) / (L + 1))
    elif (kind, typ) == ("S", 2):
        T = 2.0 * np.sin(pi * (j + 0.5) * (k + 1.0) / L)
    elif (kind, typ) == ("S", 3):
        T = 2.0 * np.sin(pi * (j + 1.0) * (k + 0.5) / L)
        T[:, L - 1] = (-1.0) ** k[:, 0]
    elif (kind, typ) == ("S", 4):
        T = 2.0 * np.sin(pi * (j + 0.5) * (k + 0.5) / L)
    else:
        raise ValueError(f"unsupported transform {kind}{typ}")
    return T


def inverse_pair(kind: str, typ: int) -> tuple[str, int]:
    """Transform whose (1/M)-scaled forward form is the inverse of T_typ, Eq. (inverse_transforms).

    T_j^{-1} = T_{j-1}/M for j = 3, 7;  T_j/M for j = 1, 4, 5, 8;  T_{j+1}/M for j = 2, 6.
    The kind (cosine or sine) is unchanged.
    """
    if typ in (3, 7):
        return kind, typ - 1
    if typ in (1, 4, 5, 8):
        return kind, typ
    if typ in (2, 6):
        return kind, typ + 1
    raise ValueError(typ)


def inverse_matrix(kind: str, typ: int, L: int) -> np.ndarray:
    """(1/M) * T_pair, the inverse of ``matrix(kind, typ, L)`` per Eq. (inverse_transforms)."""
    pk, pt = inverse_pair(kind, typ)
    return matrix(pk, pt, L) / period(kind, typ, L)


def apply(T: np.ndarray, x: np.ndarray, axis: int) -> np.ndarray:
    """Apply a transform matrix along one axis of an nd array (a plain matrix product per line)."""
    y = np.tensordot(T, x, axes=([1], [axis]))   # one matrix product over all lines
    return np.moveaxis(y, 0, axis)
