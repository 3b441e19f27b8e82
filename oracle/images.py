"""Image-source solutions of the discrete scheme: a closed form that uses no trigonometric transform.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

§1 explains Neumann and Dirichlet walls as in-phase and out-of-phase image sources, and §5 lists the
image polarities of the four 1D boundary pairs.  For a Gaussian pulse of width sigma >= 3 dx the
sampled field is band-limited to the grid's wavenumbers to double precision, so the PSTD solution is
the free-space solution summed over images, with the staggered leapfrog's own dispersion relation
omega~(k) = (2/dt) asin(c0 k dt / 2) in place of c0 k.  The free-space solution of each image is a 1D,
2D or 3D radial wavenumber integral evaluated with Gauss-Legendre quadrature.
"""
from __future__ import annotations

import numpy as np
from scipy.special import j0

from .pstd import NEUMANN


def _theta(k: np.ndarray, c0: float, dt: float) -> np.ndarray:
    s = c0 * dt * k / 2.0
    if np.any(s > 1.0):
        raise ValueError("quadrature reaches an unstable wavenumber")
    return 2.0 * np.arcsin(s)


def _time_factor(k, c0, dt, m, u_mode):
    th = _theta(k, c0, dt)
    if u_mode == "centred":
        return np.cos(m * th)
    if u_mode == "zero":
        return np.cos(m * th + th / 2.0) / np.cos(th / 2.0)
    if u_mode == "continuous":          # omega = c0 k (no time dispersion), for comparison only
        return np.cos(m * c0 * dt * k)
    raise ValueError(u_mode)


def _quadrature(kmax: float, nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    k = 0.5 * kmax * (x + 1.0)
    return k, 0.5 * kmax * w


def free_space_gaussian(r: np.ndarray, ndim: int, amp: float, sigma: float, c0: float, dt: float,
                        m: int, u_mode: str = "centred", nq: int = 1500) -> np.ndarray:
    """Field at distance r after m steps from a radially symmetric Gaussian amp*exp(-r^2 / 2 sigma^2).

    Its spectrum is amp (2 pi)^{d/2} sigma^d exp(-k^2 sigma^2 / 2); each wavenumber evolves with the
    leapfrog factor of the chosen start.  The integral is cut where the spectrum is below 1e-40.
    """
    r = np.asarray(r, dtype=np.float64)
    kmax = np.sqrt(2.0 * 92.0) / sigma
    k, w = _quadrature(kmax, nq)
    spec = amp * (2.0 * np.pi) ** (ndim / 2.0) * sigma ** ndim * np.exp(-0.5 * (k * sigma) ** 2)
    g = spec * _time_factor(k, c0, dt, m, u_mode) * w
    flat = r.reshape(-1)
    out = np.empty_like(flat)
    chunk = 4096
    for s in range(0, flat.size, chunk):
        rr = flat[s:s + chunk, None]
        if ndim == 1:
            ker = np.cos(k[None, :] * rr) / np.pi
        elif ndim == 2:
            ker = j0(k[None, :] * rr) * k[None, :] / (2.0 * np.pi)
        elif ndim == 3:
            kr = k[None, :] * rr
            sinc = np.where(kr == 0.0, 1.0, np.sin(kr) / np.where(kr == 0.0, 1.0, kr))
            ker = sinc * k[None, :] ** 2 / (2.0 * np.pi ** 2)
        else:
            raise ValueError(ndim)
        out[s:s + chunk] = ker @ g
    return out.reshape(r.shape)


def image_positions_1d(xs: float, L: float, bc_left: int, bc_right: int, reach: float):
    """Image sources of a point x_s in [0, L] with reflecting walls at 0 and L (R = +1 Neumann, -1 Dirichlet).

    Positions 2jL + x_s carry (R_L R_R)^j and positions 2jL - x_s carry R_L (R_L R_R)^j (|R| = 1), which
    reproduces the one-period picture of §5 (left image R_L, right image R_R, double image R_L R_R).
    Only images within ``reach`` of the domain are returned.
    """
    RL = 1.0 if bc_left == NEUMANN else -1.0
    RR = 1.0 if bc_right == NEUMANN else -1.0
    J = int(np.ceil((reach + 2 * L) / (2 * L))) + 1
    out = []
    for j in range(-J, J + 1):
        for pos, pol in ((2 * j * L + xs, (RL * RR) ** abs(j)), (2 * j * L - xs, RL * (RL * RR) ** abs(j))):
            if -reach <= pos <= L + reach:
                out.append((pos, pol))
    return out


def image_solution(shape, bcs, dx, c0, dt, m, centre, amp, sigma, u_mode="centred"):
    """Field on the p nodes of a box after m steps from one Gaussian at ``centre`` (physical units).

    Separable image sets per axis; the product of per-axis polarities gives each image's sign.
    """
    ndim = len(shape)
    reach = c0 * dt * m + 14.0 * sigma
    per_axis = []
    for a in range(ndim):
        L = (shape[a] - 1) * dx
        per_axis.append(image_positions_1d(centre[a], L, bcs[a][0], bcs[a][1], reach))
    grids = np.meshgrid(*[np.arange(s) * dx for s in shape], indexing="ij")
    out = np.zeros(shape)
    idx = [0] * ndim

    def rec(a, pos, pol):
        nonlocal out
        if a == ndim:
            r2 = sum((grids[b] - pos[b]) ** 2 for b in range(ndim))
            r = np.sqrt(r2)
            near = r < reach
            if np.any(near):
                vals = np.zeros(shape)
                vals[near] = free_space_gaussian(r[near], ndim, amp, sigma, c0, dt, m, u_mode)
                out += pol * vals
            return
        for x, s in per_axis[a]:
            rec(a + 1, pos + [x], pol * s)

    rec(0, [], 1.0)
    del idx
    return out


def partial_image_positions_1d(xs: float, L: float, RL: float, RR: float, reach: float):
    """Image sources of a point x_s in [0, L] between walls of real reflection coefficients R_L (at 0) and
    R_R (at L), as in §5: every reflection off a wall multiplies an image's amplitude by that wall's R.

    Positions 2jL + x_s carry (R_L R_R)^|j|; positions 2jL - x_s carry R_R^j R_L^(j-1) for j >= 1 and
    R_L^(1-j) R_R^(-j) for j <= 0 (the left image R_L at -x_s, the right image R_R at 2L - x_s, ...).
    With R = +-1 these are the polarities of ``image_positions_1d``.  Only images within ``reach`` of
    the domain are returned.
    """
    J = int(np.ceil((reach + 2 * L) / (2 * L))) + 1
    out = []
    for j in range(-J, J + 1):
        direct = (2 * j * L + xs, (RL * RR) ** abs(j))
        mirrored = (2 * j * L - xs, RR ** j * RL ** (j - 1) if j >= 1 else RL ** (1 - j) * RR ** (-j))
        for pos, amp in (direct, mirrored):
            if -reach <= pos <= L + reach and amp != 0.0:
                out.append((pos, amp))
    return out


def partial_image_solution(shape, R_faces, dx, c0, dt, m, centre, amp, sigma, u_mode="centred"):
    """Field on the p nodes of a box with a real reflection coefficient on every face, after m steps from
    one Gaussian at ``centre``: the free-space solution summed over the separable image sources, each
    carrying the product over axes of its per-axis amplitude (``partial_image_positions_1d``).

    R_faces: [(R_L, R_R)] per axis.  This is the physical solution the weighted sums of §5 reproduce
    while no wave has met the same pair of walls twice.
    """
    ndim = len(shape)
    reach = c0 * dt * m + 14.0 * sigma
    per_axis = [partial_image_positions_1d(centre[a], (shape[a] - 1) * dx, R_faces[a][0], R_faces[a][1], reach)
                for a in range(ndim)]
    grids = np.meshgrid(*[np.arange(s) * dx for s in shape], indexing="ij")
    out = np.zeros(shape)

    def rec(a, pos, weight):
        nonlocal out
        if a == ndim:
            r = np.sqrt(sum((grids[b] - pos[b]) ** 2 for b in range(ndim)))
            near = r < reach
            if np.any(near):
                vals = np.zeros(shape)
                vals[near] = free_space_gaussian(r[near], ndim, amp, sigma, c0, dt, m, u_mode)
                out += weight * vals
            return
        for x, s in per_axis[a]:
            rec(a + 1, pos + [x], weight * s)

    rec(0, [], 1.0)
    return out


def image_summed_gaussian(shape, bcs, dx, centre, amp, sigma):
    """The initial pressure that matches ``image_solution`` at m = 0 (Gaussian plus all its images)."""
    ndim = len(shape)
    reach = 14.0 * sigma
    grids = np.meshgrid(*[np.arange(s) * dx for s in shape], indexing="ij")
    per_axis = []
    for a in range(ndim):
        L = (shape[a] - 1) * dx
        per_axis.append(image_positions_1d(centre[a], L, bcs[a][0], bcs[a][1], reach))
    out = np.zeros(shape)

    def rec(a, pos, pol):
        nonlocal out
        if a == ndim:
            r2 = sum((grids[b] - pos[b]) ** 2 for b in range(ndim))
            out += pol * amp * np.exp(-0.5 * r2 / sigma ** 2)
            return
        for x, s in per_axis[a]:
            rec(a + 1, pos + [x], pol * s)

    rec(0, [], 1.0)
    return out
