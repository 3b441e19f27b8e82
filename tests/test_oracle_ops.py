"""Pins of the oracle's per-axis operators (CPU only).

* Table transform_choices is what the oracle uses (golden fixture, §4.1).
* Every eigen-mode of each boundary pair is differentiated exactly onto the staggered grid, in both
  directions (closed forms cos/sin of k_n x, Nyquist included).
* The velocity and pressure operators are adjoint up to sign, W D = -G^T, with weight 1/2 on Neumann
  wall nodes: a transposed operand or a dropped Nyquist term breaks it.
* The spectrum of -div grad is {k_n^2}; its top for a Neumann-Neumann axis is (pi/dx)^2, which gives
  the 1D stability limit CFL = 2/pi printed in §4.2.
* The printed forward transform S4 for WAWS in the staggered-differentiation appendix table is a typo:
  it does not differentiate WAWS modes, S3 (Table DTT_wavenumber_groups, Table transform_choices) does.
"""
import json
import os

import numpy as np
import pytest

from oracle import dtt, pstd
from oracle import pstd as opstd

N, D = pstd.NEUMANN, pstd.DIRICHLET
CASES = [(N, N), (N, D), (D, N), (D, D)]


def test_transform_choices_table(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "transform_choices.json")))
    for row in g["rows"]:
        ax = pstd.Axis(12, "ND".index(row["left"]), "ND".index(row["right"]), 0.1)
        assert ax.p_sym == row["p"] and ax.u_sym == row["u"]
        assert "%s%d" % ax.T1_id == row["T1"] and "%s%d" % ax.T2_id == row["T2"]
        assert ax.a1_sign == (-1.0 if row["a1"] == "-k" else 1.0)
        assert ax.a2_sign == (-1.0 if row["a2"] == "-k" else 1.0)


def _mode(ax, k, x):
    # Neumann left end -> cosine (even about node 0), Dirichlet -> sine (odd about node 0)
    return np.cos(k * x) if ax.bc_left == N else np.sin(k * x)


def _dmode(ax, k, x):
    return -k * np.sin(k * x) if ax.bc_left == N else k * np.cos(k * x)


@pytest.mark.parametrize("bc", CASES)
@pytest.mark.parametrize("n", [5, 16, 33, 64])
def test_single_modes_are_differentiated_exactly(bc, n):
    dx = 1e-4
    ax = pstd.Axis(n, bc[0], bc[1], dx)
    x = np.arange(n) * dx
    xh = (np.arange(n - 1) + 0.5) * dx
    # every wavenumber the pressure basis carries (T1 range), Nyquist of NN included
    for k in ax.k1:
        f = _mode(ax, k, x)
        g = ax.grad(f)
        assert np.max(np.abs(g - _dmode(ax, k, xh))) <= 1e-12 * max(k, 1.0 / dx)
    # velocity modes: derivative of u's basis function lands on the p nodes
    for k in ax.k2:
        uh = -np.sin(k * xh) if ax.bc_left == N else np.cos(k * xh)
        du = ax.div(uh)
        ref = -k * np.cos(k * x) if ax.bc_left == N else -k * np.sin(k * x)
        ref[ax.node_weights() == 0.0] = 0.0
        assert np.max(np.abs(du - ref)) <= 1e-12 * max(k, 1.0 / dx)


@pytest.mark.parametrize("bc", CASES)
@pytest.mark.parametrize("n", [6, 31, 50])
def test_skew_adjoint(bc, n):
    ax = pstd.Axis(n, bc[0], bc[1], 1e-4)
    G, Dm = ax.grad_matrix(), ax.div_matrix()
    W = np.diag(ax.node_weights())
    scale = np.max(np.abs(G))
    assert np.max(np.abs(W @ Dm + G.T)) < 1e-13 * scale
    # Dirichlet nodes are inert: zero columns of G, zero rows of D
    dead = ax.node_weights() == 0.0
    assert np.all(G[:, dead] == 0.0) and np.all(Dm[dead, :] == 0.0)


@pytest.mark.parametrize("bc", CASES)
def test_spectrum_and_stability_limit(bc, golden_dir):
    n, dx = 40, 1e-4
    ax = pstd.Axis(n, bc[0], bc[1], dx)
    A = -ax.div_matrix() @ ax.grad_matrix()
    live = ax.node_weights() > 0
    ev = np.sort(np.linalg.eigvals(A[np.ix_(live, live)]).real)
    assert np.allclose(ev, np.sort(ax.k1 ** 2), rtol=1e-10, atol=1e-6 * (np.pi / dx) ** 2 * 1e-6)
    prob = pstd.Problem((n,), (bc,), dx, 1e-9, 1500.0)
    if bc == (N, N):
        g = json.load(open(os.path.join(golden_dir, "stability.json")))
        assert abs(prob.cfl_limit() - g["cfl_limit_1d_num"] / np.pi) < 1e-14
        assert abs(np.max(ev) - (np.pi / dx) ** 2) < 1e-10 * (np.pi / dx) ** 2
    else:
        assert prob.cfl_limit() > 2.0 / np.pi


def test_waws_forward_transform_reading():
    # DN axis: p is WAWS.  Differentiating + interpolating with S3 (the reading used) is exact; the
    # S4 printed in the appendix's staggered table is not.
    n, dx = 20, 1e-4
    ax = pstd.Axis(n, D, N, dx)
    x = np.arange(n) * dx
    xh = (np.arange(n - 1) + 0.5) * dx
    k = ax.k1[3]
    f = np.sin(k * x)
    good = ax.grad(f)
    assert np.max(np.abs(good - k * np.cos(k * xh))) < 1e-9 * k
    sample = f[1:]
    wrong = (ax.a1_sign * ax.k1 * (dtt.matrix("S", 4, n - 1) @ sample)) @ ax.T2inv.T
    assert np.max(np.abs(wrong - k * np.cos(k * xh))) > 1e-2 * k


@pytest.mark.parametrize("bc", [(N, N), (N, D), (D, N), (D, D)])
@pytest.mark.parametrize("n", [9, 26])
def test_axis_mode_closed_form_and_eigen(bc, n):
    # the pressure basis functions are the cosines/sines of Table DTT_wavenumber_groups on the nodes:
    # NN cos(pi m j/N), DD sin(pi m j/N), ND cos(pi (m+1/2) j/N), DN sin(pi (m+1/2) j/N)
    Nn = n - 1
    j = np.arange(n)
    dx = 0.5
    ax = opstd.Axis(n, bc[0], bc[1], dx)
    for m in range(len(ax.k1)):
        mode, k = opstd.axis_mode(n, bc[0], bc[1], dx, m)
        if bc == (N, N):
            ref, kr = np.cos(np.pi * m * j / Nn), np.pi * m / Nn
        elif bc == (D, D):
            ref, kr = np.sin(np.pi * (m + 1) * j / Nn), np.pi * (m + 1) / Nn
        elif bc == (N, D):
            ref, kr = np.cos(np.pi * (m + 0.5) * j / Nn), np.pi * (m + 0.5) / Nn
        else:
            ref, kr = np.sin(np.pi * (m + 0.5) * j / Nn), np.pi * (m + 0.5) / Nn
        ref = ref / np.max(np.abs(ref))
        assert np.allclose(mode, ref, atol=1e-12)
        assert abs(k - kr / dx) < 1e-12 / dx
        # eigenfunction of div o grad with eigenvalue -k^2
        assert np.allclose(ax.div_matrix() @ (ax.grad_matrix() @ mode), -k * k * mode, atol=1e-10 * max(k * k, 1.0 / dx**2))


def test_single_mode_evolves_with_the_leapfrog_phase():
    # 2D, one mode per axis: p^m = cos(m theta) p^0 with sin(theta/2) = c0 dt |k| / 2
    shape, bcs, dx, c0 = (13, 17), ((D, N), (N, N)), 1e-3, 1500.0
    dt = 0.3 * dx / c0
    fx, kx = opstd.axis_mode(shape[0], D, N, dx, 3)
    fy, ky = opstd.axis_mode(shape[1], N, N, dx, 5)
    p0 = np.outer(fx, fy)
    th = opstd.mode_phase(c0, dt, kx * kx + ky * ky)
    prob = opstd.Problem(shape, bcs, dx, dt, c0)
    p, _ = prob.run(p0, 37)
    assert np.max(np.abs(p - np.cos(37 * th) * p0)) < 1e-12
