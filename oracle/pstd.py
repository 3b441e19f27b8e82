"""FP64 reference of the DTT-based PSTD method: operators, time stepping, closed forms, combination.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Canonical layout (the reading of "N nodes" used throughout): along an axis with ``n`` pressure nodes
p sits at x_j = j*dx, j = 0..n-1, with the two walls on nodes 0 and n-1, so L = (n-1)*dx and every
boundary case has the implied period M = 2(n-1).  The particle velocity sits on the n-1 staggered
points (j+1/2)*dx.  A Dirichlet wall node is not an unknown and holds p = 0.

Each function cites the passage of arXiv:2005.00322 it follows.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import product

import numpy as np

from . import dtt

NEUMANN = 0
DIRICHLET = 1
PERIODIC = 2   # both faces of an axis (last row of Table transform_choices: the Fourier basis)
# Right face only: the wall lies half a grid step beyond the last node, on the last staggered point
# (groups III and IV of Table DTT_wavenumber_groups, odd implied period M = 2n - 1).
NEUMANN_HALF = 3
DIRICHLET_HALF = 4

# Table transform_choices (§4.1): boundary pair (left, right) -> sequence types of p and u, the forward
# transforms T1 (acts on p) and T2 (acts on u), and the signs of the k-space coefficients a1 = ±k, a2 = ±k.
_TRANSFORM_CHOICES = {
    (NEUMANN, NEUMANN): ("NN", "WSWS", "HAHA", ("C", 1), ("S", 2), -1.0, +1.0),
    (NEUMANN, DIRICHLET): ("ND", "WSWA", "HAHS", ("C", 3), ("S", 4), -1.0, +1.0),
    (DIRICHLET, NEUMANN): ("DN", "WAWS", "HSHA", ("S", 3), ("C", 4), +1.0, -1.0),
    (DIRICHLET, DIRICHLET): ("DD", "WAWA", "HSHS", ("S", 1), ("C", 2), +1.0, -1.0),
}


def wavenumber_indices(kind: str, typ: int, M: int) -> tuple[np.ndarray, bool]:
    """Wavenumber index n carried by each output entry of a transform, and whether its group is periodic.

    Table DTT_wavenumber_groups: periodic group I has k_n = 2*pi*n/(M dx) with n = 0..M/2 (DCT-I),
    0..M/2-1 (DCT-II), 1..M/2-1 (DST-I), 1..M/2 (DST-II); antiperiodic group II has
    k_n = 2*pi*(n+1/2)/(M dx) with n = 0..M/2-1 for DCT/DST-III and -IV.
    """
    h = M // 2
    if (kind, typ) == ("C", 1):
        return np.arange(0, h + 1), True
    if (kind, typ) == ("C", 2):
        return np.arange(0, h), True
    if (kind, typ) == ("S", 1):
        return np.arange(1, h), True
    if (kind, typ) == ("S", 2):
        return np.arange(1, h + 1), True
    if typ in (3, 4):
        return np.arange(0, h), False
    raise ValueError((kind, typ))


def wavenumbers(idx: np.ndarray, periodic: bool, M: int, dx: float) -> np.ndarray:
    """k_n of Table DTT_wavenumber_groups for the given indices."""
    shift = 0.0 if periodic else 0.5
    return 2.0 * np.pi * (idx + shift) / (M * dx)


def _reindex(coef: np.ndarray, src_idx: np.ndarray, dst_idx: np.ndarray) -> np.ndarray:
    """Move k-space entries from one transform's wavenumber range to another's (last axis).

    §3.3: where the two ranges differ, the DC / Nyquist entries the inverse transform does not carry
    are dropped and those it carries but the forward transform did not produce are set to zero.
    """
    out = np.zeros(coef.shape[:-1] + (len(dst_idx),), dtype=coef.dtype)
    pos = {int(n): m for m, n in enumerate(src_idx)}
    for m_dst, n in enumerate(dst_idx):
        m_src = pos.get(int(n))
        if m_src is not None:
            out[..., m_dst] = coef[..., m_src]
    return out


@dataclass
class Axis:
    """One axis of the grid with its boundary pair, following Table transform_choices (§4.1).

    ``grad`` is the velocity-step operator T2^{-1}{a1 T1{p}} (p nodes -> staggered points) and
    ``div`` the pressure-step operator T1^{-1}{a2 T2{u}} (staggered points -> p nodes), both built
    from the rows of the appendix tables "Differentiation with staggered grids" for groups I and II.
    """

    n: int
    bc_left: int
    bc_right: int
    dx: float

    def __post_init__(self):
        if self.n < 3:
            raise ValueError("an axis needs at least 3 nodes")
        (self.name, self.p_sym, self.u_sym, self.T1_id, self.T2_id,
         self.a1_sign, self.a2_sign) = _TRANSFORM_CHOICES[(self.bc_left, self.bc_right)]
        n = self.n
        # Representative sample of p: a whole-sample antisymmetric (Dirichlet) end excludes its wall node.
        self.p_lo = 0 if self.bc_left == NEUMANN else 1
        self.p_hi = n - 1 if self.bc_right == NEUMANN else n - 2
        Lp = self.p_hi - self.p_lo + 1
        Lu = n - 1
        self.M = dtt.period(*self.T1_id, Lp)
        if self.M != dtt.period(*self.T2_id, Lu) or self.M != 2 * (n - 1):
            raise AssertionError("inconsistent implied periods")
        self.T1 = dtt.matrix(*self.T1_id, Lp)
        self.T2 = dtt.matrix(*self.T2_id, Lu)
        self.T1inv = dtt.inverse_matrix(*self.T1_id, Lp)
        self.T2inv = dtt.inverse_matrix(*self.T2_id, Lu)
        self.n1, per1 = wavenumber_indices(*self.T1_id, self.M)
        self.n2, per2 = wavenumber_indices(*self.T2_id, self.M)
        if per1 != per2:
            raise AssertionError("T1 and T2 must be in the same group")
        self.periodic = per1
        self.k1 = wavenumbers(self.n1, per1, self.M, self.dx)
        self.k2 = wavenumbers(self.n2, per2, self.M, self.dx)

    # -- the two operators of Eq. (dtt_pstd_solution), along the last axis --------------------------
    def grad(self, p: np.ndarray) -> np.ndarray:
        """T2^{-1}{a1 T1{p}}: derivative of p interpolated to the staggered points (last axis)."""
        sample = p[..., self.p_lo:self.p_hi + 1]
        coef = sample @ self.T1.T                                  # forward T1
        coef = coef * (self.a1_sign * self.k1)                     # multiply by a1 = ±k
        coef = _reindex(coef, self.n1, self.n2)                    # onto the range of T2^{-1}
        return coef @ self.T2inv.T                                 # inverse of T2 = (1/M) T2_pair

    def div(self, u: np.ndarray) -> np.ndarray:
        """T1^{-1}{a2 T2{u}}: derivative of u interpolated back to the p nodes (last axis)."""
        coef = u @ self.T2.T                                       # forward T2
        coef = coef * (self.a2_sign * self.k2)                     # multiply by a2 = ±k
        coef = _reindex(coef, self.n2, self.n1)                    # onto the range of T1^{-1}
        sample = coef @ self.T1inv.T                               # inverse of T1 = (1/M) T1_pair
        out = np.zeros(u.shape[:-1] + (self.n,), dtype=np.float64)
        out[..., self.p_lo:self.p_hi + 1] = sample                 # Dirichlet wall nodes stay 0
        return out

    # -- helpers used by the closed forms and invariants --------------------------------------------
    def node_weights(self) -> np.ndarray:
        """Quadrature weights on the p nodes: 1/2 at a Neumann wall node, 0 at a Dirichlet one, else 1."""
        w = np.ones(self.n)
        w[0] = 0.5 if self.bc_left == NEUMANN else 0.0
        w[-1] = 0.5 if self.bc_right == NEUMANN else 0.0
        return w

    @property
    def m(self) -> int:
        """Staggered points."""
        return self.n - 1

    def stag_weights(self) -> np.ndarray:
        return np.ones(self.n - 1)

    def grad_matrix(self) -> np.ndarray:
        """The linear map ``grad`` as an (n-1) x n matrix (columns of Dirichlet nodes are zero)."""
        return self.grad(np.eye(self.n)).T

    def div_matrix(self) -> np.ndarray:
        """The linear map ``div`` as an n x (n-1) matrix (rows of Dirichlet nodes are zero)."""
        return self.div(np.eye(self.n - 1)).T

    # -- collocated differentiation and staggered interpolation (§3.3, §3.4) ------------------------
    # Differentiation turns a symmetric sequence into an antisymmetric one and back; interpolation by
    # half a grid step keeps the symmetry and swaps whole-sample for half-sample ends.  On the p nodes
    # the sequence of the other symmetry is taken by the transform of the other kind and the same type
    # as T1 (the antisymmetric end of a Neumann wall excludes its node, the symmetric end of a Dirichlet
    # wall includes it); on the staggered points by the other kind and the same type as T2.
    def _dual_range(self) -> tuple[int, int]:
        lo = 1 if self.bc_left == NEUMANN else 0
        hi = self.n - 2 if self.bc_right == NEUMANN else self.n - 1
        return lo, hi

    def _dual_inverse(self, tid, L):
        kind, typ = tid
        other = ("S" if kind == "C" else "C", typ)
        idx, _ = wavenumber_indices(*other, self.M)
        return idx, dtt.inverse_matrix(*other, L)

    def _to_nodes(self, coef, src_idx):
        """Inverse transform onto the p nodes with the symmetry opposite to p's (zero outside its sample)."""
        lo, hi = self._dual_range()
        idx, inv = self._dual_inverse(self.T1_id, hi - lo + 1)
        out = np.zeros(coef.shape[:-1] + (self.n,), dtype=np.float64)
        out[..., lo:hi + 1] = _reindex(coef, src_idx, idx) @ inv.T
        return out

    def _to_staggered(self, coef, src_idx):
        """Inverse transform onto the staggered points with the symmetry opposite to u's."""
        idx, inv = self._dual_inverse(self.T2_id, self.n - 1)
        return _reindex(coef, src_idx, idx) @ inv.T

    def collocated_grad_p(self, p: np.ndarray) -> np.ndarray:
        """dp/dx on the p nodes (§3.3): forward T1, multiply by a1 = ±k, inverse of the other kind."""
        coef = p[..., self.p_lo:self.p_hi + 1] @ self.T1.T
        return self._to_nodes(coef * (self.a1_sign * self.k1), self.n1)

    def collocated_grad_u(self, u: np.ndarray) -> np.ndarray:
        """du/dx on the staggered points (§3.3): forward T2, multiply by a2 = ±k, inverse of the other kind."""
        coef = u @ self.T2.T
        return self._to_staggered(coef * (self.a2_sign * self.k2), self.n2)

    def interp_p_to_u(self, p: np.ndarray) -> np.ndarray:
        """p resampled on the staggered points (§3.4): forward T1, no k factor, half-sample inverse."""
        coef = p[..., self.p_lo:self.p_hi + 1] @ self.T1.T
        return self._to_staggered(coef, self.n1)

    def interp_u_to_p(self, u: np.ndarray) -> np.ndarray:
        """u resampled on the p nodes (§3.4): forward T2, no k factor, whole-sample inverse."""
        return self._to_nodes(u @ self.T2.T, self.n2)

    def resample_matrix(self, which: int) -> np.ndarray:
        """2: collocated d/dx on the nodes (n x n); 3: collocated d/dx on the staggered points
        ((n-1) x (n-1)); 4: nodes -> staggered points ((n-1) x n); 5: staggered points -> nodes (n x (n-1))."""
        fn, size = {2: (self.collocated_grad_p, self.n), 3: (self.collocated_grad_u, self.n - 1),
                    4: (self.interp_p_to_u, self.n), 5: (self.interp_u_to_p, self.n - 1)}[which]
        return fn(np.eye(size)).T


class PeriodicAxis:
    """A periodic axis (Fourier basis, last row of Table transform_choices): p on the n nodes j dx and u on
    the n staggered points (j + 1/2) dx, one period n dx.  The staggered derivatives are those of
    Eq. (fourier_pstd_solution) (§2) with the DFT: grad multiplies the spectrum by i k e^{+i k dx/2} (p
    nodes to u points, the shift property Eq. (fourier_shift_property) with a = dx/2), div by
    i k e^{-i k dx/2} (u points back to p nodes); k_m = 2 pi m / (n dx) over the signed indices of §2
    (m = -n/2 .. n/2 - 1 for even n).  The Nyquist factor i k e^{i k dx/2} = -pi/dx is real, so both maps
    are real.
    """

    def __init__(self, n: int, dx: float):
        if n < 3:
            raise ValueError("an axis needs at least 3 nodes")
        self.n, self.dx = int(n), float(dx)
        self.bc_left = self.bc_right = PERIODIC
        self.p_lo, self.p_hi = 0, self.n - 1
        self.m = self.n
        self.M = self.n
        self.periodic = True
        self.k = 2.0 * np.pi * np.fft.fftfreq(self.n, d=self.dx)
        self.k1 = np.abs(self.k)
        # the DFT as a matrix (for the modal closed form): T1 x = fft(x), T1inv its inverse
        j = np.arange(self.n)
        self.T1 = np.exp(-2j * np.pi * np.outer(j, j) / self.n)
        self.T1inv = np.conj(self.T1) / self.n

    def grad(self, p: np.ndarray) -> np.ndarray:
        f = 1j * self.k * np.exp(0.5j * self.k * self.dx)
        return np.fft.ifft(np.fft.fft(p, axis=-1) * f, axis=-1).real

    def div(self, u: np.ndarray) -> np.ndarray:
        f = 1j * self.k * np.exp(-0.5j * self.k * self.dx)
        return np.fft.ifft(np.fft.fft(u, axis=-1) * f, axis=-1).real

    def stag_weights(self) -> np.ndarray:
        return np.ones(self.n)

    def node_weights(self) -> np.ndarray:
        return np.ones(self.n)

    def grad_matrix(self) -> np.ndarray:
        """``grad`` as an n x n matrix."""
        return self.grad(np.eye(self.n)).T

    def div_matrix(self) -> np.ndarray:
        """``div`` as an n x n matrix."""
        return self.div(np.eye(self.n)).T


class HalfWallAxis:
    """An axis whose left wall is on node 0 and whose right wall is half a step beyond node n-1, at
    x = (n - 1/2) dx, on the last of the n staggered points (groups III/IV of Table
    DTT_wavenumber_groups: p is WSHS / WSHA / WAHS / WAHA, types V-VIII, and M = 2n - 1).

    The forward and inverse DTTs of these types are the sampled cosine / sine modes of the box and their
    inverses, so the operators of Eq. (dtt_pstd_solution) are written here from that definition: forward
    transform (the inverse of the sampled-mode matrix), multiplication by ±k, evaluation of the
    differentiated modes on the other grid.  Wavenumbers follow the group: k = 2 pi m / (M dx) when both
    walls are of one kind (group III), k = 2 pi (m + 1/2) / (M dx) otherwise (group IV).  Mode indices
    m cover as many modes as samples: a mode that vanishes on every sample of a sequence (k = pi/dx on
    an antisymmetric sequence) is not part of it.
    """

    def __init__(self, n: int, bc_left: int, bc_right: int, dx: float):
        if n < 3:
            raise ValueError("an axis needs at least 3 nodes")
        if bc_left not in (NEUMANN, DIRICHLET) or bc_right not in (NEUMANN_HALF, DIRICHLET_HALF):
            raise ValueError("a half-step wall is a right face, with a Neumann or Dirichlet left face")
        self.n, self.bc_left, self.bc_right, self.dx = n, bc_left, bc_right, dx
        self.M = 2 * n - 1
        left_n, right_n = bc_left == NEUMANN, bc_right == NEUMANN_HALF
        self.periodic = left_n == right_n                       # group III, else group IV
        shift = 0.0 if self.periodic else 0.5
        # p is a cosine series with a Neumann left wall, a sine series with a Dirichlet one; u the other
        self.pf, self.uf = (np.cos, np.sin) if left_n else (np.sin, np.cos)
        self.s1 = -1.0 if left_n else 1.0                       # d/dx of a p mode = s1 k (u mode)
        self.s2 = -self.s1                                      # d/dx of a u mode = s2 k (p mode)
        if left_n and right_n:
            m1, m2 = np.arange(0, n), np.arange(1, n)
        elif left_n:
            m1, m2 = np.arange(0, n), np.arange(0, n)
        elif right_n:
            m1, m2 = np.arange(0, n - 1), np.arange(0, n - 1)
        else:
            m1, m2 = np.arange(1, n), np.arange(0, n)
        self.n1, self.n2 = m1, m2
        self.k1 = 2.0 * np.pi * (m1 + shift) / (self.M * dx)
        self.k2 = 2.0 * np.pi * (m2 + shift) / (self.M * dx)
        self.p_lo, self.p_hi = (0 if left_n else 1), n - 1
        self.u_count = n - 1 if right_n else n                  # u = 0 on a Neumann half wall
        self.m = n                                              # staggered points stored
        self.xn = np.arange(n) * dx
        self.xs = (np.arange(n) + 0.5) * dx
        self.T1inv = self.pf(np.outer(self.xn[self.p_lo:], self.k1))
        self.T2inv = self.uf(np.outer(self.xs[:self.u_count], self.k2))
        if self.T1inv.shape[0] != len(m1) or self.T2inv.shape[0] != len(m2):
            raise AssertionError("as many modes as samples")
        self.T1 = np.linalg.inv(self.T1inv)
        self.T2 = np.linalg.inv(self.T2inv)
        self.U_all = self.uf(np.outer(self.xs, self.k2))       # u modes on all n staggered points
        self.P_all = self.pf(np.outer(self.xn, self.k1))       # p modes on all n nodes

    def grad(self, p: np.ndarray) -> np.ndarray:
        """dp/dx on the n staggered points: forward transform of p, times s1 k, u modes evaluated."""
        coef = p[..., self.p_lo:] @ self.T1.T * (self.s1 * self.k1)
        coef = _reindex(coef, self.n1, self.n2)
        return coef @ self.U_all.T

    def div(self, u: np.ndarray) -> np.ndarray:
        """du/dx on the n nodes: forward transform of u's samples, times s2 k, p modes evaluated."""
        coef = u[..., :self.u_count] @ self.T2.T * (self.s2 * self.k2)
        coef = _reindex(coef, self.n2, self.n1)
        return coef @ self.P_all.T

    def node_weights(self) -> np.ndarray:
        w = np.ones(self.n)
        w[0] = 0.5 if self.bc_left == NEUMANN else 0.0
        return w

    def stag_weights(self) -> np.ndarray:
        """Weights of the staggered points: 1/2 on the wall point of a Dirichlet half wall (where u is
        symmetric), 0 on that of a Neumann one (where u = 0)."""
        w = np.ones(self.n)
        w[-1] = 0.5 if self.bc_right == DIRICHLET_HALF else 0.0
        return w

    def grad_matrix(self) -> np.ndarray:
        return self.grad(np.eye(self.n)).T

    def div_matrix(self) -> np.ndarray:
        return self.div(np.eye(self.n)).T


def make_axis(n: int, bc_left: int, bc_right: int, dx: float):
    """The axis object of a boundary pair: periodic needs both faces periodic."""
    if (bc_left == PERIODIC) != (bc_right == PERIODIC):
        raise ValueError("a periodic axis has both faces periodic")
    if bc_left in (NEUMANN_HALF, DIRICHLET_HALF):
        raise ValueError("a half-step wall is a right face")
    if bc_right in (NEUMANN_HALF, DIRICHLET_HALF):
        return HalfWallAxis(n, bc_left, bc_right, dx)
    return PeriodicAxis(n, dx) if bc_left == PERIODIC else Axis(n, bc_left, bc_right, dx)


def _along(fn, x: np.ndarray, axis: int) -> np.ndarray:
    return np.moveaxis(fn(np.moveaxis(x, axis, -1)), -1, axis)


@dataclass
class Problem:
    """A rectangular domain with a boundary pair per axis and homogeneous (or mapped) sound speed.

    ``bcs`` holds (left, right) per axis.  ``c0`` is a scalar; an optional ``c0_map`` on the p nodes
    replaces it in the pressure step (pointwise c0(x)^2, an extension not in the paper).
    """

    shape: tuple
    bcs: tuple
    dx: float
    dt: float
    c0: float
    rho0: float = 1000.0
    c0_map: np.ndarray | None = None

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        self.bcs = tuple((int(a), int(b)) for a, b in self.bcs)
        if len(self.shape) != len(self.bcs):
            raise ValueError("one boundary pair per axis")
        self.axes = [make_axis(n, bl, br, self.dx) for n, (bl, br) in zip(self.shape, self.bcs)]

    @property
    def ndim(self) -> int:
        return len(self.shape)

    def u_shape(self, a: int) -> tuple:
        """n - 1 staggered points between two walls on nodes, n along a periodic axis or one with a
        half-step wall."""
        s = list(self.shape)
        s[a] = self.axes[a].m
        return tuple(s)

    def project(self, p: np.ndarray) -> np.ndarray:
        """Zero p on Dirichlet wall nodes (they are not unknowns of the method)."""
        q = np.array(p, dtype=np.float64, copy=True)
        for a, ax in enumerate(self.axes):
            idx = [slice(None)] * self.ndim
            if ax.bc_left == DIRICHLET:
                idx[a] = 0
                q[tuple(idx)] = 0.0
            if ax.bc_right == DIRICHLET:
                idx[a] = self.shape[a] - 1
                q[tuple(idx)] = 0.0
        return q

    def grad(self, p: np.ndarray, a: int) -> np.ndarray:
        return _along(self.axes[a].grad, p, a)

    def div(self, u: np.ndarray, a: int) -> np.ndarray:
        return _along(self.axes[a].div, u, a)

    def c2(self):
        return self.c0 ** 2 if self.c0_map is None else np.asarray(self.c0_map, dtype=np.float64) ** 2

    def initial_velocity(self, p0: np.ndarray, mode: str = "centred") -> list:
        """u^{-1/2} on every axis.

        The paper starts from zero particle velocity "accounting for the staggered grid" (§4.2) without
        a formula.  ``centred`` reads that as a time-centred u(t=0) = 0, i.e.
        u^{-1/2} = +(dt / (2 rho0)) * grad p^0, the half step of Eq. (dtt_pstd_solution_a) run
        backwards; ``zero`` is the literal u^{-1/2} = 0.
        """
        p0 = self.project(p0)
        if mode == "zero":
            return [np.zeros(self.u_shape(a)) for a in range(self.ndim)]
        if mode == "centred":
            return [(self.dt / (2.0 * self.rho0)) * self.grad(p0, a) for a in range(self.ndim)]
        raise ValueError(mode)

    def step(self, p: np.ndarray, u: list) -> tuple[np.ndarray, list]:
        """One time step, Eq. (dtt_pstd_solution) and its multi-dimensional form (§4.3).

        Every u_a is advanced from p^n first; then p^{n+1} uses all the new u_a.
        """
        u_new = [u[a] - (self.dt / self.rho0) * self.grad(p, a) for a in range(self.ndim)]
        acc = np.zeros(self.shape)
        for a in range(self.ndim):
            acc += self.div(u_new[a], a)
        p_new = p - self.dt * self.rho0 * self.c2() * acc
        return p_new, u_new

    def run(self, p0: np.ndarray, n_steps: int, u_mode: str = "centred", u0=None):
        """Advance (p^0, u^{-1/2}) by n_steps; returns (p^{n}, [u_a^{n-1/2}])."""
        p = self.project(p0)
        u = self.initial_velocity(p, u_mode) if u0 is None else [np.array(x, dtype=np.float64) for x in u0]
        for _ in range(int(n_steps)):
            p, u = self.step(p, u)
        return p, u

    # -- invariants and closed forms -----------------------------------------------------------------
    def energy(self, p: np.ndarray, u_prev: list, u_next: list) -> float:
        """Discrete acoustic energy conserved exactly by the staggered step (derived from §4.1, §4.3).

        F = sum_j w_j p_j^2 / (rho0 c0^2) + rho0 * sum_a <u_a^{n-1/2}, u_a^{n+1/2}>_a, where w is the
        product of the per-axis node weights and <.,.>_a weights the non-differentiated axes of u_a
        the same way.  It is conserved because W D_a = -G_a^T on every axis.
        """
        ws = [ax.node_weights() for ax in self.axes]
        W = ws[0]
        for w in ws[1:]:
            W = np.multiply.outer(W, w)
        F = float(np.sum(W * p * p / (self.rho0 * self.c2())))
        for a in range(self.ndim):
            Wa = np.ones(1)
            for b in range(self.ndim):
                Wa = np.multiply.outer(Wa, self.axes[a].stag_weights() if b == a else ws[b])
            Wa = Wa.reshape(self.u_shape(a))
            F += self.rho0 * float(np.sum(Wa * u_prev[a] * u_next[a]))
        return F

    def modal_solution(self, p0: np.ndarray, m: int, u_mode: str = "centred") -> np.ndarray:
        """p^m in closed form by expanding p^0 in the eigenfunctions of the T1 basis (homogeneous c0).

        Along each axis div o grad = T1^{-1} diag(-k^2) T1, so every T1 mode evolves on its own under
        the leapfrog with sin(theta/2) = c0 dt |k| / 2: p^m = P cos(m theta) for the centred start and
        P cos(m theta + theta/2) / cos(theta/2) for u^{-1/2} = 0.
        """
        if self.c0_map is not None:
            raise ValueError("modal closed form needs a homogeneous medium")
        p0 = self.project(p0)
        sample = p0[tuple(slice(ax.p_lo, ax.p_hi + 1) for ax in self.axes)]
        P = sample
        ksq = np.zeros(())
        for a, ax in enumerate(self.axes):
            P = dtt.apply(ax.T1, P, a)
            shp = [1] * self.ndim
            shp[a] = -1
            ksq = ksq + (ax.k1 ** 2).reshape(shp)
        s = self.c0 * self.dt * np.sqrt(ksq) / 2.0
        if np.any(s > 1.0):
            raise ValueError("unstable: c0 dt |k| / 2 > 1")
        theta = 2.0 * np.arcsin(s)
        if u_mode == "centred":
            fac = np.cos(m * theta)
        elif u_mode == "zero":
            fac = np.cos(m * theta + theta / 2.0) / np.cos(theta / 2.0)
        else:
            raise ValueError(u_mode)
        Q = P * fac
        for a, ax in enumerate(self.axes):
            Q = dtt.apply(ax.T1inv, Q, a)
        out = np.zeros(self.shape)
        out[tuple(slice(ax.p_lo, ax.p_hi + 1) for ax in self.axes)] = np.real(Q)   # periodic axes: the DFT
        return out

    def cfl_limit(self) -> float:
        """Largest stable c0 dt / dx: 2 / (dx * max|k|), max|k|^2 = sum over axes of the largest k^2.

        For a Neumann-Neumann axis max k = pi / dx, which gives the 1D limit 2/pi quoted in §4.2.
        """
        kmax2 = sum(float(np.max(ax.k1) ** 2) for ax in self.axes)
        return 2.0 / (self.dx * np.sqrt(kmax2))


def axis_mode(n: int, bc_left: int, bc_right: int, dx: float, m: int) -> tuple[np.ndarray, float]:
    """Pressure basis function m of one axis on its n nodes, and its wavenumber k_m.

    The basis is the inverse T1 transform of a unit coefficient (Table transform_choices gives T1,
    Table DTT_wavenumber_groups its wavenumbers): a cosine or sine of k_m x sampled on the nodes, 0 on
    Dirichlet wall nodes, scaled to a maximum magnitude of 1.  Under the operators of
    Eq. (dtt_pstd_solution) it is an eigenfunction: div(grad(mode)) = -k_m^2 mode.
    """
    ax = Axis(n, bc_left, bc_right, dx)
    e = np.zeros(len(ax.k1))
    e[m] = 1.0
    col = ax.T1inv @ e
    out = np.zeros(n)
    out[ax.p_lo:ax.p_hi + 1] = col / np.max(np.abs(col))
    return out, float(ax.k1[m])


def mode_phase(c0: float, dt: float, ksq: float) -> float:
    """Phase advance per step of a single mode under the leapfrog: sin(theta/2) = c0 dt |k| / 2."""
    s = c0 * dt * np.sqrt(ksq) / 2.0
    if s > 1.0:
        raise ValueError("unstable: c0 dt |k| / 2 > 1")
    return 2.0 * float(np.arcsin(s))


# -- §5: arbitrary real reflection coefficients by weighted sums of the Neumann/Dirichlet fields ------

# Columns: image-source polarities of the four basic 1D cases (R_L, R_R) = (1,1), (1,-1), (-1,1), (-1,-1);
# rows: left image, source, right image, doubly reflected image (matrix M of §5).
IMAGE_MATRIX = np.array([[1, 1, -1, -1],
                         [1, 1, 1, 1],
                         [1, -1, 1, -1],
                         [1, -1, -1, 1]], dtype=np.float64)

# (left, right) boundary pairs in the order of the columns of IMAGE_MATRIX (reflection 1 = Neumann).
BASIC_CASES = [(NEUMANN, NEUMANN), (NEUMANN, DIRICHLET), (DIRICHLET, NEUMANN), (DIRICHLET, DIRICHLET)]


def combination_weights_1d(RL: float, RR: float) -> np.ndarray:
    """w = (1/4) M^T r with r = [R_L, 1, R_R, R_L R_R] (§5)."""
    r = np.array([RL, 1.0, RR, RL * RR], dtype=np.float64)
    return IMAGE_MATRIX.T @ r / 4.0


def combination_weights(R_faces) -> dict:
    """Weights of the 2^(2d) basic fields for per-face reflection coefficients [(R_L, R_R) per axis].

    §5 states the 1D weights and that the same idea extends to d dimensions with 2^(2d) fields; with
    separable image sources the d-dimensional weight is the product of the per-axis 1D weights.
    Keys are tuples of (left, right) boundary pairs, one per axis.
    """
    per_axis = [combination_weights_1d(RL, RR) for RL, RR in R_faces]
    out = {}
    for choice in product(range(4), repeat=len(per_axis)):
        w = 1.0
        for a, c in enumerate(choice):
            w *= per_axis[a][c]
        out[tuple(BASIC_CASES[c] for c in choice)] = w
    return out


def combine_R(p_dirichlet: np.ndarray, p_neumann: np.ndarray, R: float) -> np.ndarray:
    """Two-field combination p_R = (1/2)(1+R) p_N + (1/2)(1-R) p_D for one coefficient R on all faces.

    This is the single-reflection restriction of §5: with every face sharing R, the all-Neumann and
    all-Dirichlet fields carry each singly reflected image with weights whose sum is R.  It is exact
    only until doubly reflected arrivals (which it weights by 1 instead of R^2).
    """
    return 0.5 * (1.0 + R) * np.asarray(p_neumann, np.float64) + 0.5 * (1.0 - R) * np.asarray(p_dirichlet, np.float64)
