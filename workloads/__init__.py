"""Seeded synthetic inputs for the PSTD workloads.

This module is the only code shared by the FP64 oracle and the HIP path.  It draws problem
parameters and initial pressure fields and holds none of the method's arithmetic.  Every random
quantity comes from ``numpy.random.default_rng(SEED_BASE + index)``.

Workloads (physical set-up of the paper's examples, §4.2: water, c0 = 1500 m/s, rho0 = 1000 kg/m^3):

* ``pstd1d``   1D, 128 nodes, Dirichlet at both ends, dx = 1e-4 m, CFL 0.2, 1000 steps, Gaussian
               p0 (sigma = 4 dx) centred on a random node at least 6 sigma from the walls.
* ``pstd2d``   2D 256 x 256, Dirichlet on the x faces and Neumann on the y faces, CFL 0.3, 2000 steps,
               cosine-tapered disc p0 (flat to 4 dx, zero beyond 8 dx), random centre >= 9 dx from walls.
* ``pstd3d``   3D 384^3, each face Dirichlet or Neumann with probability 1/2, c0 = 1540 m/s, CFL 0.3,
               500 steps, three Gaussian blobs (sigma = 4 dx, amplitude U[0.5, 1]).
* ``pstd2d_large``  2D 2049 x 2049 (axes above 512 nodes: the FFT path), x faces Dirichlet, y faces
               Neumann, CFL 0.3, 200 steps, tapered disc p0 at a random centre >= 9 dx from walls.
* ``pstd3d_mode``  3D 1025^3, faces drawn like ``pstd3d``, CFL 0.3, one pressure basis function per
               axis (the mode numbers are drawn here; the function itself is the method's basis).
* ``fft_small``    random 1D/2D/3D shapes whose sides n have 2(n-1) = 16 x 2^a 3^b 5^c, random faces,
               white-noise p0 (parity sweeps of the FFT path).
* ``batched``  128 2D instances, sides uniform in {96..512}, c0 U[1400, 1600], one Gaussian blob,
               R uniform in [-1, 1]; each instance is solved twice (all-Neumann and all-Dirichlet).
* ``nop``      2D 128 x 128 surrogate pairs: 1-3 blobs (sigma U[3, 6] dx) and a smooth c0 map in
               [1400, 1600] m/s (white noise smoothed by a Gaussian of 16 dx, min-max scaled).

``scale`` shrinks a workload's grid while keeping its recipe, for parity cases the oracle finishes
in seconds.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 200500322
NEUMANN = 0
DIRICHLET = 1
PERIODIC = 2
NEUMANN_HALF = 3     # right face half a step beyond the last node
DIRICHLET_HALF = 4
RHO0 = 1000.0
DX = 1e-4


@dataclass
class Case:
    """One single-grid problem: grid, per-axis boundary pairs, physical constants, p0 and step count."""

    name: str
    shape: tuple
    bcs: tuple
    dx: float
    dt: float
    c0: float
    steps: int
    p0: np.ndarray
    rho0: float = RHO0
    precision: str = "fp32"
    c0_map: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def points(self) -> int:
        return int(np.prod(self.shape))


def rng_for(index: int, stream: int = 0) -> np.random.Generator:
    if stream == 0:
        return np.random.default_rng(SEED_BASE + index)
    # child `stream` of SeedSequence(SEED_BASE + index), built directly (same stream as .spawn()[stream])
    return np.random.default_rng(np.random.SeedSequence(SEED_BASE + index, spawn_key=(stream,)))


def gaussian(shape, dx, centre, sigma, amp=1.0) -> np.ndarray:
    """amp * exp(-|x - centre|^2 / (2 sigma^2)) on the nodes x_j = j dx."""
    grids = np.meshgrid(*[np.arange(s) * dx for s in shape], indexing="ij", sparse=True)
    r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
    return amp * np.exp(-0.5 * r2 / sigma ** 2)


def tapered_disc(shape, dx, centre, r_flat, r_out) -> np.ndarray:
    """1 inside r_flat, 0.5 (1 + cos(pi (r - r_flat) / (r_out - r_flat))) up to r_out, 0 beyond."""
    grids = np.meshgrid(*[np.arange(s) * dx for s in shape], indexing="ij", sparse=True)
    r = np.sqrt(sum((g - c) ** 2 for g, c in zip(grids, centre)))
    t = np.clip((r - r_flat) / (r_out - r_flat), 0.0, 1.0)
    return 0.5 * (1.0 + np.cos(np.pi * t))


def _centre(rng, shape, margin_nodes, dx):
    return tuple(float(rng.integers(margin_nodes, s - margin_nodes)) * dx for s in shape)


def pstd1d(scale: float = 1.0, precision: str = "fp64") -> Case:
    rng = rng_for(0)
    n = max(int(round(128 * scale)), 40)
    sigma = 4 * DX
    c0 = 1500.0
    centre = _centre(rng, (n,), 24, DX)
    p0 = gaussian((n,), DX, centre, sigma)
    return Case("pstd1d_n%d_DD" % n, (n,), ((DIRICHLET, DIRICHLET),), DX, 0.2 * DX / c0, c0,
                1000 if scale == 1.0 else 200, p0, precision=precision, extra={"centre": centre, "sigma": sigma})


def pstd2d(scale: float = 1.0, steps: int | None = None) -> Case:
    rng = rng_for(1)
    n = max(int(round(256 * scale)), 24)
    shape = (n, n)
    c0 = 1500.0
    centre = _centre(rng, shape, 9, DX)
    p0 = tapered_disc(shape, DX, centre, 4 * DX, 8 * DX)
    bcs = ((DIRICHLET, DIRICHLET), (NEUMANN, NEUMANN))
    st = 2000 if steps is None else steps
    return Case("pstd2d_%dx%d_xDD_yNN" % shape, shape, bcs, DX, 0.3 * DX / c0, c0, st, p0,
                extra={"centre": centre})


def periodic2d(n: int = 256, steps: int = 2000) -> Case:
    """The disc of pstd2d in a 256^2 domain that is periodic along x (a Fourier axis) and bounded by a
    Neumann and a Dirichlet wall along y, CFL 0.3: the wall-bounded and the Fourier discretisations of
    the method side by side in one solve."""
    rng = rng_for(7)
    shape = (n, n)
    c0 = 1500.0
    centre = _centre(rng, shape, 9, DX)
    p0 = tapered_disc(shape, DX, centre, 4 * DX, 8 * DX)
    bcs = ((PERIODIC, PERIODIC), (NEUMANN, DIRICHLET))
    return Case("periodic2d_%dx%d_xPP_yND" % shape, shape, bcs, DX, 0.3 * DX / c0, c0, steps, p0,
                extra={"centre": centre})


def halfwall2d(n: int = 256, steps: int = 2000) -> Case:
    """The disc of pstd2d in 256 x 256 nodes whose right walls lie half a step beyond the last node:
    x Neumann then Dirichlet-half (DTT types VII/VIII), y Dirichlet then Neumann-half (types VII/VIII of
    the other kind), CFL 0.3."""
    rng = rng_for(8)
    shape = (n, n)
    c0 = 1500.0
    centre = _centre(rng, shape, 9, DX)
    p0 = tapered_disc(shape, DX, centre, 4 * DX, 8 * DX)
    bcs = ((NEUMANN, DIRICHLET_HALF), (DIRICHLET, NEUMANN_HALF))
    return Case("halfwall2d_%dx%d_xNDh_yDNh" % shape, shape, bcs, DX, 0.3 * DX / c0, c0, steps, p0,
                extra={"centre": centre})


def faces2d(n: int = 256, steps: int = 1000) -> Case:
    """2D box with a real reflection coefficient per face, uniform in [-1, 1] from the seed: the disc of
    pstd2d in a 256^2 box, CFL 0.3.  1000 steps keep c0 t = 300 dx below 2L/c0 (510 dx), where the
    weighted sum of the 16 basic-wall solves is exact.  bcs holds the coefficients ((R_L, R_R) per axis)."""
    rng = rng_for(6)
    shape = (n, n)
    c0 = 1500.0
    centre = _centre(rng, shape, 9, DX)
    p0 = tapered_disc(shape, DX, centre, 4 * DX, 8 * DX)
    R = tuple(tuple(float(v) for v in rng.uniform(-1.0, 1.0, 2)) for _ in range(2))
    return Case("faces2d_%dx%d_R" % shape, shape, R, DX, 0.3 * DX / c0, c0, steps, p0, extra={"centre": centre})


def pstd3d(scale: float = 1.0, steps: int | None = None, shape=None) -> Case:
    rng = rng_for(2)
    faces = rng.integers(0, 2, size=6)
    if shape is None:
        n = max(int(round(384 * scale)), 20)
        shape = (n, n, n)
    bcs = tuple((int(faces[2 * a]), int(faces[2 * a + 1])) for a in range(3))
    c0 = 1540.0
    sigma = 4 * DX
    p0 = np.zeros(shape)
    blobs = []
    for _ in range(3):
        margin = min(24, min(shape) // 3)
        centre = _centre(rng, shape, margin, DX)
        amp = float(rng.uniform(0.5, 1.0))
        blobs.append((centre, amp))
        p0 += gaussian(shape, DX, centre, sigma, amp)
    st = 500 if steps is None else steps
    name = "pstd3d_%dx%dx%d_%s" % (shape + ("".join("ND"[b] for pair in bcs for b in pair),))
    return Case(name, tuple(shape), bcs, DX, 0.3 * DX / c0, c0, st, p0, precision="split_bf16",
                extra={"blobs": blobs, "sigma": sigma})


@dataclass
class BatchInstance:
    shape: tuple
    c0: float
    dt: float
    R: float
    p0: np.ndarray


def batched(count: int = 128, lo: int = 96, hi: int = 512, steps: int = 1000) -> dict:
    """Instances of the batched 2D workload (paired all-Neumann / all-Dirichlet solves)."""
    rng = rng_for(3)
    inst = []
    for _ in range(count):
        nx, ny = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        c0 = float(rng.uniform(1400.0, 1600.0))
        R = float(rng.uniform(-1.0, 1.0))
        centre = _centre(rng, (nx, ny), 24, DX)
        p0 = gaussian((nx, ny), DX, centre, 4 * DX)
        inst.append(BatchInstance((nx, ny), c0, 0.3 * DX / c0, R, p0))
    return {"instances": inst, "dx": DX, "steps": steps, "rho0": RHO0}


def smooth_c0_map(rng, shape, corr_nodes=16.0, lo=1400.0, hi=1600.0) -> np.ndarray:
    """White noise smoothed by a periodic Gaussian filter of width corr_nodes, min-max scaled to [lo, hi]."""
    noise = rng.standard_normal(shape)
    F = np.fft.fftn(noise)
    ks = np.meshgrid(*[np.fft.fftfreq(s) for s in shape], indexing="ij")
    k2 = sum(k ** 2 for k in ks)
    sm = np.real(np.fft.ifftn(F * np.exp(-2.0 * (np.pi * corr_nodes) ** 2 * k2)))
    sm = (sm - sm.min()) / (sm.max() - sm.min())
    return lo + (hi - lo) * sm


def nop_pairs(count: int, n: int = 128, index_offset: int = 0):
    """Inputs of surrogate training pairs: p0 blobs and c0 maps (targets come from the solver)."""
    out = []
    for i in range(count):
        rng = rng_for(4, stream=index_offset + i + 1)
        nb = int(rng.integers(1, 4))
        p0 = np.zeros((n, n))
        for _ in range(nb):
            sig = float(rng.uniform(3.0, 6.0)) * DX
            centre = _centre(rng, (n, n), min(20, n // 4), DX)
            p0 += gaussian((n, n), DX, centre, sig, float(rng.uniform(0.5, 1.0)))
        c0m = smooth_c0_map(rng, (n, n))
        out.append((p0, c0m))
    return out


def nop_init(shapes, seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """Initial surrogate parameters: for each (name, shape, fan_in), N(0, gain^2 / fan_in) entries for
    weight arrays and zeros for biases (fan_in 0); mixing matrices R* and W* get an extra 1/sqrt(2) since
    their two paths are summed.  Returns the flat float64 vector."""
    rng = np.random.default_rng(SEED_BASE + 4000 + seed)
    parts = []
    for name, shape, fan_in in shapes:
        n = int(np.prod(shape))
        if fan_in == 0:
            parts.append(np.zeros(n))
            continue
        g = gain / np.sqrt(fan_in)
        if name[0] in "RW":
            g /= np.sqrt(2.0)
        parts.append(g * rng.standard_normal(n))
    return np.concatenate(parts)


def nop_inputs(count: int, n: int = 128, index_offset: int = 0):
    """Arrays (p0s, c0s) of shape (count, n, n) for surrogate pairs, as nop_pairs draws them."""
    pairs = nop_pairs(count, n, index_offset)
    return np.stack([p for p, _ in pairs]), np.stack([c for _, c in pairs])


NOP_BCS = ((DIRICHLET, DIRICHLET), (NEUMANN, NEUMANN))
NOP_STEPS = 800
NOP_DT = 0.3 * DX / 1600.0


def pstd2d_large(n: int = 2049, steps: int = 200) -> Case:
    rng = rng_for(5)
    shape = (n, n)
    c0 = 1500.0
    centre = _centre(rng, shape, 9, DX)
    p0 = tapered_disc(shape, DX, centre, 4 * DX, 8 * DX)
    bcs = ((DIRICHLET, DIRICHLET), (NEUMANN, NEUMANN))
    return Case("pstd2d_%dx%d_xDD_yNN" % shape, shape, bcs, DX, 0.3 * DX / c0, c0, steps, p0,
                extra={"centre": centre})


def pstd3d_mode(n: int = 1025, steps: int = 50) -> Case:
    """Grid, faces and mode numbers; p0 is left to the caller (one basis function per axis)."""
    rng = rng_for(6)
    faces = rng.integers(0, 2, size=6)
    bcs = tuple((int(faces[2 * a]), int(faces[2 * a + 1])) for a in range(3))
    modes = tuple(int(m) for m in rng.integers(1, n // 8, size=3))
    c0 = 1540.0
    return Case("pstd3d_mode_%d^3" % n, (n, n, n), bcs, DX, 0.3 * DX / c0, c0, steps, None,
                extra={"modes": modes})


FFT_SIDES = (9, 17, 25, 33, 41, 49, 65, 81, 97, 121, 129, 161, 193, 241, 257)


def fft_small_case(seed: int, ndim: int, precision: str = "fp32", steps: int = 30, sides=FFT_SIDES) -> Case:
    """Random sides from ``sides`` (2(n-1) = 16 x 2^a 3^b 5^c), random faces, white-noise p0."""
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    limit = {1: len(sides), 2: len(sides), 3: 9}[ndim]
    shape = tuple(int(sides[i]) for i in rng.integers(0, limit, size=ndim))
    faces = rng.integers(0, 2, size=2 * ndim)
    bcs = tuple((int(faces[2 * a]), int(faces[2 * a + 1])) for a in range(ndim))
    c0 = float(rng.uniform(1400.0, 1600.0))
    cfl = 0.25 if ndim > 1 else 0.4
    p0 = rng.standard_normal(shape)
    return Case("fft%dd_%d" % (ndim, seed), shape, bcs, DX, cfl * DX / c0, c0, steps, p0, precision=precision)


def random_small_case(seed: int, ndim: int, max_n: int = 40, precision: str = "fp32", steps: int = 20) -> Case:
    """A small problem with random sizes and boundary faces, for parity sweeps."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    shape = tuple(int(v) for v in rng.integers(5, max_n + 1, size=ndim))
    faces = rng.integers(0, 2, size=2 * ndim)
    bcs = tuple((int(faces[2 * a]), int(faces[2 * a + 1])) for a in range(ndim))
    c0 = float(rng.uniform(1400.0, 1600.0))
    cfl = 0.25 if ndim > 1 else 0.4
    p0 = rng.standard_normal(shape)
    return Case("rand%dd_%d" % (ndim, seed), shape, bcs, DX, cfl * DX / c0, c0, steps, p0, precision=precision)
