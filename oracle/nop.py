"""FP64 reference of the DCT-basis neural operator that stands in for the solver at a fixed time.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not a method of the paper: the surrogate is an extension whose training data and error reference are the
PSTD solver of §4.  The network maps an initial pressure p0 and a sound-speed map c0 on an H x W grid to
the pressure after a fixed number of steps:

    features  f = [p0, (c0 - 1500)/100, x, y]            (4 channels; x, y in [0, 1] along each axis)
    lift      v = P f + pb                                (C channels, pointwise)
    layer l   v = GELU(W_l v + b_l + IDCT(R_l . DCT(v)))  (l = 0 .. layers-1)
    project   q = GELU(Q1 v + q1b),  out = Q2 q + q2b     (hidden width Hp, one output channel)

DCT is the orthonormal DCT-II along both axes truncated to the Mm lowest modes per axis; IDCT is its
transpose (the orthonormal DCT-III restricted to those modes).  R_l mixes channels per mode with one
C x C matrix shared by each 2 x 2 block of modes.  GELU is x Phi(x) with the exact normal CDF.  The loss
is the batch mean of |out - target|^2 / |target|^2.

Everything is written out with plain NumPy contractions in float64; backward() is the hand-derived
gradient of the loss, pinned against central finite differences in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import erf, sqrt

import numpy as np


@dataclass(frozen=True)
class Config:
    H: int = 128
    W: int = 128
    C: int = 32          # channels
    Mm: int = 48         # retained modes per axis (even: modes are mixed in 2 x 2 blocks)
    layers: int = 4
    Hp: int = 128        # hidden width of the projection


def param_shapes(cfg: Config):
    """Ordered (name, shape) list of the flat parameter vector."""
    C, B2 = cfg.C, cfg.Mm // 2
    out = [("P", (C, 4)), ("pb", (C,))]
    for l in range(cfg.layers):
        out += [("R%d" % l, (B2, B2, C, C)), ("W%d" % l, (C, C)), ("b%d" % l, (C,))]
    out += [("Q1", (cfg.Hp, C)), ("q1b", (cfg.Hp,)), ("Q2", (cfg.Hp,)), ("q2b", (1,))]
    return out


def param_count(cfg: Config) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(cfg)))


def unflatten(cfg: Config, theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in param_shapes(cfg):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def flatten(cfg: Config, d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in param_shapes(cfg)])


def dct_matrix(n: int, m: int) -> np.ndarray:
    """First m rows of the orthonormal DCT-II of length n: C[k, j] = s_k cos(pi k (2j+1) / (2n))."""
    k = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    s = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
    return s * np.cos(np.pi * k * (2 * j + 1) / (2 * n))


def gelu(x):
    return x * 0.5 * (1.0 + np.vectorize(erf)(x / sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / sqrt(2.0 * np.pi)
    return 0.5 * (1.0 + np.vectorize(erf)(x / sqrt(2.0))) + x * phi


def features(cfg: Config, p0: np.ndarray, c0: np.ndarray) -> np.ndarray:
    """(B, 4, H, W): p0, normalised c0 and the two coordinates."""
    B = p0.shape[0]
    x = np.broadcast_to(np.linspace(0.0, 1.0, cfg.H)[:, None], (cfg.H, cfg.W))
    y = np.broadcast_to(np.linspace(0.0, 1.0, cfg.W)[None, :], (cfg.H, cfg.W))
    f = np.empty((B, 4, cfg.H, cfg.W))
    f[:, 0] = p0
    f[:, 1] = (c0 - 1500.0) / 100.0
    f[:, 2] = x
    f[:, 3] = y
    return f


def _expand_R(cfg: Config, R: np.ndarray) -> np.ndarray:
    """(Mm, Mm, C, C): the block-shared mixing matrix of every mode."""
    return np.repeat(np.repeat(R, 2, axis=0), 2, axis=1)


def spectral(cfg: Config, R: np.ndarray, v: np.ndarray) -> np.ndarray:
    """IDCT(R . DCT(v)) for v of shape (B, C, H, W)."""
    Ch, Cw = dct_matrix(cfg.H, cfg.Mm), dct_matrix(cfg.W, cfg.Mm)
    a = np.einsum("kh,bchw,lw->bckl", Ch, v, Cw)                  # DCT along both axes, truncated
    z = np.einsum("klij,bjkl->bikl", _expand_R(cfg, R), a)        # z[b, o, k, l] = sum_i R[k, l, o, i] a[b, i, k, l]
    return np.einsum("kh,bokl,lw->bohw", Ch, z, Cw)               # IDCT (transpose of the truncated DCT)


def forward(cfg: Config, theta: np.ndarray, p0: np.ndarray, c0: np.ndarray, keep: bool = False):
    """out (B, H, W), and the saved activations when keep is set."""
    prm = unflatten(cfg, theta)
    f = features(cfg, p0, c0)
    v = np.einsum("oi,bihw->bohw", prm["P"], f) + prm["pb"][None, :, None, None]
    saved = {"f": f, "v": [v]}
    saved["pre"] = []
    for l in range(cfg.layers):
        pre = (np.einsum("oi,bihw->bohw", prm["W%d" % l], v) + prm["b%d" % l][None, :, None, None]
               + spectral(cfg, prm["R%d" % l], v))
        v = gelu(pre)
        saved["pre"].append(pre)
        saved["v"].append(v)
    qpre = np.einsum("jc,bchw->bjhw", prm["Q1"], v) + prm["q1b"][None, :, None, None]
    q = gelu(qpre)
    out = np.einsum("j,bjhw->bhw", prm["Q2"], q) + prm["q2b"][0]
    saved.update(qpre=qpre, q=q)
    return (out, saved) if keep else out


def loss(out: np.ndarray, target: np.ndarray) -> float:
    """Mean over the batch of |out - target|^2 / |target|^2."""
    num = np.sum((out - target) ** 2, axis=(1, 2))
    den = np.sum(target ** 2, axis=(1, 2))
    return float(np.mean(num / den))


def backward(cfg: Config, theta: np.ndarray, p0: np.ndarray, c0: np.ndarray, target: np.ndarray):
    """(loss, gradient of the loss with respect to theta), by the chain rule through forward()."""
    prm = unflatten(cfg, theta)
    out, sv = forward(cfg, theta, p0, c0, keep=True)
    B = out.shape[0]
    den = np.sum(target ** 2, axis=(1, 2))
    L = float(np.mean(np.sum((out - target) ** 2, axis=(1, 2)) / den))
    g = {}
    dout = 2.0 * (out - target) / (den[:, None, None] * B)
    g["q2b"] = np.array([dout.sum()])
    g["Q2"] = np.einsum("bhw,bjhw->j", dout, sv["q"])
    dq = np.einsum("j,bhw->bjhw", prm["Q2"], dout) * gelu_grad(sv["qpre"])
    g["q1b"] = dq.sum(axis=(0, 2, 3))
    v = sv["v"][-1]
    g["Q1"] = np.einsum("bjhw,bchw->jc", dq, v)
    dv = np.einsum("jc,bjhw->bchw", prm["Q1"], dq)
    Ch, Cw = dct_matrix(cfg.H, cfg.Mm), dct_matrix(cfg.W, cfg.Mm)
    for l in reversed(range(cfg.layers)):
        vin = sv["v"][l]
        dpre = dv * gelu_grad(sv["pre"][l])
        g["b%d" % l] = dpre.sum(axis=(0, 2, 3))
        g["W%d" % l] = np.einsum("bohw,bihw->oi", dpre, vin)
        dv = np.einsum("oi,bohw->bihw", prm["W%d" % l], dpre)
        # spectral path: spec = Ch^T z Cw with z = R . a, a = Ch v Cw^T
        dz = np.einsum("kh,bohw,lw->bokl", Ch, dpre, Cw)
        a = np.einsum("kh,bchw,lw->bckl", Ch, vin, Cw)
        dRfull = np.einsum("bokl,bikl->kloi", dz, a)
        g["R%d" % l] = dRfull.reshape(cfg.Mm // 2, 2, cfg.Mm // 2, 2, cfg.C, cfg.C).sum(axis=(1, 3))
        da = np.einsum("klij,bikl->bjkl", _expand_R(cfg, prm["R%d" % l]), dz)
        dv = dv + np.einsum("kh,bckl,lw->bchw", Ch, da, Cw)
    g["pb"] = dv.sum(axis=(0, 2, 3))
    g["P"] = np.einsum("bohw,bihw->oi", dv, sv["f"])
    return L, flatten(cfg, g)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
