"""Pins of the FP64 surrogate reference (CPU only).

* The truncated DCT is the orthonormal DCT-II of scipy.fft (an independent implementation); with all
  modes kept it is orthogonal, and the spectral layer with identity mixing is the identity map.
* GELU and its derivative agree with torch's exact-erf GELU and with finite differences.
* backward() agrees with central finite differences of loss() for every parameter group (a dropped
  term, a transposed operand or a wrong sign in any of them shows up here).
* adam_step() agrees with torch.optim.Adam.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import nop

TINY = nop.Config(H=8, W=6, C=3, Mm=4, layers=2, Hp=5)


def _inputs(cfg, B, seed):
    rng = np.random.default_rng(seed)
    p0 = rng.standard_normal((B, cfg.H, cfg.W))
    c0 = 1400.0 + 200.0 * rng.random((B, cfg.H, cfg.W))
    tgt = rng.standard_normal((B, cfg.H, cfg.W))
    theta = 0.3 * rng.standard_normal(nop.param_count(cfg))
    return theta, p0, c0, tgt


def test_default_config_size():
    assert nop.param_count(nop.Config()) == 2368033


@pytest.mark.parametrize("n,m", [(8, 8), (8, 5), (128, 48)])
def test_dct_matrix_is_scipy_orthonormal_dct2(n, m):
    x = np.random.default_rng(n).standard_normal(n)
    ref = scipy.fft.dct(x, type=2, norm="ortho")[:m]
    assert np.allclose(nop.dct_matrix(n, m) @ x, ref, atol=1e-12)


def test_full_dct_is_orthogonal_and_identity_mixing_is_identity():
    C = nop.dct_matrix(10, 10)
    assert np.allclose(C @ C.T, np.eye(10), atol=1e-13)
    cfg = nop.Config(H=6, W=6, C=2, Mm=6, layers=1, Hp=2)
    R = np.zeros((3, 3, 2, 2))
    R[..., 0, 0] = R[..., 1, 1] = 1.0
    v = np.random.default_rng(1).standard_normal((2, 2, 6, 6))
    assert np.allclose(nop.spectral(cfg, R, v), v, atol=1e-12)


def test_gelu_against_torch_and_finite_differences():
    import torch
    x = np.linspace(-5, 5, 101)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    assert np.allclose(nop.gelu(x), ref, atol=1e-14)
    h = 1e-6
    fd = (nop.gelu(x + h) - nop.gelu(x - h)) / (2 * h)
    assert np.allclose(nop.gelu_grad(x), fd, atol=1e-8)


def test_backward_matches_finite_differences():
    cfg = TINY
    theta, p0, c0, tgt = _inputs(cfg, 2, 3)
    L, g = nop.backward(cfg, theta, p0, c0, tgt)
    assert abs(L - nop.loss(nop.forward(cfg, theta, p0, c0), tgt)) < 1e-14
    rng = np.random.default_rng(4)
    offsets, o = {}, 0
    for name, shp in nop.param_shapes(cfg):
        n = int(np.prod(shp))
        offsets[name] = (o, n)
        o += n
    h = 1e-6
    for name, (o, n) in offsets.items():
        for idx in rng.choice(n, size=min(n, 4), replace=False):
            e = np.zeros_like(theta)
            e[o + idx] = h
            fd = (nop.loss(nop.forward(cfg, theta + e, p0, c0), tgt)
                  - nop.loss(nop.forward(cfg, theta - e, p0, c0), tgt)) / (2 * h)
            assert abs(fd - g[o + idx]) < 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[o + idx])


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(7)
    t_ref = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([t_ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(7)
    v = np.zeros(7)
    th = theta.copy()
    for t in range(1, 6):
        g = rng.standard_normal(7)
        th, m, v = nop.adam_step(th, g, m, v, t, 1e-2)
        opt.zero_grad()
        t_ref.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.allclose(th, t_ref.detach().numpy(), atol=1e-12)
