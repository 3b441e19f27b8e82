"""Binding of the DCT-basis neural-operator surrogate (include/pstd.h, pstd_nop_*): argument marshalling,
plus the host-side orchestration around it (training loop, target generation through the batched solver,
the input gate and the solver fallback).  Every contraction and update runs in libpstd's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import NopConfig, check, load
from .pstd import Batch, _stream_handle, _torch


@dataclass(frozen=True)
class SurrogateConfig:
    H: int = 128
    W: int = 128
    channels: int = 32
    modes: int = 48
    layers: int = 4
    hidden: int = 128


def param_shapes(cfg: SurrogateConfig):
    """(name, shape, fan_in) of the flat parameter vector, in the order pstd_nop_set_params expects."""
    C_, B2 = cfg.channels, cfg.modes // 2
    out = [("P", (C_, 4), 4), ("pb", (C_,), 0)]
    for l in range(cfg.layers):
        out += [("R%d" % l, (B2, B2, C_, C_), C_), ("W%d" % l, (C_, C_), C_), ("b%d" % l, (C_,), 0)]
    out += [("Q1", (cfg.hidden, C_), C_), ("q1b", (cfg.hidden,), 0), ("Q2", (cfg.hidden,), cfg.hidden),
            ("q2b", (1,), 0)]
    return out


class Surrogate:
    """The network of include/pstd.h on the current torch device and stream."""

    def __init__(self, cfg: SurrogateConfig = SurrogateConfig(), max_batch: int = 64, split: bool = False,
                 stream=None):
        torch = _torch()
        self.cfg = cfg
        self.max_batch = int(max_batch)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        c = NopConfig(cfg.H, cfg.W, cfg.channels, cfg.modes, cfg.layers, cfg.hidden, self.max_batch, int(bool(split)))
        h = C.c_void_p()
        check(load().pstd_nop_create(C.byref(c), _stream_handle(self._stream), C.byref(h)), "pstd_nop_create")
        self._h = h
        self.n_params = int(load().pstd_nop_param_count(h))
        self._out = None

    # -- parameters -----------------------------------------------------------------------------------
    def set_params(self, theta) -> None:
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        if a.size != self.n_params:
            raise ValueError("expected %d parameters, got %d" % (self.n_params, a.size))
        check(load().pstd_nop_set_params(self._h, a.ctypes.data_as(C.c_void_p), a.size), "pstd_nop_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, np.float32)
        check(load().pstd_nop_get_params(self._h, a.ctypes.data_as(C.c_void_p), a.size), "pstd_nop_get_params")
        return a

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.n_params, np.float32)
        check(load().pstd_nop_get_grads(self._h, a.ctypes.data_as(C.c_void_p), a.size), "pstd_nop_get_grads")
        return a

    # -- compute --------------------------------------------------------------------------------------
    def _dev(self, x):
        torch = _torch()
        t = torch.as_tensor(x).to(device=self.device, dtype=torch.float32).contiguous()
        if t.dim() != 3 or tuple(t.shape[1:]) != (self.cfg.H, self.cfg.W):
            raise ValueError("expected (batch, %d, %d), got %s" % (self.cfg.H, self.cfg.W, tuple(t.shape)))
        return t

    def forward(self, p0, c0, out=None):
        """out = network(p0, c0) for a batch (batch x H x W); keeps activations for backward()."""
        torch = _torch()
        p, cm = self._dev(p0), self._dev(c0)
        if p.shape != cm.shape:
            raise ValueError("p0 and c0 shapes differ")
        B = int(p.shape[0])
        if out is None:
            out = torch.empty_like(p)
        check(load().pstd_nop_forward(self._h, p.data_ptr(), cm.data_ptr(), out.data_ptr(), B), "pstd_nop_forward")
        self._keep = (p, cm)
        return out

    def infer(self, p0, c0, out=None):
        """out = network(p0, c0) without keeping activations (the inference form)."""
        torch = _torch()
        p, cm = self._dev(p0), self._dev(c0)
        if p.shape != cm.shape:
            raise ValueError("p0 and c0 shapes differ")
        B = int(p.shape[0])
        if out is None:
            out = torch.empty_like(p)
        check(load().pstd_nop_infer(self._h, p.data_ptr(), cm.data_ptr(), out.data_ptr(), B), "pstd_nop_infer")
        return out

    def backward(self, target) -> float:
        t = self._dev(target)
        loss = C.c_double()
        check(load().pstd_nop_backward(self._h, t.data_ptr(), C.byref(loss)), "pstd_nop_backward")
        return float(loss.value)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        check(load().pstd_nop_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)),
              "pstd_nop_adam_step")

    def relative_errors(self, pred, target) -> np.ndarray:
        p, t = self._dev(pred), self._dev(target)
        B = int(p.shape[0])
        err = np.empty(B, np.float64)
        check(load().pstd_nop_relative_errors(self._h, p.data_ptr(), t.data_ptr(), B,
                                              err.ctypes.data_as(C.c_void_p)), "pstd_nop_relative_errors")
        return err

    def close(self):
        if getattr(self, "_h", None):
            load().pstd_nop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def solver_targets(p0s, c0s, dx, dt, steps, bcs, batch=256):
    """p after `steps` PSTD steps of every (p0, c0 map) pair, through the batched solver in chunks of
    `batch` solves (FP32, centred start).  Returns a float32 device tensor (count x H x W)."""
    torch = _torch()
    p0s = torch.as_tensor(p0s)
    c0s = torch.as_tensor(c0s)
    n = int(p0s.shape[0])
    H, W = int(p0s.shape[1]), int(p0s.shape[2])
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    for s0 in range(0, n, batch):
        s1 = min(n, s0 + batch)
        cm = c0s[s0:s1].to(device=dev, dtype=torch.float32)
        cmax = cm.amax(dim=(1, 2)).double().cpu().numpy()
        solves = [{"shape": (H, W), "bcs": bcs, "dx": dx, "dt": dt, "c0": float(cmax[i])} for i in range(s1 - s0)]
        b = Batch(solves)
        try:
            b.set_c0_maps([cm[i] for i in range(s1 - s0)])
            st = b.new_states([p0s[i] for i in range(s0, s1)])
            b.init_states(st)
            b.step(st, steps)
            b.synchronize()
            for i in range(s1 - s0):
                out[s0 + i].copy_(st[i].p)
            torch.cuda.synchronize()
        finally:
            b.close()
    return out


def input_stats(net: Surrogate, p0, c0, margin: int = 10) -> np.ndarray:
    """(batch, 4): min c0, max c0, max |p0|, share of sum p0^2 within `margin` nodes of a wall."""
    p, cm = net._dev(p0), net._dev(c0)
    B = int(p.shape[0])
    out = np.empty((B, 4), np.float64)
    check(load().pstd_nop_input_stats(net._h, p.data_ptr(), cm.data_ptr(), B, int(margin),
                                      out.ctypes.data_as(C.c_void_p)), "pstd_nop_input_stats")
    return out


@dataclass(frozen=True)
class Gate:
    """When the surrogate may answer instead of the solver.

    validated_error: the surrogate's relative L2 error against the solver on held-out pairs (a high
    quantile); a request whose tolerance is below it always goes to the solver.  The remaining fields
    bound the training distribution: c0 range, peak |p0|, and the share of p0's energy near the walls
    (training sources sit at least 20 nodes inside).
    """
    validated_error: float
    c0_lo: float = 1400.0
    c0_hi: float = 1600.0
    p_max: float = 3.0
    wall_margin: int = 10
    wall_share_max: float = 1e-3


def predict(net: Surrogate, p0, c0, tol: float, gate: Gate, dx, dt, steps, bcs, rho0=1000.0):
    """Surrogate answer where the gate admits it, the FP32 PSTD solver's answer elsewhere
    (``pstd_nop_predict``: statistics, gate, inference and the batched fallback all run in the library).

    Returns (out, fallback) with fallback a boolean array marking the samples the solver produced."""
    torch = _torch()
    p, cm = net._dev(p0), net._dev(c0)
    B = int(p.shape[0])
    out = torch.empty_like(p)
    g = _lib.NopGate(float(gate.validated_error), float(gate.c0_lo), float(gate.c0_hi), float(gate.p_max),
                     int(gate.wall_margin), float(gate.wall_share_max))
    pr = _lib.NopProblem()
    pr.dx, pr.dt, pr.rho0, pr.steps = float(dx), float(dt), float(rho0), int(steps)
    faces = [int(f) for pair in bcs for f in pair]
    for i in range(4):
        pr.bc[i] = faces[i]
    fb = np.zeros(B, np.int32)
    nf = C.c_int32(0)
    check(load().pstd_nop_predict(net._h, C.byref(g), C.byref(pr), p.data_ptr(), cm.data_ptr(), out.data_ptr(), B,
                                  float(tol), fb.ctypes.data_as(C.c_void_p), C.byref(nf)), "pstd_nop_predict")
    return out, fb.astype(bool)
