"""Python binding of libpstd: plans, states and the combination calls (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import DIRICHLET, NEUMANN, PRECISIONS, PstdError, check, load

lib_path = _lib.LIB_PATH


def load_library():
    return load()


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _faces(bcs, ndim):
    if len(bcs) != ndim:
        raise ValueError("one (left, right) boundary pair per axis")
    arr = (C.c_int32 * 6)()
    for a, (l, r) in enumerate(bcs):
        arr[2 * a] = int(l)
        arr[2 * a + 1] = int(r)
    return arr


def axis_operator(n: int, bc_left: int, bc_right: int, dx: float, which: int) -> np.ndarray:
    """Unscaled FP64 operator of one axis as the library builds it (host only, no GPU needed)."""
    lib = load()
    shape = (n - 1, n) if which == 0 else (n, n - 1)
    out = np.zeros(shape, dtype=np.float64)
    check(lib.pstd_axis_operator(int(n), int(bc_left), int(bc_right), float(dx), int(which),
                                 out.ctypes.data_as(C.POINTER(C.c_double))), "pstd_axis_operator")
    return out


@dataclass
class State:
    """Device state (torch tensors): p and one velocity field per axis."""
    p: object
    u: list
    step: int = 0

    def _c(self):
        s = _lib.State()
        s.p = C.c_void_p(self.p.data_ptr())
        for a, t in enumerate(self.u):
            s.u[a] = C.c_void_p(t.data_ptr())
        s.step = self.step
        return s


class Plan:
    """A PSTD plan: grid, per-axis boundary pairs, constants, precision and stream (include/pstd.h)."""

    def __init__(self, shape, dx, dt, c0, bcs, rho0=1000.0, precision="fp32", c0_map=None, stream=None):
        torch = _torch()
        lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        if not 1 <= self.ndim <= 3:
            raise ValueError("1, 2 or 3 dimensions")
        self.bcs = tuple((int(l), int(r)) for l, r in bcs)
        self.precision = precision
        self.prec_code = PRECISIONS[precision]
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.dx, self.dt, self.c0, self.rho0 = float(dx), float(dt), float(c0), float(rho0)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self.c0_map = None
        cmap_ptr = None
        if c0_map is not None:
            cm = c0_map if isinstance(c0_map, torch.Tensor) else torch.as_tensor(np.asarray(c0_map))
            cm = cm.to(device=self.device, dtype=torch.float32).contiguous()
            if tuple(cm.shape) != self.shape:
                raise ValueError("c0_map must have the grid's shape")
            self.c0_map = cm  # kept alive for the plan's lifetime
            cmap_ptr = C.c_void_p(cm.data_ptr())
        g = _lib.Grid()
        g.ndim = self.ndim
        for a, n in enumerate(self.shape):
            g.n[a] = n
        h = C.c_void_p()
        check(lib.pstd_plan_create_ex(C.byref(g), self.dx, self.dt, self.c0, _faces(self.bcs, self.ndim),
                                      self.rho0, self.prec_code, cmap_ptr, _stream_handle(self._stream),
                                      C.byref(h)), "pstd_plan_create_ex")
        self._h = h

    # -- state -------------------------------------------------------------------------------------
    def u_shape(self, a):
        s = list(self.shape)
        s[a] -= 1
        return tuple(s)

    def new_state(self, p0) -> State:
        torch = _torch()
        p = torch.as_tensor(np.asarray(p0) if not isinstance(p0, torch.Tensor) else p0)
        p = p.to(device=self.device, dtype=self.dtype).contiguous().clone()
        if tuple(p.shape) != self.shape:
            raise ValueError("p0 has shape %s, plan expects %s" % (tuple(p.shape), self.shape))
        u = [torch.zeros(self.u_shape(a), device=self.device, dtype=self.dtype) for a in range(self.ndim)]
        return State(p, u, 0)

    def _check_state(self, st: State):
        torch = _torch()
        for t, shp in [(st.p, self.shape)] + [(st.u[a], self.u_shape(a)) for a in range(self.ndim)]:
            if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype:
                raise ValueError("state tensors must be %s on %s" % (self.dtype, self.device))
            if tuple(t.shape) != shp or not t.is_contiguous():
                raise ValueError("state tensor has shape %s (contiguous %s), expected %s"
                                 % (tuple(t.shape), t.is_contiguous(), shp))

    def init_state(self, st: State, u_mode: str = "centred") -> State:
        self._check_state(st)
        mode = {"centred": 0, "zero": 1, "keep": 2}[u_mode]
        cs = st._c()
        check(load().pstd_state_init(self._h, C.byref(cs), mode), "pstd_state_init")
        st.step = cs.step
        return st

    def step(self, st: State, n_steps: int) -> State:
        self._check_state(st)
        cs = st._c()
        check(load().pstd_step(self._h, C.byref(cs), int(n_steps)), "pstd_step")
        st.step = cs.step
        return st

    PATHS = {"auto": 0, "per_axis": 1, "fused": 2}

    def set_path(self, path: str) -> None:
        """Execution path of later steps: "auto", "per_axis" or "fused" (2D FP32: two kernels per step)."""
        check(load().pstd_plan_set_path(self._h, self.PATHS[path]), "pstd_plan_set_path")

    def apply_axis(self, st: State, axis: int, which: int) -> None:
        """One velocity (which=0) or pressure (which=1) update along one axis: a single kernel launch."""
        cs = st._c()
        check(load().pstd_apply_axis(self._h, C.byref(cs), int(axis), int(which)), "pstd_apply_axis")

    def check_finite(self, st: State) -> bool:
        self._check_state(st)
        cs = st._c()
        r = load().pstd_check_finite(self._h, C.byref(cs))
        if r == _lib.E_NONFINITE:
            return False
        check(r, "pstd_check_finite")
        return True

    def operator(self, axis: int, which: int) -> np.ndarray:
        n = self.shape[axis]
        shape = (n - 1, n) if which == 0 else (n, n - 1)
        out = np.zeros(shape, dtype=np.float64)
        check(load().pstd_plan_get_operator(self._h, axis, which, out.ctypes.data_as(C.POINTER(C.c_double))),
              "pstd_plan_get_operator")
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().pstd_plan_destroy(self._h)
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


def combine_R(p_dirichlet, p_neumann, R: float, out=None, stream=None):
    """out = (1+R)/2 p_neumann + (1-R)/2 p_dirichlet on the device (float32 tensors of equal size)."""
    torch = _torch()
    for t in (p_dirichlet, p_neumann):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError("combine_R takes contiguous float32 device tensors")
    if p_dirichlet.numel() != p_neumann.numel():
        raise ValueError("fields differ in size")
    if out is None:
        out = torch.empty_like(p_neumann)
    check(load().pstd_combine_R(C.c_void_p(p_dirichlet.data_ptr()), C.c_void_p(p_neumann.data_ptr()), float(R),
                                C.c_void_p(out.data_ptr()), p_neumann.numel(), _stream_handle(stream)),
          "pstd_combine_R")
    return out


def combine_fields(fields, weights, out=None, stream=None):
    """out = sum_i weights[i] * fields[i] on the device (§5's weighted sum of basic fields)."""
    torch = _torch()
    n = len(fields)
    if n != len(weights) or n < 1:
        raise ValueError("one weight per field")
    for t in fields:
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != fields[0].numel():
            raise ValueError("fields must be contiguous float32 tensors of equal size")
    if out is None:
        out = torch.empty_like(fields[0])
    ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in fields])
    w = (C.c_double * n)(*[float(x) for x in weights])
    check(load().pstd_combine_fields(ptrs, w, n, C.c_void_p(out.data_ptr()), fields[0].numel(),
                                     _stream_handle(stream)), "pstd_combine_fields")
    return out
