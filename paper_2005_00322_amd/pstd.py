"""Python binding of libpstd: plans, states and the combination calls (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import DIRICHLET, DIRICHLET_HALF, NEUMANN, NEUMANN_HALF, PERIODIC, PRECISIONS, PstdError, check, load

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


# Collocated differentiation and half-step interpolation operators (pstd_apply_axis_operator)
GRAD_NODES, GRAD_STAG, NODES_TO_STAG, STAG_TO_NODES = 2, 3, 4, 5


def operator_shape(n: int, m: int, which: int) -> tuple:
    """(rows, cols) of operator `which` of an axis with n nodes and m staggered points."""
    return {0: (m, n), 1: (n, m), GRAD_NODES: (n, n), GRAD_STAG: (m, m), NODES_TO_STAG: (m, n),
            STAG_TO_NODES: (n, m)}[which]


def axis_operator(n: int, bc_left: int, bc_right: int, dx: float, which: int) -> np.ndarray:
    """FP64 operator of one axis as the library builds it (host only, no GPU needed): 0 / 1 the
    unscaled velocity / pressure operators, 2..5 the collocated derivatives and interpolations."""
    lib = load()
    m = n if (int(bc_left) == PERIODIC or int(bc_right) in (NEUMANN_HALF, DIRICHLET_HALF)) else n - 1
    shape = operator_shape(n, m, which) if which in range(6) else (1, 1)   # the library rejects others
    out = np.zeros(shape, dtype=np.float64)
    check(lib.pstd_axis_operator(int(n), int(bc_left), int(bc_right), float(dx), int(which),
                                 out.ctypes.data_as(C.POINTER(C.c_double))), "pstd_axis_operator")
    return out


def axis_operator_structure(n: int, bc_left: int, bc_right: int, dx: float, which: int):
    """Toeplitz-plus-Hankel form of axis_operator(...) as the library finds it (host only):
    (f, g, w, residual) with A[r][c] = wr[r] wc[c] (f[r - c + C - 1] + g[r + c]), w = (wr[0], wr[-1],
    wc[0], wc[-1]) and every other weight one.  Raises if the operator has no such form."""
    lib = load()
    m = n if (int(bc_left) == PERIODIC or int(bc_right) in (NEUMANN_HALF, DIRICHLET_HALF)) else n - 1
    rows, cols = operator_shape(n, m, which) if which in range(6) else (1, 1)
    f = np.zeros(rows + cols - 1)
    g = np.zeros(rows + cols - 1)
    w = np.zeros(4)
    r = C.c_double(0.0)
    P = C.POINTER(C.c_double)
    check(lib.pstd_axis_operator_structure(int(n), int(bc_left), int(bc_right), float(dx), int(which),
                                           f.ctypes.data_as(P), g.ctypes.data_as(P), w.ctypes.data_as(P),
                                           C.byref(r)), "pstd_axis_operator_structure")
    return f, g, w, r.value


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
        """n - 1 staggered points between walls on nodes, n along a periodic axis or one whose right wall
        lies half a step beyond the last node."""
        s = list(self.shape)
        if int(self.bcs[a][0]) != PERIODIC and int(self.bcs[a][1]) not in (NEUMANN_HALF, DIRICHLET_HALF):
            s[a] -= 1
        return tuple(s)

    def new_state(self, p0=None) -> State:
        """Device state with p = p0 (zeros if None) and u = 0."""
        torch = _torch()
        if p0 is None:
            p = torch.zeros(self.shape, device=self.device, dtype=self.dtype)
        else:
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

    def prepare(self, st: State, n_steps: int) -> None:
        """Capture, without running them, the step graphs a later step(st, n_steps) replays."""
        self._check_state(st)
        cs = st._c()
        check(load().pstd_step_prepare(self._h, C.byref(cs), int(n_steps)), "pstd_step_prepare")

    PATHS = {"auto": 0, "per_axis": 1, "fused": 2, "fft": 3, "stored": 4, "fft_generic": 5}

    def set_path(self, path: str) -> None:
        """Execution path of later steps: "auto", "per_axis" (dense contractions), "fused" (2D FP32: two
        kernels per step), "fft" (LDS-resident FFTs on every axis whose 2(n-1) is 16 x 2^a 3^b 5^c),
        "fft_generic" (fft with every axis on the mixed-radix kernel, also where an FP32 power-of-two
        length has its own) or "stored" (per_axis with split-bf16 operators read from memory rather than
        formed from their Toeplitz and Hankel parts)."""
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

    def apply_operator(self, axis: int, which: int, x, out=None):
        """out = A x along `axis` on the GPU, A one of GRAD_NODES, GRAD_STAG, NODES_TO_STAG, STAG_TO_NODES:
        x has the plan's extents on the other axes and A's column count on `axis` (e.g. STAG_TO_NODES
        along a maps u[a] onto the p grid)."""
        import torch
        n = self.shape[axis]
        rows, cols = operator_shape(n, n - 1, which)
        in_shape = list(self.shape)
        in_shape[axis] = cols
        out_shape = list(self.shape)
        out_shape[axis] = rows
        if (not isinstance(x, torch.Tensor) or tuple(x.shape) != tuple(in_shape) or x.dtype != self.dtype
                or x.device != self.device or not x.is_contiguous()):
            raise ValueError("x must be a contiguous %s tensor of shape %s on %s" % (self.dtype, tuple(in_shape),
                                                                                    self.device))
        if out is None:
            out = torch.empty(out_shape, device=self.device, dtype=self.dtype)
        elif (tuple(out.shape) != tuple(out_shape) or out.dtype != self.dtype or out.device != self.device
              or not out.is_contiguous()):
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (self.dtype, tuple(out_shape)))
        check(load().pstd_apply_axis_operator(self._h, int(axis), int(which), C.c_void_p(x.data_ptr()),
                                              C.c_void_p(out.data_ptr())), "pstd_apply_axis_operator")
        return out

    def operator(self, axis: int, which: int) -> np.ndarray:
        n, m = self.shape[axis], self.u_shape(axis)[axis]
        shape = (m, n) if which == 0 else (n, m)
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


def face_weights(R_faces):
    """Basic fields and weights of §5 for per-face reflection coefficients (pstd_face_weights, host only).

    R_faces: one (R_left, R_right) pair per axis.  Returns (cases, weights): cases[f] is the tuple of
    ((left, right), ...) wall pairs of basic field f, weights[f] its weight (float64 array).
    """
    nd = len(R_faces)
    nf = 4 ** nd
    r = (C.c_double * (2 * nd))(*[float(x) for pair in R_faces for x in pair])
    bc = (C.c_int32 * (2 * nd * nf))()
    w = (C.c_double * nf)()
    check(load().pstd_face_weights(nd, r, bc, w), "pstd_face_weights")
    cases = [tuple((int(bc[f * 2 * nd + 2 * a]), int(bc[f * 2 * nd + 2 * a + 1])) for a in range(nd)) for f in range(nf)]
    return cases, np.array(list(w), dtype=np.float64)


def solve_faces_2d(shape, dx, dt, c0, R_faces, p0, n_steps, rho0=1000.0, batch=None, out=None):
    """The 2D field for per-face reflection coefficients: the 16 basic-wall solves of the same problem in one
    batched launch (pstd_batch_*), then their weighted sum (pstd_combine_fields) with pstd_face_weights.

    Returns (p, batch, states); pass the returned batch back to reuse it (same shape and constants).
    """
    cases, w = face_weights(R_faces)
    if batch is None:
        batch = Batch([{"shape": tuple(shape), "bcs": cs, "dx": dx, "dt": dt, "c0": c0} for cs in cases], rho0=rho0)
        if max(shape) <= 512:
            batch.set_config(tile=16)     # one shape: two fused phase launches per step over all 16 solves
    states = batch.new_states([p0] * len(cases))
    batch.init_states(states)
    batch.step(states, n_steps)
    p = combine_fields([st.p for st in states], w, out=out, stream=batch._stream)
    return p, batch, states


def solve_faces(shape, dx, dt, c0, R_faces, p0, n_steps, rho0=1000.0, precision="fp32", stream=None, out=None):
    """The field for per-face reflection coefficients in 1D, 2D or 3D (§5): the 4^d basic-wall solves of the
    same problem, one plan each on one stream, then their weighted sum (pstd_combine_fields) with the
    weights of pstd_face_weights.  For many 2D solves of one shape ``solve_faces_2d`` runs them as one batch.

    Returns p (float32, the plans' precision must be fp32 or split_bf16).
    """
    torch = _torch()
    if precision not in ("fp32", "split_bf16"):
        raise ValueError("the weighted sum runs on float32 fields")
    cases, w = face_weights(R_faces)
    s = torch.cuda.Stream() if stream is None else stream
    fields = []
    for cs in cases:
        with Plan(shape, dx, dt, c0, cs, rho0=rho0, precision=precision, stream=s) as pl:
            st = pl.new_state(p0)
            pl.init_state(st)
            pl.step(st, n_steps)
            fields.append(st.p)
            s.synchronize()
    return combine_fields(fields, w, out=out, stream=s)


class Batch:
    """Many independent 2D FP32 solves stepped by one persistent launch (include/pstd.h, pstd_batch_*).

    solves: list of dicts with keys shape (nx, ny), bcs ((l, r), (l, r)), dx, dt, c0.
    """

    def __init__(self, solves, rho0=1000.0, stream=None):
        torch = _torch()
        lib = load()
        self.solves = [dict(s) for s in solves]
        self.count = len(self.solves)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        n = (C.c_int64 * (2 * self.count))()
        bc = (C.c_int32 * (4 * self.count))()
        dx = (C.c_double * self.count)()
        dt = (C.c_double * self.count)()
        c0 = (C.c_double * self.count)()
        for i, s in enumerate(self.solves):
            n[2 * i], n[2 * i + 1] = int(s["shape"][0]), int(s["shape"][1])
            (bl, br), (bd, bu) = s["bcs"]
            bc[4 * i:4 * i + 4] = [int(bl), int(br), int(bd), int(bu)]
            dx[i], dt[i], c0[i] = float(s["dx"]), float(s["dt"]), float(s["c0"])
        h = C.c_void_p()
        check(lib.pstd_batch_create(self.count, n, bc, dx, dt, c0, float(rho0), _stream_handle(self._stream),
                                    C.byref(h)), "pstd_batch_create")
        self._h = h

    def new_states(self, p0s):
        torch = _torch()
        out = []
        for s, p0 in zip(self.solves, p0s):
            nx, ny = s["shape"]
            p = p0 if isinstance(p0, torch.Tensor) else torch.as_tensor(np.asarray(p0))
            p = p.to(device=self.device, dtype=torch.float32).contiguous().clone()
            if tuple(p.shape) != (nx, ny):
                raise ValueError("p0 shape mismatch")
            ux = torch.zeros((nx - 1, ny), device=self.device, dtype=torch.float32)
            uy = torch.zeros((nx, ny - 1), device=self.device, dtype=torch.float32)
            out.append(State(p, [ux, uy], 0))
        return out

    def _c_states(self, states):
        arr = (_lib.State * self.count)()
        for i, st in enumerate(states):
            arr[i] = st._c()
        return arr

    def init_states(self, states, u_mode="centred"):
        arr = self._c_states(states)
        check(load().pstd_batch_state_init(self._h, arr, {"centred": 0, "zero": 1, "keep": 2}[u_mode]),
              "pstd_batch_state_init")
        for st in states:
            st.step = 0

    def step(self, states, n_steps):
        arr = self._c_states(states)
        check(load().pstd_batch_step(self._h, arr, int(n_steps)), "pstd_batch_step")
        for st in states:
            st.step += int(n_steps)

    def combine_R(self, states, pairs, R, outs=None):
        """outs[i] = (1+R[i])/2 p_N + (1-R[i])/2 p_D for pairs (dirichlet index, neumann index)."""
        torch = _torch()
        npairs = len(pairs)
        if outs is None:
            outs = [torch.empty_like(states[d].p) for d, _ in pairs]
        pr = (C.c_int32 * (2 * npairs))(*[int(x) for pair in pairs for x in pair])
        rr = (C.c_double * npairs)(*[float(x) for x in R])
        op = (C.c_void_p * npairs)(*[t.data_ptr() for t in outs])
        check(load().pstd_batch_combine_R(self._h, self._c_states(states), pr, rr, op, npairs), "pstd_batch_combine_R")
        return outs

    def set_c0_maps(self, maps):
        """Per-solve sound-speed maps (float32 device tensors of the solve's shape, or None): the pressure
        update of those solves uses c0(x)^2 pointwise.  The solve's c0 given at creation must be the
        map's maximum (it sets the stability check)."""
        torch = _torch()
        keep = []
        ptrs = (C.c_void_p * self.count)()
        for i, (s, m) in enumerate(zip(self.solves, maps)):
            if m is None:
                continue
            t = torch.as_tensor(m).to(device=self.device, dtype=torch.float32).contiguous()
            if tuple(t.shape) != tuple(s["shape"]):
                raise ValueError("c0 map %d has shape %s, solve is %s" % (i, tuple(t.shape), s["shape"]))
            keep.append(t)
            ptrs[i] = t.data_ptr()
        check(load().pstd_batch_set_c0_maps(self._h, ptrs), "pstd_batch_set_c0_maps")
        self._stream.synchronize()   # the maps are squared into the batch's own buffers
        del keep

    def synchronize(self):
        """Wait for the batch's work; raises if a grid barrier of the persistent launch timed out."""
        check(load().pstd_batch_synchronize(self._h), "pstd_batch_synchronize")

    def set_config(self, blocks=0, order=0, tile=32):
        check(load().pstd_batch_set_config(self._h, int(blocks), int(order), int(tile)), "pstd_batch_set_config")

    def autotune(self, trial_steps=5, cache_path=None):
        cfg = (C.c_int32 * 4)()
        check(load().pstd_batch_autotune(self._h, int(trial_steps),
                                         cache_path.encode() if cache_path else None, cfg), "pstd_batch_autotune")
        return {"blocks": cfg[0], "order": cfg[1], "tile": cfg[2], "from_cache": bool(cfg[3])}

    def close(self):
        if getattr(self, "_h", None):
            load().pstd_batch_destroy(self._h)
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
