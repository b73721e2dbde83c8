"""Thin Python binding of the C ABI in ``include/pat.h`` (``libpat.so``).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Arrays are torch tensors on the GPU (float32, contiguous); the work
is enqueued on torch's current stream.  Importing this module never falls back
to anything: if the library is missing, the first call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpat.so")

PAT_OK, PAT_EINVAL, PAT_EUNSUPPORTED, PAT_EWORKSPACE, PAT_EHIP, PAT_ENONFINITE = 0, -1, -2, -3, -4, -5

EXPORTS = (
    "pat_plan_create", "pat_plan_destroy", "pat_workspace_size", "pat_forward", "pat_history_field", "pat_misfit",
    "pat_free_part", "pat_axpby", "pat_mul", "pat_absmax",
    "pat_adjoint_gradient", "pat_project_update", "pat_prolong", "pat_prolong_phys", "pat_time_interp",
    "pat_lbfgs_scratch_bytes", "pat_lbfgs_direction", "pat_lbfgs_direction_noalloc", "pat_dot", "pat_status_string",
    "pat_trace_start", "pat_trace_stop", "pat_trace_read", "pat_plan_set_tile", "pat_plan_set_col_order",
    "pat_batch_gradient",
    "pat_batch_release",
    "pat_ou_create", "pat_ou_destroy", "pat_ou_scratch_bytes", "pat_ou_apply", "pat_ou_prior",
)

LBFGS_NOALLOC_MAX_PAIRS = 64

PASS_KINDS = ("fwd_col_grad", "fwd_row_u", "fwd_col_div", "fwd_row_rho",
              "adj_col_summ", "adj_row_rho", "adj_col_grad", "adj_row_u")


class PatError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class pat_problem(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("plan", "c", "p0", "y", "w", "data", "resid", "J", "g_p0", "g_c", "ws")] + \
        [("ws_bytes", ctypes.c_size_t)]


class pat_grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nt", ctypes.c_int32), ("pml", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("c_ref", ctypes.c_double),
        ("rho0", ctypes.c_double), ("pml_alpha", ctypes.c_double),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libpat.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2505_08482_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                  ctypes.c_double, ctypes.c_size_t)
    L.pat_plan_create.argtypes = [ctypes.POINTER(pat_grid), i32, i32, vp, ctypes.POINTER(vp)]
    L.pat_plan_destroy.argtypes = [vp]
    L.pat_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.pat_forward.argtypes = [vp, vp, vp, vp, vp, sz, i32, i32, vp]
    L.pat_history_field.argtypes = [vp, vp, i32, ctypes.POINTER(vp)]
    L.pat_misfit.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pat_adjoint_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.pat_project_update.argtypes = [i64, vp, vp, f32, vp, vp, f32, f32, vp]
    L.pat_prolong.argtypes = [i32, vp, i32, i32, vp, i32, i32, vp]
    L.pat_prolong_phys.argtypes = [i32, vp, i32, i32, ctypes.c_double, vp, i32, i32, ctypes.c_double, vp]
    L.pat_time_interp.argtypes = [i32, i32, i32, vp, f64, vp, i32, f64, vp]
    L.pat_lbfgs_scratch_bytes.argtypes = [i32]
    L.pat_lbfgs_scratch_bytes.restype = sz
    L.pat_lbfgs_direction.argtypes = [i64, vp, i32, vp, vp, vp, vp, vp]
    L.pat_lbfgs_direction_noalloc.argtypes = [i64, vp, i32, vp, vp, vp, vp]
    L.pat_dot.argtypes = [i64, vp, vp, vp, vp, vp]
    L.pat_absmax.argtypes = [i64, vp, vp, vp, vp]
    L.pat_free_part.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    L.pat_axpby.argtypes = [i64, f32, vp, f32, vp, vp, vp]
    L.pat_mul.argtypes = [i64, vp, vp, vp, vp]
    L.pat_trace_start.argtypes = [i32]
    L.pat_trace_stop.argtypes = []
    L.pat_trace_read.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(f64)]
    L.pat_plan_set_tile.argtypes = [vp, i32]
    L.pat_plan_set_col_order.argtypes = [vp, i32]
    L.pat_batch_gradient.argtypes = [i32, vp, i32, vp]
    L.pat_batch_release.argtypes = []
    L.pat_ou_create.argtypes = [i32, i32, f64, f64, vp, ctypes.POINTER(vp)]
    L.pat_ou_destroy.argtypes = [vp]
    L.pat_ou_scratch_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.pat_ou_apply.argtypes = [vp, i32, vp, vp, vp, sz, vp]
    L.pat_ou_prior.argtypes = [vp, i32, vp, vp, vp, vp, vp, f64, i32, vp, sz, ctypes.POINTER(i32), vp]
    L.pat_status_string.argtypes = [ctypes.c_int]
    L.pat_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("pat_lbfgs_scratch_bytes", "pat_status_string"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().pat_status_string(int(status)).decode()


def _check(status: int, what: str) -> None:
    if status != PAT_OK:
        raise PatError(status, what)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _f32(t, n: Optional[int] = None, name: str = "array"):
    import torch
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return _ptr(t)


def _stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_grid(g) -> pat_grid:
    """``pat_grid`` from any object with nx, ny, nt, pml, dx, dt, c_ref, rho0, pml_alpha."""
    return pat_grid(int(g.nx), int(g.ny), int(g.nt), int(g.pml), float(g.dx), float(g.dt),
                    float(g.c_ref), float(g.rho0), float(g.pml_alpha))


class Plan:
    """A ``pat_plan``: K datasets on one grid with m sensors."""

    def __init__(self, grid, K: int, sensor_xy):
        self.grid = grid
        self.K = int(K)
        xy = np.ascontiguousarray(np.asarray(sensor_xy, dtype=np.float64))
        if xy.ndim != 2 or xy.shape[1] != 2:
            raise ValueError("sensor_xy must be [m][2]")
        self.m = xy.shape[0]
        self._g = make_grid(grid)
        h = ctypes.c_void_p()
        _check(lib().pat_plan_create(ctypes.byref(self._g), self.K, self.m,
                                     xy.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)), "pat_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pat_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def field_shape(self):
        return (self.K, self.grid.ny, self.grid.nx)

    @property
    def data_shape(self):
        return (self.K, self.grid.nt, self.m)

    def set_tile(self, col_tile: int):
        """Column-pass tile width (0 = default, 8); results do not change."""
        _check(lib().pat_plan_set_tile(self._h, int(col_tile)), "pat_plan_set_tile")

    def set_col_order(self, order: int):
        """Column-pass transform order (0 = together, 1 = one after the other, 2 = the two arrays on two
        halves of a block); results do not change."""
        _check(lib().pat_plan_set_col_order(self._h, int(order)), "pat_plan_set_col_order")

    def workspace_size(self, ckpt_every: int = 0) -> int:
        b = ctypes.c_size_t()
        _check(lib().pat_workspace_size(self._h, int(ckpt_every), ctypes.byref(b)), "pat_workspace_size")
        return b.value

    def workspace(self, ckpt_every: int = 0, device="cuda"):
        import torch
        return torch.empty(self.workspace_size(ckpt_every), dtype=torch.uint8, device=device)

    def forward(self, c, p0, data, ws, ckpt_every: int = 0, record: bool = True):
        g = self.grid
        _check(lib().pat_forward(self._h, _f32(c, g.ny * g.nx, "c"), _f32(p0, self.K * g.ny * g.nx, "p0"),
                                 _f32(data, self.K * g.nt * self.m, "data"), _ptr(ws), ws.numel(),
                                 int(ckpt_every), 1 if record else 0, _stream()), "pat_forward")

    def history_field(self, ws, n: int):
        """The recorded pressure field p^n [K][ny][nx] of a store-all workspace,
        as a device tensor view into ``ws`` (valid until the next forward)."""
        import torch
        ptr = ctypes.c_void_p()
        _check(lib().pat_history_field(self._h, _ptr(ws), int(n), ctypes.byref(ptr)), "pat_history_field")
        nbytes = self.K * self.grid.ny * self.grid.nx * 4
        off = ptr.value - ws.data_ptr()
        if off < 0 or off + nbytes > ws.numel():
            raise PatError(PAT_EINVAL, "pat_history_field: address outside the workspace")
        return ws[off:off + nbytes].view(torch.float32).view(self.field_shape)

    def misfit(self, data, y, w, resid, J):
        import torch
        n = self.K * self.grid.nt * self.m
        if J.dtype != torch.float64 or J.numel() < 1:
            raise ValueError("J must be a float64 device scalar")
        _check(lib().pat_misfit(self._h, _f32(data, n, "data"), _f32(y, n, "y"), _f32(w, self.K, "w"),
                                _f32(resid, n, "resid"), _ptr(J), _stream()), "pat_misfit")

    def adjoint_gradient(self, c, p0, resid, g_p0, g_c, ws):
        g = self.grid
        N = g.ny * g.nx
        _check(lib().pat_adjoint_gradient(self._h, _f32(c, N, "c"), _f32(p0, self.K * N, "p0"),
                                          _f32(resid, self.K * g.nt * self.m, "resid"),
                                          _f32(g_p0, self.K * N, "g_p0"), _f32(g_c, N, "g_c"),
                                          _ptr(ws), ws.numel(), _stream()), "pat_adjoint_gradient")


def project_update(x, d, alpha: float, lo=None, hi=None, lo_s: float = -np.inf, hi_s: float = np.inf):
    n = x.numel()
    _check(lib().pat_project_update(n, _f32(x, n, "x"), _f32(d, n, "d"), float(alpha),
                                    None if lo is None else _f32(lo, n, "lo"),
                                    None if hi is None else _f32(hi, n, "hi"), float(lo_s), float(hi_s),
                                    _stream()), "pat_project_update")


def prolong(coarse, fine):
    """``coarse [nchan][nyc][nxc]`` -> ``fine [nchan][nyf][nxf]``."""
    nchan, nyc, nxc = coarse.shape
    nchan2, nyf, nxf = fine.shape
    if nchan != nchan2:
        raise ValueError("channel mismatch")
    _check(lib().pat_prolong(nchan, _f32(coarse), nxc, nyc, _f32(fine), nxf, nyf, _stream()), "pat_prolong")


def prolong_phys(coarse, dx_coarse: float, fine, dx_fine: float):
    """``coarse [nchan][nyc][nxc]`` (spacing ``dx_coarse``) -> ``fine [nchan][nyf][nxf]``
    (spacing ``dx_fine``), both centred on the origin."""
    nchan, nyc, nxc = coarse.shape
    nchan2, nyf, nxf = fine.shape
    if nchan != nchan2:
        raise ValueError("channel mismatch")
    _check(lib().pat_prolong_phys(nchan, _f32(coarse), nxc, nyc, float(dx_coarse), _f32(fine), nxf, nyf,
                                  float(dx_fine), _stream()), "pat_prolong_phys")


def time_interp(y, dt_src: float, out, dt_dst: float):
    """``y [nlead][nt_src][m]`` -> ``out [nlead][nt_dst][m]``."""
    nlead, nt_src, m = y.shape
    nlead2, nt_dst, m2 = out.shape
    if nlead != nlead2 or m != m2:
        raise ValueError("shape mismatch")
    _check(lib().pat_time_interp(nlead, nt_src, m, _f32(y), float(dt_src), _f32(out), nt_dst, float(dt_dst),
                                 _stream()), "pat_time_interp")


def lbfgs_scratch_bytes(npairs: int) -> int:
    return int(lib().pat_lbfgs_scratch_bytes(int(npairs)))


def lbfgs_direction(g, s_list: Sequence, y_list: Sequence, d, scratch):
    n = g.numel()
    npairs = len(s_list)
    S = (ctypes.c_void_p * max(npairs, 1))(*[_f32(s, n, "s") for s in s_list])
    Y = (ctypes.c_void_p * max(npairs, 1))(*[_f32(y, n, "y") for y in y_list])
    _check(lib().pat_lbfgs_direction(n, _f32(g, n, "g"), npairs, ctypes.cast(S, ctypes.c_void_p),
                                     ctypes.cast(Y, ctypes.c_void_p), _f32(d, n, "d"), _ptr(scratch), _stream()),
           "pat_lbfgs_direction")


def lbfgs_direction_noalloc(g, s_list: Sequence, y_list: Sequence, d):
    """Alg. 1 without a scratch argument (the library's static per-GPU array;
    at most PAT_LBFGS_NOALLOC_MAX_PAIRS pairs); bit-identical to lbfgs_direction."""
    n = g.numel()
    npairs = len(s_list)
    S = (ctypes.c_void_p * max(npairs, 1))(*[_f32(s, n, "s") for s in s_list])
    Y = (ctypes.c_void_p * max(npairs, 1))(*[_f32(y, n, "y") for y in y_list])
    _check(lib().pat_lbfgs_direction_noalloc(n, _f32(g, n, "g"), npairs, ctypes.cast(S, ctypes.c_void_p),
                                             ctypes.cast(Y, ctypes.c_void_p), _f32(d, n, "d"), _stream()),
           "pat_lbfgs_direction_noalloc")


def free_part(x, g, lo, hi, v, out):
    """Eq. (10)-(11): ``out = 0`` on the active set of (x, g) for bounds lo, hi, else ``v``."""
    n = x.numel()
    _check(lib().pat_free_part(n, _f32(x, n, "x"), _f32(g, n, "g"), _f32(lo, n, "lo"), _f32(hi, n, "hi"),
                               _f32(v, n, "v"), _f32(out, n, "out"), _stream()), "pat_free_part")


def axpby(a: float, x, b: float, y, out):
    """``out = a x + b y`` (``y`` None: ``out = a x``)."""
    n = x.numel()
    _check(lib().pat_axpby(n, float(a), _f32(x, n, "x"), float(b), _f32(y, n, "y") if y is not None else None,
                           _f32(out, n, "out"), _stream()), "pat_axpby")


def mul(x, s, out):
    """``out = x * s`` element-wise."""
    n = x.numel()
    _check(lib().pat_mul(n, _f32(x, n, "x"), _f32(s, n, "s"), _f32(out, n, "out"), _stream()), "pat_mul")


def absmax(x, out, scratch):
    """``max |x|`` into the float64 device scalar ``out``."""
    n = x.numel()
    _check(lib().pat_absmax(n, _f32(x, n, "x"), _ptr(out), _ptr(scratch), _stream()), "pat_absmax")


def dot(a, b, out, scratch):
    n = a.numel()
    _check(lib().pat_dot(n, _f32(a, n, "a"), _f32(b, n, "b"), _ptr(out), _ptr(scratch), _stream()), "pat_dot")


def trace_start(every: int = 1):
    """Time every ``every``-th launch of each fused pass with HIP events."""
    _check(lib().pat_trace_start(int(every)), "pat_trace_start")


def trace_stop():
    _check(lib().pat_trace_stop(), "pat_trace_stop")


def trace_read():
    """``{pass kind: (timed launches, summed ms)}`` (waits for the events)."""
    out = {}
    for i, name in enumerate(PASS_KINDS):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().pat_trace_read(i, ctypes.byref(n), ctypes.byref(ms)), "pat_trace_read")
        out[name] = (n.value, ms.value)
    return out


def batch_gradient(jobs, nstreams: int = 8):
    """Objective + gradient of independent problems at once.  ``jobs``: list of
    dicts with keys plan, c, p0, y, w, data, resid, J, g_p0, g_c, ws (tensors as
    for the single-problem calls; store-all workspaces)."""
    arr = (pat_problem * len(jobs))()
    for i, j in enumerate(jobs):
        plan = j["plan"]
        g = plan.grid
        N = g.ny * g.nx
        nd = plan.K * g.nt * plan.m
        arr[i].plan = plan._h.value
        arr[i].c = _f32(j["c"], N, "c")
        arr[i].p0 = _f32(j["p0"], plan.K * N, "p0")
        arr[i].y = _f32(j["y"], nd, "y")
        arr[i].w = _f32(j["w"], plan.K, "w")
        arr[i].data = _f32(j["data"], nd, "data")
        arr[i].resid = _f32(j["resid"], nd, "resid")
        arr[i].J = _ptr(j["J"])
        arr[i].g_p0 = _f32(j["g_p0"], plan.K * N, "g_p0")
        arr[i].g_c = _f32(j["g_c"], N, "g_c")
        arr[i].ws = _ptr(j["ws"])
        arr[i].ws_bytes = j["ws"].numel()
    _check(lib().pat_batch_gradient(len(jobs), ctypes.cast(arr, ctypes.c_void_p), int(nstreams), _stream()),
           "pat_batch_gradient")


def batch_release():
    """Destroy the library's internal batch streams (recreated by the next batch)."""
    _check(lib().pat_batch_release(), "pat_batch_release")


class OuPrior:
    """Ornstein-Uhlenbeck prior operator of eq. (4) (Sec. 4.1.2) over the pixels
    of ``mask [ny][nx]`` (bool, host; None = the whole grid), spacing ``dx``,
    correlation length ``tau`` (metres)."""

    def __init__(self, ny: int, nx: int, dx: float, tau: float, mask=None):
        self.ny, self.nx = int(ny), int(nx)
        self._mask = None
        mp = None
        if mask is not None:
            m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            if m.shape != (self.ny, self.nx):
                raise ValueError("mask shape mismatch")
            self._mask = m
            mp = m.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(lib().pat_ou_create(self.ny, self.nx, float(dx), float(tau), mp, ctypes.byref(h)), "pat_ou_create")
        self._h = h
        self._scratch = {}

    def scratch(self, nvec: int, device="cuda"):
        import torch
        if nvec not in self._scratch:
            b = ctypes.c_size_t()
            _check(lib().pat_ou_scratch_bytes(self._h, int(nvec), ctypes.byref(b)), "pat_ou_scratch_bytes")
            self._scratch[nvec] = torch.empty(b.value, dtype=torch.uint8, device=device)
        return self._scratch[nvec]

    def apply(self, v, out):
        """``out = Xi v`` on the mask (``v``, ``out``: [nvec][ny][nx] float32)."""
        nvec = v.numel() // (self.ny * self.nx)
        n = nvec * self.ny * self.nx
        ws = self.scratch(nvec)
        _check(lib().pat_ou_apply(self._h, nvec, _f32(v, n, "v"), _f32(out, n, "out"), _ptr(ws), ws.numel(),
                                  _stream()), "pat_ou_apply")

    def prior(self, z, eta, inv_var, grad, J, tol: float = 1e-6, maxit: int = 500) -> int:
        """Prior terms of eq. (4) for the vectors ``z [nvec][ny][nx]`` (means
        ``eta [nvec]``, ``inv_var [nvec]`` = 1/sigma^2): fills ``grad`` and the
        device scalar ``J``; returns the conjugate-gradient iterations."""
        nvec = z.numel() // (self.ny * self.nx)
        n = nvec * self.ny * self.nx
        ws = self.scratch(nvec)
        it = ctypes.c_int32()
        _check(lib().pat_ou_prior(self._h, nvec, _f32(z, n, "z"), _f32(eta, nvec, "eta"),
                                  _f32(inv_var, nvec, "inv_var"), _f32(grad, n, "grad"), _ptr(J), float(tol),
                                  int(maxit), _ptr(ws), ws.numel(), ctypes.byref(it), _stream()), "pat_ou_prior")
        return it.value

    def close(self):
        if self._h:
            lib().pat_ou_destroy(self._h)
            self._h = None
        self._scratch = {}
