"""Forward map and exact discrete adjoint gradient, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
Sec. 2.1, eq. (1): the lossless wave initial value problem
``(1/c^2) p_tt - lap p = 0, p(0) = p0, p_t(0) = 0``, solved with a k-space
pseudospectral method.  The paper names the method but not the scheme; the
reading used here is the first-order staggered split-field system with a
constant ambient density ``rho0`` (which cancels from ``p``):

    u_x^{n+1/2} = as_x (as_x u_x^{n-1/2} - dt/rho0 * Dx+ p^n)        (same for y)
    rho_x^{n+1} = a_x  (a_x  rho_x^n     - dt*rho0 * Dx- u_x^{n+1/2}) (same for y)
    p^{n+1}     = c^2 (rho_x^{n+1} + rho_y^{n+1})

with spectral staggered derivatives ``D+- f = IFFT2[ i k kappa exp(+-i k dx/2) FFT2 f ]``,
the k-space correction ``kappa = sinc(c_ref |k| dt / 2)``, FFT-order wavenumbers
with the Nyquist bin negative and the multiplier taken real there, and a
multiplicative PML ``a = exp(-alpha dt / 2)`` with
``alpha = pml_alpha * (c_ref/dx) * (depth/P)^4`` (``as``: staggered by half a cell).
Initial state: ``rho_x = rho_y = p0/(2 c^2)`` and ``u^{-1/2} = +dt/(2 rho0) D+ p0``
(this makes the discrete velocity odd in time, i.e. ``p_t(0) = 0``).

Sec. 2.2, eq. (2): data ``d^n = S p^n`` for ``n = 0..nt-1`` (``d^0 = S p0``), one
dataset per initial pressure, all sharing ``c``.

Eq. (4) data term: ``J = sum_i 1/2 ||W_i (d_i - y_i)||^2`` with ``W_i = 1/sigma_i``
(zero-mean noise, diagonal covariance).

Eqs. (5)-(9): the gradient of ``J`` with respect to every ``p0_i`` and ``c``.
The paper states the continuous adjoint; the oracle computes the exact gradient
of the *discrete* ``J`` above by running the transposed recurrence backwards in
time (the adjoint wave field is driven by the time-reversed weighted residual
injected at the sensors, as eq. (5)/(6) describe).

Pins (tests/test_oracle_forward.py, tests/test_oracle_adjoint.py)
-----------------------------------------------------------------
* homogeneous, PML off: ``p^n = IFFT2[cos(c_ref |k| n dt) FFT2 p0]`` exactly;
* homogeneous Gaussian: the continuum solution of eq. (1) (Hankel integral);
* 1-D heterogeneous reduction: an independent fine-grid finite-difference
  solution of eq. (1);
* PML off: the discrete energy is conserved for any c; PML on: it decays;
* dot-product identity in p0 and a tangent-linear identity in c;
* central finite differences of J for every pixel of c and p0 on a 32^2 grid.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import sensors as _sensors

# Number of threads scipy.fft may use; the benchmark's CPU leg may change it.
WORKERS = 1


def _fft2(f):
    return sfft.fft2(f, axes=(-2, -1), workers=WORKERS)


def _ifft2(F):
    return sfft.ifft2(F, axes=(-2, -1), workers=WORKERS)


def wavenumbers(n: int, d: float) -> np.ndarray:
    """FFT-order wavenumbers ``2 pi m / (n d)``, ``m = 0..n/2-1, -n/2..-1``."""
    m = np.arange(n)
    m = np.where(m < (n + 1) // 2, m, m - n)
    return 2.0 * np.pi * m / (n * d)


def _pml_depth(n: int, P: int, x: np.ndarray) -> np.ndarray:
    """Depth (grid points) of position ``x`` into the PML of width ``P``."""
    left = P - x
    right = x - (n - 1 - P)
    return np.maximum(np.maximum(left, right), 0.0)


def pml_profiles(n: int, P: int, pml_alpha: float, c_ref: float, dx: float, dt: float):
    """``(a, a_stag)`` along one axis: ``exp(-alpha dt / 2)`` at the grid points and
    half a cell to the right of them."""
    if P == 0:
        return np.ones(n), np.ones(n)
    i = np.arange(n, dtype=np.float64)
    alpha = lambda d: pml_alpha * (c_ref / dx) * (d / P) ** 4
    a = np.exp(-alpha(_pml_depth(n, P, i)) * dt / 2.0)
    a_s = np.exp(-alpha(_pml_depth(n, P, i + 0.5)) * dt / 2.0)
    return a, a_s


class Operators:
    """Spectral multipliers and PML profiles of one grid (duck-typed ``grid``
    with ``nx, ny, dx, dt, pml, pml_alpha, c_ref, rho0``)."""

    def __init__(self, grid):
        self.g = grid
        nx, ny, dx, dt = grid.nx, grid.ny, grid.dx, grid.dt
        kx = wavenumbers(nx, dx)
        ky = wavenumbers(ny, dx)
        KX, KY = np.meshgrid(kx, ky)           # [ny][nx]
        kabs = np.sqrt(KX ** 2 + KY ** 2)
        arg = grid.c_ref * kabs * dt / 2.0
        with np.errstate(invalid="ignore", divide="ignore"):
            kappa = np.where(arg == 0.0, 1.0, np.sin(arg) / np.where(arg == 0.0, 1.0, arg))
        self.kappa = kappa
        self.kabs = kabs
        self.Mxp = 1j * KX * kappa * np.exp(+1j * KX * dx / 2.0)
        self.Mxm = 1j * KX * kappa * np.exp(-1j * KX * dx / 2.0)
        self.Myp = 1j * KY * kappa * np.exp(+1j * KY * dx / 2.0)
        self.Mym = 1j * KY * kappa * np.exp(-1j * KY * dx / 2.0)
        # Nyquist bins (even length only): the staggered multiplier is real there.
        if nx % 2 == 0:
            for M in (self.Mxp, self.Mxm):
                M[:, nx // 2] = M[:, nx // 2].real
        if ny % 2 == 0:
            for M in (self.Myp, self.Mym):
                M[ny // 2, :] = M[ny // 2, :].real
        self.ax, self.asx = pml_profiles(nx, grid.pml, grid.pml_alpha, grid.c_ref, dx, dt)
        ay, asy = pml_profiles(ny, grid.pml, grid.pml_alpha, grid.c_ref, dx, dt)
        self.ay, self.asy = ay[:, None], asy[:, None]

    def apply(self, M: np.ndarray, f: np.ndarray) -> np.ndarray:
        """Real part of ``IFFT2[M FFT2 f]`` over the last two axes."""
        return _ifft2(M * _fft2(f)).real

    def Dxp(self, f):
        return self.apply(self.Mxp, f)

    def Dxm(self, f):
        return self.apply(self.Mxm, f)

    def Dyp(self, f):
        return self.apply(self.Myp, f)

    def Dym(self, f):
        return self.apply(self.Mym, f)


def initial_state(ops: Operators, c: np.ndarray, p0: np.ndarray):
    """``(p, ux, uy, rx, ry)`` at n = 0: eq. (1) initial conditions."""
    g = ops.g
    c2 = c ** 2
    p = np.array(p0, dtype=np.float64)
    rx = p / (2.0 * c2)
    ry = rx.copy()
    ux = (g.dt / (2.0 * g.rho0)) * ops.Dxp(p)
    uy = (g.dt / (2.0 * g.rho0)) * ops.Dyp(p)
    return p, ux, uy, rx, ry


def step(ops: Operators, c2, p, ux, uy, rx, ry):
    """One update n -> n+1 of the staggered k-space scheme."""
    g = ops.g
    ux = ops.asx * (ops.asx * ux - (g.dt / g.rho0) * ops.Dxp(p))
    uy = ops.asy * (ops.asy * uy - (g.dt / g.rho0) * ops.Dyp(p))
    rx = ops.ax * (ops.ax * rx - g.dt * g.rho0 * ops.Dxm(ux))
    ry = ops.ay * (ops.ay * ry - g.dt * g.rho0 * ops.Dym(uy))
    p = c2 * (rx + ry)
    return p, ux, uy, rx, ry


def forward(grid, xy, c, p0, record: bool = True, ops: Operators = None, return_state: bool = False):
    """Forward map f(p0, c) of eq. (2).

    ``c``: ``[ny][nx]`` (shared by all datasets) or ``[K][ny][nx]``;
    ``p0``: ``[K][ny][nx]``.  Returns ``(data [K][nt][m], hist)`` where ``hist`` is
    the pressure history ``[nt][K][ny][nx]`` (``None`` unless ``record``)."""
    ops = ops or Operators(grid)
    S = _sensors.sensor_matrix(grid.nx, grid.ny, grid.dx, xy)
    c = np.asarray(c, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    if p0.ndim != 3 or p0.shape[1:] != (grid.ny, grid.nx):
        raise ValueError("p0 must be [K][ny][nx]")
    K = p0.shape[0]
    c2 = c ** 2
    p, ux, uy, rx, ry = initial_state(ops, c, p0)
    data = np.empty((K, grid.nt, S.shape[0]))
    hist = np.empty((grid.nt, K, grid.ny, grid.nx)) if record else None
    data[:, 0] = _sensors.sample(S, p)
    if record:
        hist[0] = p
    for n in range(grid.nt - 1):
        p, ux, uy, rx, ry = step(ops, c2, p, ux, uy, rx, ry)
        data[:, n + 1] = _sensors.sample(S, p)
        if record:
            hist[n + 1] = p
    if return_state:
        return data, hist, (p, ux, uy, rx, ry)
    return data, hist


def misfit(data, y, w):
    """Eq. (4) data term with ``W_i = w[i]``: returns ``(resid, J)`` where
    ``resid = W^2 (data - y)`` drives the adjoint (eq. (6), sign folded in)."""
    data = np.asarray(data, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w2 = np.asarray(w, dtype=np.float64)[:, None, None] ** 2
    diff = data - y
    return w2 * diff, 0.5 * float(np.sum(w2 * diff * diff))


def adjoint_gradient(grid, xy, c, p0, resid, hist, ops: Operators = None):
    """Exact gradient of ``J`` (eq. (4) data term) w.r.t. every ``p0_i`` and ``c``.

    ``resid [K][nt][m]`` is ``dJ/d data`` (``W^2 (f - y)`` for the misfit above);
    ``hist`` is the forward pressure history.  Returns ``(g_p0 [K][ny][nx],
    g_c)``; ``g_c`` is summed over datasets when ``c`` is 2-D (eq. (8)'s sum over
    i), otherwise one gradient per dataset.

    The recurrence transposes the forward step by step (reverse mode):
    adjoint pressure ``ph^n = S^T r^n + dt/rho0 sum_j Dj-(as_j uh_j)``; adjoint
    densities ``rh_j += c^2 ph^n``; sound-speed sensitivity of ``p^n = c^2 (...)``
    ``g_c += (2/c) p^n ph^n``; adjoint velocities
    ``uh_j <- as_j^2 uh_j + dt rho0 Dj+(a_j rh_j)``; then ``rh_j <- a_j^2 rh_j``.
    The initial state contributes ``p0`` directly, through ``rho = p0/(2c^2)`` and
    through ``u^{-1/2}``."""
    ops = ops or Operators(grid)
    g = ops.g
    S = _sensors.sensor_matrix(grid.nx, grid.ny, grid.dx, xy)
    c = np.asarray(c, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    resid = np.asarray(resid, dtype=np.float64)
    K = p0.shape[0]
    c2 = c ** 2
    shape = (K, grid.ny, grid.nx)
    uhx = np.zeros(shape)
    uhy = np.zeros(shape)
    rhx = np.zeros(shape)
    rhy = np.zeros(shape)
    gc = np.zeros(shape)
    bu = g.dt / g.rho0
    br = g.dt * g.rho0
    for n in range(grid.nt - 1, 0, -1):
        ph = _sensors.inject(S, resid[:, n], grid.ny, grid.nx) \
            + bu * (ops.Dxm(ops.asx * uhx) + ops.Dym(ops.asy * uhy))
        rhx = rhx + c2 * ph
        rhy = rhy + c2 * ph
        gc = gc + (2.0 / c) * hist[n] * ph
        uhx = ops.asx ** 2 * uhx + br * ops.Dxp(ops.ax * rhx)
        uhy = ops.asy ** 2 * uhy + br * ops.Dyp(ops.ay * rhy)
        rhx = ops.ax ** 2 * rhx
        rhy = ops.ay ** 2 * rhy
    ph0 = _sensors.inject(S, resid[:, 0], grid.ny, grid.nx) \
        + bu * (ops.Dxm(ops.asx * uhx) + ops.Dym(ops.asy * uhy))
    g_p0 = ph0 + (rhx + rhy) / (2.0 * c2) \
        - (bu / 2.0) * (ops.Dxm(ops.asx ** 2 * uhx) + ops.Dym(ops.asy ** 2 * uhy))
    gc = gc - (p0 / c ** 3) * (rhx + rhy)
    g_c = gc.sum(axis=0) if c.ndim == 2 else gc
    return g_p0, g_c


def objective(grid, xy, c, p0, y, w, ops: Operators = None):
    """``J(p0, c)`` of eq. (4) (data term) — used by finite-difference tests."""
    data, _ = forward(grid, xy, c, p0, record=False, ops=ops)
    return misfit(data, y, w)[1]


def objective_batch(grid, xy, c, p0, y, w, ops: Operators = None):
    """``J`` for a batch of independent problems (``c, p0 [B][ny][nx]``, one
    dataset each, the same ``y [nt][m]`` and weight ``w``): returns ``J [B]``."""
    data, _ = forward(grid, xy, c, p0, record=False, ops=ops)
    diff = data - np.asarray(y)[None]
    return 0.5 * w ** 2 * np.sum(diff * diff, axis=(1, 2))
