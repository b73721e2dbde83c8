"""Optimiser pieces of the reconstruction, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``project``            eq. (11): element-wise clamp to ``[L, U]``.
* ``project_update``     eq. (10): ``P(x - alpha d)``.
* ``lbfgs_direction``    Alg. 1, the two-loop recursion for ``H_k g``, read with
                         the corrections the printed listing needs (the first
                         loop takes ``s_j^T phi`` and subtracts ``lambda_j y_j``;
                         ``H^0 = (s^T y / y^T y) I`` from the newest pair).
* ``lbfgs_dense``        ``H_k`` built explicitly from the product formula of
                         Sec. 3 (the pin for ``lbfgs_direction``).
* ``projected_lbfgs``    eq. (10) iterations with a backtracking (Armijo) line
                         search, memory ``l`` (Sec. 4.1.2 uses l = 20).
* ``prolong``, ``prolong_phys``  Sec. 3.1: linear (bilinear) interpolation of a converged
                         coarse-grid solution to the next, finer grid.
* ``time_interp``        Sec. 4.1.2: linear interpolation of the data onto a
                         level's time grid.
* ``relative_error``     eq. (12).

Pins (tests/test_oracle_optim.py): projection closed form and idempotence;
two-loop vs the dense product formula; the projected L-BFGS reaches the optimum
that SciPy's L-BFGS-B finds on a bound-constrained quadratic; prolongation is
exact on affine fields away from the clamped border and on constants
everywhere; time interpolation is exact on piecewise-linear signals and on
factor-2 decimation.
"""
from __future__ import annotations

from typing import Callable, List, Optional, Tuple

import numpy as np


def project(z, lo, hi):
    """Eq. (11): ``L`` where ``z <= L``, ``U`` where ``z >= U``, else ``z``."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z <= lo, lo, np.where(z >= hi, hi, z))


def project_update(x, d, alpha, lo, hi):
    """Eq. (10): ``P(x - alpha d)``."""
    return project(np.asarray(x, dtype=np.float64) - alpha * np.asarray(d, dtype=np.float64), lo, hi)


def lbfgs_direction(g, s_list: List[np.ndarray], y_list: List[np.ndarray]) -> np.ndarray:
    """Alg. 1: ``H_k g`` from pairs ``(s_j, y_j)`` ordered oldest -> newest."""
    q = np.array(g, dtype=np.float64)
    n = len(s_list)
    if n == 0:
        return q
    rho = [1.0 / float(np.dot(y_list[j], s_list[j])) for j in range(n)]
    lam = [0.0] * n
    for j in range(n - 1, -1, -1):
        lam[j] = rho[j] * float(np.dot(s_list[j], q))
        q = q - lam[j] * y_list[j]
    s, y = s_list[-1], y_list[-1]
    psi = (float(np.dot(s, y)) / float(np.dot(y, y))) * q
    for j in range(n):
        beta = rho[j] * float(np.dot(y_list[j], psi))
        psi = psi + s_list[j] * (lam[j] - beta)
    return psi


def lbfgs_dense(s_list, y_list, nvar: int) -> np.ndarray:
    """``H_k`` as the explicit sum of products of ``V_j = I - rho_j y_j s_j^T``
    (Sec. 3), with ``H^0 = (s^T y / y^T y) I`` of the newest pair."""
    n = len(s_list)
    I = np.eye(nvar)
    if n == 0:
        return I
    s, y = s_list[-1], y_list[-1]
    H0 = (s @ y) / (y @ y) * I
    rho = [1.0 / (y_list[j] @ s_list[j]) for j in range(n)]
    V = [I - rho[j] * np.outer(y_list[j], s_list[j]) for j in range(n)]

    def chain(a, b):
        """``V_b ... V_{a}`` product ``V_{a} V_{a+1} ... V_{b}`` (right side)."""
        out = I.copy()
        for j in range(a, b + 1):
            out = out @ V[j]
        return out

    H = chain(0, n - 1).T @ H0 @ chain(0, n - 1)
    for j in range(n):
        R = chain(j + 1, n - 1)
        H = H + rho[j] * R.T @ np.outer(s_list[j], s_list[j]) @ R
    return H


def relative_error(true, rec, mask=None) -> float:
    """Eq. (12), in percent, optionally restricted to a mask."""
    t = np.asarray(true, dtype=np.float64)
    r = np.asarray(rec, dtype=np.float64)
    if mask is not None:
        t, r = t[..., mask], r[..., mask]
    return 100.0 * float(np.linalg.norm(t - r) / np.linalg.norm(t))


def prolong(coarse: np.ndarray, nyf: int, nxf: int) -> np.ndarray:
    """Bilinear interpolation of ``coarse [..., nyc, nxc]`` onto a finer cell-centred
    grid of the same physical extent, clamped at the border (no wrap)."""
    coarse = np.asarray(coarse, dtype=np.float64)
    nyc, nxc = coarse.shape[-2:]

    def axis_weights(nf, nc):
        f = (np.arange(nf) + 0.5) * (nc / nf) - 0.5
        f = np.clip(f, 0.0, nc - 1.0)
        i0 = np.minimum(np.floor(f).astype(np.int64), max(nc - 2, 0))
        t = f - i0
        i1 = np.minimum(i0 + 1, nc - 1)
        return i0, i1, t

    iy0, iy1, ty = axis_weights(nyf, nyc)
    ix0, ix1, tx = axis_weights(nxf, nxc)
    rows = coarse[..., iy0, :] * (1.0 - ty)[:, None] + coarse[..., iy1, :] * ty[:, None]
    return rows[..., :, ix0] * (1.0 - tx) + rows[..., :, ix1] * tx


def prolong_phys(coarse: np.ndarray, dx_coarse: float, nyf: int, nxf: int, dx_fine: float) -> np.ndarray:
    """Sec. 3.1 between grids of different physical extent, both centred on the
    origin: each fine pixel (at ``(i + 1/2 - n/2) dx_fine``) takes the bilinear
    interpolant of ``coarse [..., nyc, nxc]`` (spacing ``dx_coarse``) at its own
    position, clamped to the coarse grid."""
    coarse = np.asarray(coarse, dtype=np.float64)
    nyc, nxc = coarse.shape[-2:]

    def axis_weights(nf, nc):
        x = (np.arange(nf) + 0.5 - nf / 2.0) * dx_fine          # physical position
        f = np.clip(x / dx_coarse + nc / 2.0 - 0.5, 0.0, nc - 1.0)  # fractional coarse index
        i0 = np.minimum(np.floor(f).astype(np.int64), max(nc - 2, 0))
        return i0, np.minimum(i0 + 1, nc - 1), f - i0

    iy0, iy1, ty = axis_weights(nyf, nyc)
    ix0, ix1, tx = axis_weights(nxf, nxc)
    rows = coarse[..., iy0, :] * (1.0 - ty)[:, None] + coarse[..., iy1, :] * ty[:, None]
    return rows[..., :, ix0] * (1.0 - tx) + rows[..., :, ix1] * tx


def time_interp(y: np.ndarray, dt_src: float, dt_dst: float, nt_dst: int) -> np.ndarray:
    """Linear interpolation of ``y [..., nt_src, m]`` sampled at ``n dt_src`` onto
    ``n dt_dst``, ``n < nt_dst`` (held at the last sample beyond the end)."""
    y = np.asarray(y, dtype=np.float64)
    nt_src = y.shape[-2]
    t_src = np.arange(nt_src) * dt_src
    t_dst = np.arange(nt_dst) * dt_dst
    flat = np.moveaxis(y, -2, -1).reshape(-1, nt_src)
    out = np.stack([np.interp(t_dst, t_src, row) for row in flat])
    return np.moveaxis(out.reshape(y.shape[:-2] + (y.shape[-1], nt_dst)), -1, -2)


def projected_lbfgs(fun: Callable[[np.ndarray], Tuple[float, np.ndarray]], x0, lo, hi,
                    scale=None, iters: int = 40, memory: int = 20, c1: float = 1e-4,
                    max_halvings: int = 20, callback: Optional[Callable] = None):
    """Eq. (10) iterations ``x <- P(x - alpha H g)`` with backtracking.

    Works in scaled variables ``z = x / scale``.  Variables held at a bound whose
    gradient points out of the box are excluded from the direction.  The first
    direction (and any restart) is ``g / ||g||_inf``.  Step: ``alpha = 1`` halved
    until ``J(x+) <= J(x) + c1 g^T (x+ - x)``, at most ``max_halvings`` times.
    Pairs with ``y^T s <= 1e-10 |y| |s|`` are not stored.  Returns
    ``(x, J, history)``."""
    x = project(np.asarray(x0, dtype=np.float64), lo, hi)
    scale = np.ones_like(x) if scale is None else np.broadcast_to(scale, x.shape).astype(np.float64)
    J, g = fun(x)
    s_list: List[np.ndarray] = []
    y_list: List[np.ndarray] = []
    hist = [J]
    for it in range(iters):
        gz = g * scale
        active = ((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0))
        gf = np.where(active, 0.0, gz)
        if s_list:
            d = lbfgs_direction(gf, s_list, y_list)
            d = np.where(active, 0.0, d)
            if float(np.dot(d, gf)) <= 0.0:
                s_list.clear(); y_list.clear()
        if not s_list:
            nrm = np.max(np.abs(gf))
            if nrm == 0.0:
                break
            d = gf / nrm
        accepted = False
        for attempt in range(2):
            alpha = 1.0
            for _ in range(max_halvings):
                xt = project(x - alpha * d * scale, lo, hi)
                Jt, gt = fun(xt)
                if np.isfinite(Jt) and Jt <= J + c1 * float(np.dot(g, xt - x)):
                    accepted = True
                    break
                alpha *= 0.5
            if accepted or not s_list:
                break
            # the quasi-Newton direction failed: restart from projected steepest descent
            s_list.clear(); y_list.clear()
            nrm = np.max(np.abs(gf))
            d = gf / nrm
        if not accepted:
            break
        sz = (xt - x) / scale
        yz = (gt - g) * scale
        if float(np.dot(yz, sz)) > 1e-10 * np.linalg.norm(yz) * np.linalg.norm(sz):
            s_list.append(sz); y_list.append(yz)
            if len(s_list) > memory:
                s_list.pop(0); y_list.pop(0)
        x, J, g = xt, Jt, gt
        hist.append(J)
        if callback is not None:
            callback(it, x, J, g)
    return x, J, hist
