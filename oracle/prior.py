"""Ornstein-Uhlenbeck prior terms of eq. (4), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
Eq. (4) adds, for every parameter distribution z (each initial pressure and the
sound speed), the term ``1/2 || L_z (z - eta_z) ||^2`` with
``L_z^T L_z = Gamma_z^{-1}``.  Sec. 4.1.2 takes the Ornstein-Uhlenbeck prior:
``Gamma_z = sigma_z^2 Xi`` with ``Xi_ij = exp(-|r_i - r_j| / tau)`` over the
pixel positions ``r_i`` of the reconstruction domain.  So

    J_prior(z)    = 1/(2 sigma_z^2) (z - eta)^T Xi^{-1} (z - eta)
    grad J_prior  = Xi^{-1} (z - eta) / sigma_z^2        (eqs. (7)-(8), last terms)

The oracle builds ``Xi`` densely over the masked pixels and solves with a
Cholesky factorisation (the plainest route; small grids only).

Pins (tests/test_oracle_prior.py)
---------------------------------
* one row of pixels: the exponential covariance of a regular 1-D grid is the
  AR(1) correlation ``rho^|i-j|`` (``rho = exp(-dx/tau)``), whose inverse is the
  known tridiagonal matrix ``(1/(1-rho^2)) [1, 1+rho^2, ..., 1+rho^2, 1]`` on the
  diagonal and ``-rho/(1-rho^2)`` beside it;
* the gradient equals central finite differences of ``J_prior``;
* ``Xi`` is symmetric positive definite with unit diagonal and decays with
  distance; in the limit tau -> 0 the prior reduces to the independent
  Gaussian ``|z - eta|^2 / (2 sigma^2)``.
"""
from __future__ import annotations

import numpy as np


def ou_correlation(ny: int, nx: int, dx: float, tau: float, mask=None) -> np.ndarray:
    """``Xi`` over the pixels of an ``ny x nx`` box (spacing ``dx``), restricted to
    ``mask`` (bool ``[ny][nx]``, row-major order of the kept pixels) if given."""
    Y, X = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1) * dx
    if mask is not None:
        pts = pts[np.asarray(mask, dtype=bool).ravel()]
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    return np.exp(-d / tau)


def ou_prior(z: np.ndarray, eta: float, sigma: float, dx: float, tau: float, mask=None):
    """``(J_prior, grad)`` of one distribution ``z [ny][nx]``; pixels outside
    ``mask`` are not part of the prior (their gradient is zero)."""
    z = np.asarray(z, dtype=np.float64)
    ny, nx = z.shape
    m = np.ones((ny, nx), dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    Xi = ou_correlation(ny, nx, dx, tau, m)
    r = z[m] - eta
    L = np.linalg.cholesky(Xi)
    w = np.linalg.solve(L.T, np.linalg.solve(L, r))      # Xi^{-1} (z - eta)
    J = 0.5 * float(r @ w) / sigma ** 2
    g = np.zeros((ny, nx))
    g[m] = w / sigma ** 2
    return J, g


def ou_solve(b: np.ndarray, dx: float, tau: float, mask=None) -> np.ndarray:
    """``Xi^{-1} b`` on the masked pixels of ``b [ny][nx]`` (zero elsewhere)."""
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    m = np.ones((ny, nx), dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    Xi = ou_correlation(ny, nx, dx, tau, m)
    out = np.zeros((ny, nx))
    out[m] = np.linalg.solve(Xi, b[m])
    return out
