"""Pins of the Ornstein-Uhlenbeck prior terms of eq. (4) (oracle/prior.py)."""
import numpy as np

from oracle import prior


def test_one_row_is_ar1_with_tridiagonal_inverse():
    """A single row of n pixels: Xi = rho^|i-j| with rho = exp(-dx/tau); its
    inverse is the known tridiagonal AR(1) precision matrix."""
    n, dx, tau = 12, 0.2e-3, 1.5e-3
    Xi = prior.ou_correlation(1, n, dx, tau)
    rho = np.exp(-dx / tau)
    i = np.arange(n)
    assert np.allclose(Xi, rho ** np.abs(i[:, None] - i[None, :]), rtol=0, atol=1e-15)
    P = np.zeros((n, n))
    P[i, i] = 1.0 + rho ** 2
    P[0, 0] = P[-1, -1] = 1.0
    P[i[:-1], i[:-1] + 1] = P[i[:-1] + 1, i[:-1]] = -rho
    P /= 1.0 - rho ** 2
    assert np.allclose(P @ Xi, np.eye(n), atol=1e-10)
    # and the solver returns P b
    b = np.random.default_rng(0).standard_normal((1, n))
    assert np.allclose(prior.ou_solve(b, dx, tau)[0], P @ b[0], rtol=1e-9, atol=1e-9)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    ny, nx, dx, tau = 7, 9, 0.3e-3, 1.0e-3
    mask = np.ones((ny, nx), dtype=bool)
    mask[0, :3] = False
    z = 1450.0 + 60.0 * rng.standard_normal((ny, nx))
    eta, sigma = 1505.0, 125.0
    J, g = prior.ou_prior(z, eta, sigma, dx, tau, mask)
    assert np.all(g[~mask] == 0.0)
    h = 1e-3
    for (yy, xx) in [(0, 5), (3, 4), (6, 8), (2, 0)]:
        zp = z.copy(); zp[yy, xx] += h
        zm = z.copy(); zm[yy, xx] -= h
        fd = (prior.ou_prior(zp, eta, sigma, dx, tau, mask)[0] - prior.ou_prior(zm, eta, sigma, dx, tau, mask)[0]) / (2 * h)
        assert abs(fd - g[yy, xx]) <= 1e-6 * max(1.0, abs(g[yy, xx])), (yy, xx, fd, g[yy, xx])


def test_correlation_is_spd_and_reduces_to_white_noise():
    Xi = prior.ou_correlation(6, 5, 0.2e-3, 1.5e-3)
    assert np.allclose(Xi, Xi.T) and np.allclose(np.diag(Xi), 1.0)
    assert np.linalg.eigvalsh(Xi).min() > 0.0
    # correlation decays with distance from pixel 0
    assert np.all(np.diff(Xi[0, :5]) < 0)
    # tau -> 0: independent pixels, J = |z - eta|^2 / (2 sigma^2)
    z = np.random.default_rng(2).standard_normal((4, 4))
    J, g = prior.ou_prior(z, 0.1, 2.0, 1e-3, 1e-7)
    assert np.isclose(J, np.sum((z - 0.1) ** 2) / 8.0, rtol=1e-12)
    assert np.allclose(g, (z - 0.1) / 4.0, rtol=1e-12)
