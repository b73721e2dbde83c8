"""Pins for the optimiser pieces: eq. (10)-(11), Alg. 1, Sec. 3.1, Sec. 4.1.2."""
import numpy as np
import pytest
import scipy.optimize as sopt

from oracle import optim


def test_projection_closed_form_and_idempotent():
    z = np.array([-2.0, 0.0, 0.5, 1.0, 3.0])
    lo = np.array([0.0, 0.0, 0.0, 0.0, 0.0])
    hi = np.array([1.0, 1.0, 1.0, 1.0, 1.0])
    pz = optim.project(z, lo, hi)
    assert np.array_equal(pz, [0.0, 0.0, 0.5, 1.0, 1.0])
    assert np.array_equal(optim.project(pz, lo, hi), pz)
    # no upper bound on p0 (Sec. 4.1.2): hi = +inf
    assert np.array_equal(optim.project(z, 0.0, np.inf), [0.0, 0.0, 0.5, 1.0, 3.0])
    # a masked pixel with lo == hi is pinned
    assert np.array_equal(optim.project_update(np.array([5.0]), np.array([3.0]), 2.0, 1500.0, 1500.0), [1500.0])


def _pairs(rng, nvar, npairs):
    A = rng.standard_normal((nvar, nvar))
    A = A @ A.T + nvar * np.eye(nvar)        # SPD Hessian: y^T s > 0 always
    s_list = [rng.standard_normal(nvar) for _ in range(npairs)]
    y_list = [A @ s for s in s_list]
    return s_list, y_list


@pytest.mark.parametrize("npairs", [1, 2, 5, 8])
def test_two_loop_equals_dense_product_formula(npairs):
    rng = np.random.default_rng(npairs)
    nvar = 8
    s_list, y_list = _pairs(rng, nvar, npairs)
    g = rng.standard_normal(nvar)
    H = optim.lbfgs_dense(s_list, y_list, nvar)
    assert np.allclose(optim.lbfgs_direction(g, s_list, y_list), H @ g, rtol=1e-12, atol=1e-12)


def test_dense_formula_satisfies_secant_condition():
    """Independent of both implementations: BFGS's H_k maps the newest y to s."""
    rng = np.random.default_rng(11)
    s_list, y_list = _pairs(rng, 6, 4)
    H = optim.lbfgs_dense(s_list, y_list, 6)
    assert np.allclose(H @ y_list[-1], s_list[-1], rtol=1e-12, atol=1e-12)
    assert np.allclose(H, H.T, atol=1e-12)
    assert np.all(np.linalg.eigvalsh(H) > 0)


def test_projected_lbfgs_matches_scipy_lbfgsb_on_box_quadratic():
    rng = np.random.default_rng(5)
    n = 30
    A = rng.standard_normal((n, n))
    A = A @ A.T / n + 0.5 * np.eye(n)
    b = rng.standard_normal(n) * 3.0
    lo = np.full(n, -0.5)
    hi = np.full(n, 0.7)
    lo[:5] = -np.inf
    fun = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    ref = sopt.minimize(fun, np.zeros(n), jac=True, method="L-BFGS-B",
                        bounds=list(zip(lo, hi)), options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 1000})
    x, J, hist = optim.projected_lbfgs(fun, np.zeros(n), lo, hi, iters=300, memory=20)
    assert np.all(np.diff(hist) <= 1e-12)
    assert np.abs(x - ref.x).max() < 1e-6, np.abs(x - ref.x).max()


def test_prolong_reproduces_affine_and_constant_fields():
    nc, nf = 16, 32
    xc = np.arange(nc) + 0.5 - nc / 2
    xf = (np.arange(nf) + 0.5 - nf / 2) * (nc / nf)
    Xc, Yc = np.meshgrid(xc, xc)
    Xf, Yf = np.meshgrid(xf, xf)
    coarse = np.stack([1.5 + 0.3 * Xc - 0.2 * Yc, np.full((nc, nc), 1500.0)])
    fine = optim.prolong(coarse, nf, nf)
    inner = (np.abs(Xf) <= xc.max()) & (np.abs(Yf) <= xc.max())
    assert np.allclose(fine[0][inner], (1.5 + 0.3 * Xf - 0.2 * Yf)[inner], atol=1e-13)
    assert np.all(fine[1] == 1500.0)
    # symmetric input gives symmetric output
    sym = np.exp(-(Xc ** 2 + Yc ** 2) / 10.0)
    f = optim.prolong(sym, nf, nf)
    assert np.allclose(f, f[::-1, :], atol=1e-15) and np.allclose(f, f.T, atol=1e-15)
    # each fine value is a convex combination of coarse values
    rng = np.random.default_rng(0)
    r = rng.uniform(0, 1, (nc, nc))
    fr = optim.prolong(r, nf, nf)
    assert fr.min() >= r.min() - 1e-15 and fr.max() <= r.max() + 1e-15


def test_prolong_phys_between_grids_of_different_extent():
    """Table 1's levels differ in physical extent: a coarse 39-px grid at
    0.5263 mm onto an 89-px grid at 0.2273 mm (the target square of both).
    An affine field in physical coordinates is reproduced exactly wherever the
    fine pixel lies inside the coarse pixel centres; outside, the value is the
    clamped edge value; constants are kept everywhere."""
    nc, dxc, nf, dxf = 39, 0.5263e-3, 125, 0.2273e-3
    xc = (np.arange(nc) + 0.5 - nc / 2) * dxc
    xf = (np.arange(nf) + 0.5 - nf / 2) * dxf
    Xc, Yc = np.meshgrid(xc, xc)
    Xf, Yf = np.meshgrid(xf, xf)
    affine = lambda X, Y: 1450.0 + 2.0e4 * X - 3.0e4 * Y
    fine = optim.prolong_phys(np.stack([affine(Xc, Yc), np.full((nc, nc), 7.0)]), dxc, nf, nf, dxf)
    inside = (np.abs(Xf) <= xc.max()) & (np.abs(Yf) <= xc.max())
    assert inside.sum() > 0.4 * nf * nf
    assert np.allclose(fine[0][inside], affine(Xf, Yf)[inside], rtol=0, atol=1e-9)
    assert np.all(fine[1] == 7.0)
    # beyond the last coarse centre along x (and inside along y) the x-edge value is held
    col = np.argmax(xf > xc.max())
    rows = np.abs(xf) <= xc.max()
    assert np.allclose(fine[0][rows, col:], affine(xc.max(), Yf[rows, col:]), atol=1e-9)
    # a grid of the same extent reduces to the same-extent prolongation (16 -> 32 pixels)
    rng = np.random.default_rng(3)
    r = rng.uniform(0, 1, (2, 16, 16))
    assert np.allclose(optim.prolong_phys(r, 2.0e-4, 32, 32, 1.0e-4), optim.prolong(r, 32, 32), atol=1e-15)


def test_time_interp_exact_for_piecewise_linear_and_decimation():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((2, 41, 3))
    dec = optim.time_interp(y, 1.0, 2.0, 21)
    assert np.array_equal(dec, y[:, ::2])
    t = np.arange(41) * 0.5
    lin = np.stack([2.0 - 0.25 * t, 1.0 + 3.0 * t], axis=-1)[None]
    out = optim.time_interp(lin, 0.5, 0.3, 60)
    t2 = np.arange(60) * 0.3
    assert np.allclose(out[0, :, 0], 2.0 - 0.25 * t2)
    assert np.allclose(out[0, :, 1], 1.0 + 3.0 * t2)


def test_relative_error_eq12():
    a = np.array([3.0, 4.0])
    assert optim.relative_error(a, np.zeros(2)) == 100.0
    assert optim.relative_error(a, a) == 0.0
