"""Pins for the oracle's forward map (eq. (1), Sec. 2.1; eq. (2), Sec. 2.2).

Each test checks the oracle against something it does not compute itself:
a closed form, the continuum solution of eq. (1), an independent finite
difference solver, or an invariant of the discrete scheme.
"""
import numpy as np
import pytest
import scipy.integrate as integrate
import scipy.special as special

from oracle import kspace
from oracle import sensors as osens
from paper_2505_08482_amd.inputs import Grid, cfl_dt, circle_sensors, pixel_centres


def _grid(n, nt, pml=0, dx=1e-4, ny=None):
    return Grid(nx=n, ny=ny or n, dx=dx, dt=cfl_dt(dx), nt=nt, pml=pml)


def _run_fields(grid, c, p0, nsteps):
    ops = kspace.Operators(grid)
    st = kspace.initial_state(ops, c, p0)
    out = [st]
    for _ in range(nsteps):
        st = kspace.step(ops, c ** 2, *st)
        out.append(st)
    return out


def test_homogeneous_periodic_is_exact_in_time():
    """c = c_ref and no PML: the k-space scheme reproduces the exact time
    dependence cos(c |k| t) of every Fourier mode (eq. (1) with p_t(0) = 0)."""
    g = _grid(32, 60)
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal((1, 32, 32))
    c = np.full((32, 32), g.c_ref)
    states = _run_fields(g, c, p0, 50)
    kx = 2 * np.pi * np.fft.fftfreq(32, d=g.dx)
    KX, KY = np.meshgrid(kx, kx)
    kabs = np.sqrt(KX ** 2 + KY ** 2)
    P0 = np.fft.fft2(p0[0])
    for n in (1, 2, 7, 50):
        exact = np.real(np.fft.ifft2(P0 * np.cos(g.c_ref * kabs * n * g.dt)))
        err = np.abs(states[n][0][0] - exact).max() / np.abs(exact).max()
        assert err < 1e-12, (n, err)


def test_homogeneous_gaussian_matches_continuum_solution():
    """Radially symmetric Gaussian in a homogeneous medium: compare with the
    continuum solution of eq. (1), p(r,t) = int P0(k) cos(c k t) J0(k r) k dk / (2 pi)."""
    n, sig = 128, 3.0
    g = _grid(n, 201)
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    R = np.sqrt(X ** 2 + Y ** 2)
    p0 = np.exp(-R ** 2 / (2 * sig ** 2))[None]
    c = np.full((n, n), g.c_ref)
    nsteps = 200
    states = _run_fields(g, c, p0, nsteps)
    ct = g.c_ref * nsteps * g.dt / g.dx          # distance travelled, in pixels
    radii = np.unique(np.round(R[R < 50.0], 12))[::37]

    def cont(r):
        f = lambda k: sig ** 2 * np.exp(-0.5 * (k * sig) ** 2) * np.cos(k * ct) * special.j0(k * r) * k
        val, _ = integrate.quad(f, 0.0, 12.0 / sig, limit=800, epsabs=1e-13, epsrel=1e-12)
        return val

    p = states[nsteps][0][0]
    for r in radii:
        i = np.argmin(np.abs(R - r))
        iy, ix = np.unravel_index(i, R.shape)
        assert abs(p[iy, ix] - cont(R[iy, ix])) < 1e-6, (r, p[iy, ix], cont(R[iy, ix]))


def _fd_reference_1d(c_fun, p0_fun, L, n_fine, t_end, dt_fine):
    """Independent solver of (1/c^2) p_tt = p_xx on a periodic line: 6th-order
    central differences in space, classical RK4 in time on (p, p_t)."""
    h = L / n_fine
    x = (np.arange(n_fine) + 0.5 - n_fine / 2) * h
    c2 = c_fun(x) ** 2
    coef = np.array([1 / 90, -3 / 20, 3 / 2, -49 / 18, 3 / 2, -3 / 20, 1 / 90]) / h ** 2

    def lap(p):
        return sum(coef[j] * np.roll(p, 3 - j) for j in range(7))

    def rhs(s):
        p, v = s
        return np.array([v, c2 * lap(p)])

    s = np.array([p0_fun(x), np.zeros(n_fine)])
    nsteps = int(round(t_end / dt_fine))
    for _ in range(nsteps):
        k1 = rhs(s)
        k2 = rhs(s + 0.5 * dt_fine * k1)
        k3 = rhs(s + 0.5 * dt_fine * k2)
        k4 = rhs(s + dt_fine * k3)
        s = s + dt_fine / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return x, s[0]


def test_heterogeneous_1d_reduction_matches_independent_solver():
    """Fields constant along y with a smoothly varying c(x): the 2-D scheme must
    follow eq. (1) as computed by an unrelated finite-difference solver.  The
    k-space correction is exact only at c = c_ref, so elsewhere the scheme is
    second order in dt: halving dt must cut the difference about fourfold."""
    n, nsteps = 128, 200
    dx = 1e-4
    L = n * dx
    c_fun = lambda x: 1500.0 + 80.0 * np.sin(2 * np.pi * x / L) + 30.0 * np.cos(4 * np.pi * x / L)
    p0_fun = lambda x: np.exp(-x ** 2 / (2 * (4 * dx) ** 2))
    xs = pixel_centres(n) * dx
    c = np.tile(c_fun(xs), (2, 1))
    p0 = np.tile(p0_fun(xs), (2, 1))[None]
    t_end = nsteps * cfl_dt(dx)
    xf, p_fd = _fd_reference_1d(c_fun, p0_fun, L, 3 * n, t_end, cfl_dt(dx) / 10)
    p_fd_c = p_fd[1::3]
    assert np.allclose(xf[1::3], xs)
    errs = []
    for refine in (1, 2):
        g = Grid(nx=n, ny=2, dx=dx, dt=cfl_dt(dx) / refine, nt=1, pml=0)
        p_ks = _run_fields(g, c, p0, nsteps * refine)[-1][0][0, 0]
        errs.append(np.abs(p_ks - p_fd_c).max() / np.abs(p_fd_c).max())
    assert errs[0] < 2e-3, errs
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def _energy(grid, c, p_n, p_np1, ux, uy):
    return 0.5 * grid.rho0 * (np.sum(ux ** 2) + np.sum(uy ** 2)) \
        + 0.5 / grid.rho0 * np.sum(p_n * p_np1 / c ** 2)


def test_energy_conserved_without_pml_for_any_c():
    """PML off: E^{n+1/2} = rho0/2 |u^{n+1/2}|^2 + 1/(2 rho0) sum p^n p^{n+1}/c^2 is an
    exact invariant of the staggered scheme for any c (derived from eq. (1)'s
    first-order form: rho0 u_t = -grad p, rho_t = -rho0 div u, p = c^2 rho)."""
    n = 40
    g = _grid(n, 300)
    rng = np.random.default_rng(7)
    c = 1500.0 + 100.0 * rng.uniform(-1, 1, (n, n))
    p0 = rng.standard_normal((1, n, n))
    states = _run_fields(g, c, p0, 200)
    E = [_energy(g, c, states[i][0], states[i + 1][0], states[i + 1][1], states[i + 1][2])
         for i in range(200)]
    E = np.array(E)
    assert np.abs(E - E[0]).max() / abs(E[0]) < 1e-12


def test_pml_absorbs_outgoing_waves():
    """PML on: the energy decays, and once the wave has left the interior the
    interior pressure is small compared with the initial peak."""
    n, P = 64, 10
    g = _grid(n, 1)
    g = Grid(nx=n, ny=n, dx=g.dx, dt=g.dt, nt=1, pml=P)
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    p0 = np.exp(-(X ** 2 + Y ** 2) / (2 * 2.0 ** 2))[None]
    c = np.full((n, n), 1500.0)
    nsteps = int(2.5 * n * np.sqrt(2) / 0.3)
    states = _run_fields(g, c, p0, nsteps)
    E = np.array([_energy(g, c, states[i][0], states[i + 1][0], states[i + 1][1], states[i + 1][2])
                  for i in range(nsteps)])
    assert E[-1] < 1e-4 * E[0]
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    interior = np.abs(states[-1][0][0, P:-P, P:-P]).max()
    assert interior < 5e-3 * p0.max(), interior


def test_linearity_in_p0_and_rotation_symmetry():
    """f is linear in p0 (eq. (2) at fixed c), and a 90-degree rotation of c and
    p0 rotates the sensor traces (circle of 4k sensors, no preferred axis)."""
    n, m = 48, 16
    g = Grid(nx=n, ny=n, dx=1e-4, dt=cfl_dt(1e-4), nt=80, pml=6)
    rng = np.random.default_rng(3)
    c = 1500.0 + 50.0 * rng.uniform(-1, 1, (n, n))
    xy = circle_sensors(m, 17 * g.dx)
    a = rng.standard_normal((1, n, n))
    b = rng.standard_normal((1, n, n))
    da, _ = kspace.forward(g, xy, c, a, record=False)
    db, _ = kspace.forward(g, xy, c, b, record=False)
    dab, _ = kspace.forward(g, xy, c, 2.0 * a - 3.0 * b, record=False)
    assert np.abs(dab - (2 * da - 3 * db)).max() < 1e-12 * np.abs(dab).max()
    # np.rot90 moves a feature at (x, y) to (y, -x) on the cell-centred grid
    rot = lambda f: np.rot90(f, k=1, axes=(-2, -1))
    d0, _ = kspace.forward(g, xy, c, a, record=False)
    d1, _ = kspace.forward(g, xy, rot(c), rot(a), record=False)
    # so the new sensor at angle theta sees what the old one at theta + 90 deg saw
    perm = (np.arange(m) + m // 4) % m
    assert np.abs(d1 - d0[:, :, perm]).max() < 1e-10 * np.abs(d0).max()
