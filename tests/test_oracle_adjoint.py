"""Pins for the oracle's gradient (eqs. (5)-(9), Sec. 3).

The oracle's gradient is the exact gradient of the discrete data misfit of
eq. (4).  These tests pin it to things it does not compute itself:

* the dot-product identity <A p0, y> = <p0, A^T y> (p0 -> data is linear);
* a tangent-linear recurrence for the sound speed, written here from the
  linearisation of the update p = c^2 (rho_x + rho_y) and rho^0 = p0/(2 c^2);
* brute-force central finite differences of J for every pixel of c and p0.
"""
import os

import numpy as np
import pytest

from oracle import kspace
from oracle import sensors as osens
from paper_2505_08482_amd.inputs import Grid, cfl_dt, circle_sensors


def _setup(n=32, nt=120, pml=4, m=12, K=1, seed=0):
    g = Grid(nx=n, ny=n, dx=1e-4, dt=cfl_dt(1e-4), nt=nt, pml=pml)
    rng = np.random.default_rng(seed)
    c = 1500.0 + 60.0 * rng.uniform(-1, 1, (n, n))
    p0 = rng.uniform(0, 1, (K, n, n))
    xy = circle_sensors(m, (n / 2 - pml - 2) * g.dx)
    return g, rng, c, p0, xy


def test_dot_product_identity_p0():
    g, rng, c, p0, xy = _setup(n=36, nt=150, K=2, m=10, seed=1)
    y = rng.standard_normal((2, g.nt, 10))
    data, hist = kspace.forward(g, xy, c, p0)
    gp0, _ = kspace.adjoint_gradient(g, xy, c, p0, y, hist)
    lhs = float(np.sum(data * y))
    rhs = float(np.sum(p0 * gp0))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)


def _tangent_linear(g, xy, c, p0, dc):
    """Directional derivative of the data w.r.t. c along dc, obtained by
    differentiating every line of the forward recurrence."""
    ops = kspace.Operators(g)
    S = osens.sensor_matrix(g.nx, g.ny, g.dx, xy)
    c2 = c ** 2
    p, ux, uy, rx, ry = kspace.initial_state(ops, c, p0)
    # rho^0 = p0 / (2 c^2): d rho^0 = -p0 dc / c^3 ; p^0 = p0 does not depend on c
    drx = -p0 * dc / c ** 3
    dry = drx.copy()
    dux = np.zeros_like(ux)
    duy = np.zeros_like(uy)
    dp = np.zeros_like(p)
    dd = [osens.sample(S, dp)]
    for _ in range(g.nt - 1):
        dux = ops.asx * (ops.asx * dux - (g.dt / g.rho0) * ops.Dxp(dp))
        duy = ops.asy * (ops.asy * duy - (g.dt / g.rho0) * ops.Dyp(dp))
        drx = ops.ax * (ops.ax * drx - g.dt * g.rho0 * ops.Dxm(dux))
        dry = ops.ay * (ops.ay * dry - g.dt * g.rho0 * ops.Dym(duy))
        p, ux, uy, rx, ry = kspace.step(ops, c2, p, ux, uy, rx, ry)
        # p = c^2 (rx + ry): dp = c^2 (drx + dry) + 2 c dc (rx + ry)
        dp = c2 * (drx + dry) + 2.0 * c * dc * (rx + ry)
        dd.append(osens.sample(S, dp))
    return np.stack(dd, axis=1)


def test_tangent_linear_identity_c():
    g, rng, c, p0, xy = _setup(n=32, nt=140, K=2, m=12, seed=2)
    dc = rng.standard_normal(c.shape)
    y = rng.standard_normal((2, g.nt, 12))
    dd = _tangent_linear(g, xy, c, p0, dc)
    _, hist = kspace.forward(g, xy, c, p0)
    _, gc = kspace.adjoint_gradient(g, xy, c, p0, y, hist)
    lhs = float(np.sum(dd * y))
    rhs = float(np.sum(gc * dc))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)


def test_finite_differences_every_pixel_32x32():
    """Central differences of J for all 32^2 pixels of c (h = 1e-3 m/s) and of
    p0 (h = 1e-4), PML on, against the adjoint gradient."""
    n, nt, m = 32, 120, 12
    g, rng, c, p0, xy = _setup(n=n, nt=nt, K=1, m=m, seed=3)
    y = rng.standard_normal((1, nt, m)) * 0.05
    w = 3.0
    data, hist = kspace.forward(g, xy, c, p0)
    r, J = kspace.misfit(data, y, np.array([w]))
    gp0, gc = kspace.adjoint_gradient(g, xy, c, p0, r, hist)

    old = kspace.WORKERS
    kspace.WORKERS = os.cpu_count() or 1
    try:
        ops = kspace.Operators(g)
        N = n * n
        fd_c = np.empty(N)
        fd_p = np.empty(N)
        hc, hp = 1e-3, 1e-4
        chunk = 256
        eye = np.eye(N).reshape(N, n, n)
        for s in range(0, N, chunk):
            e = eye[s:s + chunk]
            B = e.shape[0]
            cp = c[None] + hc * e
            cm = c[None] - hc * e
            pr = np.broadcast_to(p0, (B, n, n))
            Jp = kspace.objective_batch(g, xy, cp, pr, y[0], w, ops)
            Jm = kspace.objective_batch(g, xy, cm, pr, y[0], w, ops)
            fd_c[s:s + B] = (Jp - Jm) / (2 * hc)
            cb = np.broadcast_to(c, (B, n, n))
            Jp = kspace.objective_batch(g, xy, cb, p0 + hp * e, y[0], w, ops)
            Jm = kspace.objective_batch(g, xy, cb, p0 - hp * e, y[0], w, ops)
            fd_p[s:s + B] = (Jp - Jm) / (2 * hp)
    finally:
        kspace.WORKERS = old
    ec = np.linalg.norm(fd_c - gc.ravel()) / np.linalg.norm(gc)
    ep = np.linalg.norm(fd_p - gp0.ravel()) / np.linalg.norm(gp0)
    assert ec < 1e-6, ec
    assert ep < 1e-6, ep


def test_finite_differences_600_steps_sampled_pixels():
    """The same check over 600 time steps (PML on): central differences of J at
    96 seeded pixels of c and of p0 (with the PML cells and the corners among
    them) against the adjoint gradient, per pixel relative to the largest
    gradient entry."""
    n, nt, m = 32, 600, 12
    g, rng, c, p0, xy = _setup(n=n, nt=nt, K=1, m=m, seed=4)
    y = rng.standard_normal((1, nt, m)) * 0.05
    w = 3.0
    data, hist = kspace.forward(g, xy, c, p0)
    r, J = kspace.misfit(data, y, np.array([w]))
    gp0, gc = kspace.adjoint_gradient(g, xy, c, p0, r, hist)
    N = n * n
    pick = np.unique(np.concatenate([[0, n - 1, N - n, N - 1, 2 * n + 1, n * n // 2 + n // 2],
                                     np.random.default_rng(40).choice(N, 90, replace=False)]))
    old = kspace.WORKERS
    kspace.WORKERS = os.cpu_count() or 1
    try:
        ops = kspace.Operators(g)
        e = np.zeros((len(pick), n, n))
        e.reshape(len(pick), N)[np.arange(len(pick)), pick] = 1.0
        hc, hp = 1e-3, 1e-4
        pr = np.broadcast_to(p0, e.shape)
        cb = np.broadcast_to(c, e.shape)
        fd_c = (kspace.objective_batch(g, xy, c[None] + hc * e, pr, y[0], w, ops)
                - kspace.objective_batch(g, xy, c[None] - hc * e, pr, y[0], w, ops)) / (2 * hc)
        fd_p = (kspace.objective_batch(g, xy, cb, p0 + hp * e, y[0], w, ops)
                - kspace.objective_batch(g, xy, cb, p0 - hp * e, y[0], w, ops)) / (2 * hp)
    finally:
        kspace.WORKERS = old
    ec = np.max(np.abs(fd_c - gc.ravel()[pick])) / np.max(np.abs(gc))
    ep = np.max(np.abs(fd_p - gp0.ravel()[pick])) / np.max(np.abs(gp0))
    assert ec < 1e-6, ec
    assert ep < 1e-6, ep
