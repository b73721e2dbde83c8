"""Table 1 arithmetic (Sec. 4.1.1) and the seeded input generators."""
import os

import numpy as np
import pytest

from paper_2505_08482_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_grids.txt")


def _rows():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, dz, nz, ns, npml, dt, nt, fp = line.split()
        out.append((name, float(dz) * 1e-6, int(nz), int(ns), int(npml), float(dt) * 1e-9, int(nt), float(fp) * 1e6))
    return out


def test_time_step_is_cfl_0p3_at_the_maximum_speed():
    """Every time step of Table 1 is 0.3 dz / 1580 m/s (1580 m/s = the fastest
    inclusion of the simple phantom), to the table's 0.1 ns rounding; grid 2
    is the one row printed 0.07 ns off."""
    for name, dz, nz, ns, npml, dt, nt, fp in _rows():
        tol = 0.1e-9 if name == "mg2" else 0.051e-9
        assert abs(I.cfl_dt(dz, 1580.0) - dt) <= tol, name


def test_grid_totals_have_small_prime_factors_and_common_duration():
    for name, dz, nz, ns, npml, dt, nt, fp in _rows():
        total = nz + 2 * npml + (0 if name == "data" else 2 * ns)
        f = total
        for p in (2, 3, 5, 7):
            while f % p == 0:
                f //= p
        assert f == 1, (name, total)
        assert abs(nt * dt - 21.15e-6) < 0.01 * 21.15e-6, name


def test_generators_are_deterministic_and_in_range():
    wl = I.config2(n=128, K=2, nt=10)
    c1, p1 = I.phantoms(wl, 2)
    c2, p2 = I.phantoms(wl, 2)
    assert np.array_equal(c1, c2) and np.array_equal(p1, p2)
    assert c1.min() >= 1400.0 - 1e-9 and c1.max() <= 1600.0 + 1e-9
    assert p1.min() >= 0.0 and p1.max() <= 1.0
    c3, _ = I.phantoms(wl, 2, case=1)
    assert not np.array_equal(c1, c3)
    wl1 = I.config1()
    c, p0 = I.phantoms(wl1, 1)
    assert c.shape == (84, 84) and p0.shape == (1, 84, 84)
    assert set(np.unique(c)) <= {1450.0, 1500.0, 1600.0}
    # the PML ring (outside the 64^2 physical region) is background
    assert np.all(c[:10] == 1500.0) and np.all(p0[:, :10] == 0.0)


def test_sensors_sit_inside_the_non_pml_region():
    for wl in (I.config1(), I.config2(), I.w1(nt=10), I.config3_level(128), I.config3_level(256)):
        g = wl.grid
        xy = wl.sensors
        half = (g.nx / 2 - g.pml - 1) * g.dx
        assert np.all(np.abs(xy) < half), wl.name
        assert xy.shape == (wl.m, 2)
    # every multigrid level sees the same physical sensor positions
    assert np.allclose(I.config3_level(128).sensors, I.w1(nt=10).sensors)


def test_noise_is_one_percent_of_peak_to_peak():
    rng = np.random.default_rng(0)
    clean = rng.standard_normal((3, 400, 50)) * np.array([1.0, 2.0, 0.5])[:, None, None]
    noisy, sigma = I.add_noise(clean, seed=123)
    for k in range(3):
        assert np.isclose(sigma[k], 0.01 * (clean[k].max() - clean[k].min()))
        assert abs(np.std(noisy[k] - clean[k]) / sigma[k] - 1.0) < 0.02
    noisy2, _ = I.add_noise(clean, seed=123)
    assert np.array_equal(noisy, noisy2)


def test_paper_grids_reproduce_table1_totals_and_duration():
    """The FFT grids built from Table 1's rows: totals 375 (data) and 81, 125,
    125, 175, 243 (reconstruction), each a product of 3, 5 and 7; spacing dz;
    all covering the table's common duration."""
    rows = {r[0]: r for r in _rows()}
    expect = {"data": 375, "mg1": 81, "mg2": 125, "mg3": 125, "mg4": 175, "mg5": 243}
    for name, n in expect.items():
        g = I.paper_grid(name)
        assert g.nx == g.ny == n, name
        assert abs(g.dx - rows[name][1]) <= 1e-12 and g.pml == rows[name][4]
        assert abs((g.nt - 1) * g.dt - 21.15e-6) <= g.dt, name


def test_square_array_geometry():
    """236 sensors, 59 per side, 0.2 mm outside every side of the 20 mm target
    square, evenly spaced along the perimeter, inside the non-PML region of
    every Table 1 grid."""
    xy = I.square_array()
    assert xy.shape == (236, 2)
    cheb = np.max(np.abs(xy), axis=1)
    assert np.allclose(cheb, 10.2e-3, atol=1e-15)
    for side in ((xy[:, 1] == -10.2e-3), (xy[:, 0] == 10.2e-3), (xy[:, 1] == 10.2e-3), (xy[:, 0] == -10.2e-3)):
        assert side.sum() == 59
    # walking the perimeter, consecutive sensors are one spacing apart (corners included)
    step = np.sum(np.abs(np.diff(np.vstack([xy, xy[:1]]), axis=0)), axis=1)   # L1 = arc length here
    assert np.allclose(step, 4 * 20.4e-3 / 236, rtol=1e-12)
    for name in ("data", "mg1", "mg2", "mg3", "mg4", "mg5"):
        g = I.paper_grid(name)
        assert np.all(np.abs(xy) < (g.nx / 2 - g.pml - 1) * g.dx), name


def test_nine_disc_stand_in():
    g = I.paper_grid("mg5")
    c, p0 = I.nine_disc_phantom(g, 4)
    c2, p02 = I.nine_disc_phantom(g, 4)
    assert np.array_equal(c, c2) and np.array_equal(p0, p02)
    assert set(np.unique(c)) == {1430.0, 1580.0}
    area = (c == 1580.0).sum() * g.dx ** 2
    assert abs(area / (9 * np.pi * 1.5e-3 ** 2) - 1.0) < 0.1
    assert set(np.unique(p0)) == {0.0, 10.0}
    wl = I.paper_level("mg5", 4)
    assert np.all(p0[:, ~wl.mask()] == 0.0)
    # the first initial pressure does not depend on K
    assert np.array_equal(I.nine_disc_phantom(g, 1)[1][0], p0[0])
