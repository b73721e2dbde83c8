"""GPU (HIP, float32) vs oracle (float64) parity of the forward map and the
adjoint gradient, through the C ABI.

Bars: sensor data rel-L2 <= 1e-4; gradients g_p0, g_c rel-L2 <= 1e-3 (the
accumulation order of the FFTs differs between the two sides).  Inputs are
rounded to float32 first so both sides see the same numbers.
"""
import dataclasses

import numpy as np
import pytest

from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce, gpu_forward_adjoint, oracle_forward_adjoint, observed_data, rel_l2

pytestmark = pytest.mark.gpu

DATA_TOL = 1e-4
GRAD_TOL = 1e-3


def _reduced(wl, nt=None, K=None, name=None):
    g = wl.grid if nt is None else dataclasses.replace(wl.grid, nt=nt)
    return I.Workload(name or wl.name, g, K=K or wl.K, m=wl.m, sensor_radius_px=wl.sensor_radius_px,
                      support_radius_px=wl.support_radius_px, phys_px=wl.phys_px)


def _parity(wl, config, seed_case=0, c_guess=1500.0):
    c_true, p0 = (a for a in _case(wl, config, seed_case))
    y, w = observed_data(wl, c_true, p0, noise_seed=1000 * config + seed_case + 500)
    c = np.full_like(c_true, np.float32(c_guess)) if c_guess else c_true
    announce(f"{wl.name} oracle")
    ora = oracle_forward_adjoint(wl, c, p0, y=y, w=w)
    announce(f"{wl.name} gpu forward+adjoint K={wl.K} nt={wl.grid.nt} n={wl.grid.nx}x{wl.grid.ny}")
    gpu = gpu_forward_adjoint(wl, c, p0, resid32=ora["resid"].astype(np.float32))
    e_d = rel_l2(gpu["data"], ora["data"])
    e_p = rel_l2(gpu["g_p0"], ora["g_p0"])
    e_c = rel_l2(gpu["g_c"], ora["g_c"])
    print(f"[parity] {wl.name}: data {e_d:.2e}  g_p0 {e_p:.2e}  g_c {e_c:.2e}", flush=True)
    assert e_d <= DATA_TOL, e_d
    assert e_p <= GRAD_TOL, e_p
    assert e_c <= GRAD_TOL, e_c


def _case(wl, config, seed_case):
    c, p0 = I.phantoms(wl, config, case=seed_case)
    return c.astype(np.float32), p0.astype(np.float32)


def test_config1_full_84x84_k1_600_steps():
    _parity(I.config1(), 1)


def test_config2_full_256x256_k4_2000_steps():
    _parity(I.config2(), 2)


def test_config3_level128_full_k8_1000_steps():
    _parity(I.config3_level(128), 3)


def test_config3_level256_k8_500_steps():
    """The 256^2 multigrid level with all 8 datasets on a quarter of its time
    axis (the float64 oracle needs about a minute per 1e9 grid-point steps)."""
    _parity(_reduced(I.config3_level(256), nt=500, name="cfg3_256_K8_nt500"), 3)


def test_radix3_192_k2():
    _parity(_reduced(I.config2(n=192, K=2, nt=160), name="r3_192_K2"), 2)


def test_odd_81_and_125():
    for n in (81, 125):
        g = I.make_grid(n, 1e-4, 120, 8)
        rs = int(round(0.38 * n))
        wl = I.Workload(f"odd_{n}", g, K=3 if n == 81 else 1, m=24, sensor_radius_px=float(rs),
                        support_radius_px=float(rs - 4))
        _parity(wl, 2)


def test_nonsquare_96x64():
    g = I.Grid(nx=96, ny=64, dx=1e-4, dt=I.cfl_dt(1e-4), nt=140, pml=8)
    wl = I.Workload("nonsq_96x64", g, K=2, m=20, sensor_radius_px=20.0, support_radius_px=16.0)
    c_true = np.full((64, 96), 1500.0, dtype=np.float32)
    c_true[20:40, 30:60] = 1560.0
    xs = I.pixel_centres(96)
    ys = I.pixel_centres(64)
    X, Y = np.meshgrid(xs, ys)
    p0 = np.stack([np.exp(-((X - 5) ** 2 + (Y + 3) ** 2) / 8.0),
                   np.exp(-((X + 7) ** 2 + (Y - 4) ** 2) / 8.0)]).astype(np.float32)
    y, w = observed_data(wl, c_true, p0, noise_seed=7)
    c = np.full_like(c_true, np.float32(1500.0))
    ora = oracle_forward_adjoint(wl, c, p0, y=y, w=w)
    announce("nonsq_96x64 gpu")
    gpu = gpu_forward_adjoint(wl, c, p0, resid32=ora["resid"].astype(np.float32))
    assert rel_l2(gpu["data"], ora["data"]) <= DATA_TOL
    assert rel_l2(gpu["g_p0"], ora["g_p0"]) <= GRAD_TOL
    assert rel_l2(gpu["g_c"], ora["g_c"]) <= GRAD_TOL


def test_single_time_sample_and_two_samples():
    """Degenerate time axes: nt = 1 (data = S p0, g_p0 = S^T r, g_c = 0) and nt = 2."""
    for nt in (1, 2):
        wl = _reduced(I.config2(n=64, K=2, nt=nt), name=f"nt{nt}")
        c, _ = _case(wl, 2, 0)
        rng = np.random.default_rng(nt)
        p0 = rng.standard_normal((wl.K, 64, 64)).astype(np.float32)
        resid = rng.standard_normal((wl.K, nt, wl.m))
        from oracle import kspace
        data, hist = kspace.forward(wl.grid, wl.sensors, c.astype(np.float64), p0.astype(np.float64))
        gp0, gc = kspace.adjoint_gradient(wl.grid, wl.sensors, c.astype(np.float64), p0.astype(np.float64),
                                          resid, hist)
        announce(f"nt={nt} gpu")
        gpu = gpu_forward_adjoint(wl, c, p0, resid32=resid.astype(np.float32))
        assert rel_l2(gpu["data"], data) <= DATA_TOL
        assert rel_l2(gpu["g_p0"], gp0) <= GRAD_TOL
        if nt == 1:
            assert np.all(gpu["g_c"] == 0.0)
        else:
            assert rel_l2(gpu["g_c"], gc) <= GRAD_TOL


@pytest.mark.parametrize("level", ["mg1", "mg4"])
def test_paper_geometry_square_array_k4(level):
    """Table 1 grids (81^2: radix 3; 175^2: radix 5 and 7) with the 236-sensor
    square array and the nine-disc stand-in, K = 4, on a shortened time axis."""
    wl0 = I.paper_level(level, K=4)
    wl = dataclasses.replace(wl0, grid=dataclasses.replace(wl0.grid, nt=160), name=f"paper_{level}_K4_nt160")
    c_true, p0 = I.nine_disc_phantom(wl.grid, 4)
    c_true = c_true.astype(np.float32)
    p0 = p0.astype(np.float32)
    y, w = observed_data(wl, c_true, p0, noise_seed=6500)
    c = np.full_like(c_true, np.float32(1505.0))
    announce(f"{wl.name} oracle")
    ora = oracle_forward_adjoint(wl, c, p0, y=y, w=w)
    announce(f"{wl.name} gpu")
    gpu = gpu_forward_adjoint(wl, c, p0, resid32=ora["resid"].astype(np.float32))
    e = (rel_l2(gpu["data"], ora["data"]), rel_l2(gpu["g_p0"], ora["g_p0"]), rel_l2(gpu["g_c"], ora["g_c"]))
    print(f"[parity] {wl.name}: {e}", flush=True)
    assert e[0] <= DATA_TOL and e[1] <= GRAD_TOL and e[2] <= GRAD_TOL
