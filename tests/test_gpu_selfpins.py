"""GPU pins that need no oracle: properties the discrete scheme of Sec. 2.1
has in exact arithmetic, checked on the float32 HIP path through the C ABI
(the recorded pressure history is read with pat_history_field).

* Homogeneous medium at the reference speed, PML off: the k-space scheme is
  exact in time, p^n = IFFT2[cos(c_ref |k| n dt) FFT2 p0].
* Any heterogeneous medium, PML off: the leapfrog recurrence
  (p^{n+1} - 2 p^n + p^{n-1}) / c^2 = -dt^2 L p^n, with L the symmetric
  operator of symbol |k|^2 kappa^2 (the product of the two staggered
  derivatives), conserves
  E^{n+1/2} = 1/2 |(p^{n+1} - p^n) / dt|^2_{1/c^2} + 1/2 (p^{n+1})^T L p^n.

Bars from a float32 emulation of the same recurrence (NumPy complex64 FFTs,
128^2, 400 samples): exact-in-time error 5e-6 (rel-L2 at the last sample),
energy drift 9e-8 of E.  The bars are the data bar 1e-4 for the first and
1e-5 for the second (20x and 100x those figures).
"""
import numpy as np
import pytest

from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce, rel_l2

pytestmark = pytest.mark.gpu

EXACT_TOL = 1e-4
ENERGY_TOL = 1e-5


def _wavenumbers(n, d):
    m = np.fft.fftfreq(n) * n
    return 2.0 * np.pi * m / (n * d)


def _kabs_kappa(g):
    kx = _wavenumbers(g.nx, g.dx)
    ky = _wavenumbers(g.ny, g.dx)
    KX, KY = np.meshgrid(kx, ky)
    kabs = np.sqrt(KX ** 2 + KY ** 2)
    arg = g.c_ref * kabs * g.dt / 2.0
    kappa = np.ones_like(arg)
    nz = arg != 0.0
    kappa[nz] = np.sin(arg[nz]) / arg[nz]
    return kabs, kappa


def _history(wl, c32, p032, levels):
    """GPU pressure fields p^n (float64 copies) at the requested levels."""
    import torch
    from paper_2505_08482_amd import pat
    g = wl.grid
    plan = pat.Plan(g, wl.K, wl.sensors)
    ws = plan.workspace(0)
    c = torch.from_numpy(c32).cuda()
    p0 = torch.from_numpy(p032).cuda()
    data = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
    plan.forward(c, p0, data, ws, record=True)
    torch.cuda.synchronize()
    out = {n: plan.history_field(ws, n).double().cpu().numpy() for n in levels}
    plan.close()
    return out


def _wl(n, K=2, nt=400):
    g = I.Grid(nx=n, ny=n, dx=1e-4, dt=I.cfl_dt(1e-4), nt=nt, pml=0)
    rs = round(0.38 * n)
    return I.Workload(f"pml0_{n}_K{K}_nt{nt}", g, K=K, m=32, sensor_radius_px=float(rs),
                      support_radius_px=float(rs - 4))


@pytest.mark.parametrize("n", [128, 84])
def test_homogeneous_exact_in_time(n):
    """128^2: the power-of-two kernels; 84^2: the any-radix kernels."""
    wl = _wl(n)
    g = wl.grid
    _, p0 = I.phantoms(wl, 2)
    p032 = p0.astype(np.float32)
    c32 = np.full((g.ny, g.nx), np.float32(g.c_ref))
    levels = (1, 2, 100, g.nt - 1)
    announce(f"exact in time {wl.name}")
    hist = _history(wl, c32, p032, levels)
    kabs, _ = _kabs_kappa(g)
    F0 = np.fft.fft2(p032.astype(np.float64))
    for n_ in levels:
        exact = np.fft.ifft2(np.cos(g.c_ref * kabs * n_ * g.dt) * F0).real
        e = rel_l2(hist[n_], exact)
        print(f"[exact-in-time] {wl.name} n={n_}: rel-L2 {e:.2e}", flush=True)
        assert e <= EXACT_TOL, (n_, e)


@pytest.mark.parametrize("n", [128, 84])
def test_energy_conserved_heterogeneous_pml_off(n):
    """The random-field medium of the 256^2 workload's generator at this size
    (1400-1600 m/s plus ellipses) with the PML off."""
    wl = _wl(n)
    g = wl.grid
    c, p0 = I.phantoms(wl, 2)
    c32 = c.astype(np.float32)
    assert np.ptp(c32) > 100.0
    levels = tuple(range(g.nt))
    announce(f"energy invariant {wl.name}")
    hist = _history(wl, c32, p0.astype(np.float32), levels)
    kabs, kappa = _kabs_kappa(g)
    L = (kabs * kappa) ** 2
    inv_c2 = 1.0 / c32.astype(np.float64) ** 2
    E = np.empty((g.nt - 1, wl.K))
    for n_ in range(g.nt - 1):
        a, b = hist[n_], hist[n_ + 1]
        d = b - a
        Lp = np.fft.ifft2(L * np.fft.fft2(a)).real
        E[n_] = 0.5 * np.sum(d * d * inv_c2, axis=(1, 2)) / g.dt ** 2 + 0.5 * np.sum(b * Lp, axis=(1, 2))
    drift = np.max(np.abs(E - E[0]) / E[0])
    print(f"[energy] {wl.name}: E0 {E[0]} max relative drift {drift:.2e}", flush=True)
    assert np.all(E[0] > 0)
    assert drift <= ENERGY_TOL, drift
