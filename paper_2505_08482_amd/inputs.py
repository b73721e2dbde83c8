"""Seeded synthetic inputs: grids, sensor geometry, phantoms and measurement noise.

This module is shared by the tests, the benchmark and the smoke run.  It holds
no arithmetic of the acoustic method itself (no wave propagation, no sensor
interpolation, no gradients): it only describes *where* things are and draws the
seeded random phantoms that stand in for the paper's phantoms, which exist only
in stripped figures or an external dataset (Sec. 4.1.1, Sec. 4.2.1).

Conventions
-----------
* Fields are ``[ny][nx]`` row-major, x fastest.  Pixel ``i`` along an axis of
  length ``n`` sits at ``(i + 1/2 - n/2) * dx``: the origin is the grid centre
  and every multigrid level covers the same physical square ``n * dx``.
* Sensor positions are physical coordinates in metres, ``[m][2]`` = ``(x, y)``.
* The time step follows CFL 0.3 at a fixed reference speed ``c_ref`` (Table 1's
  steps are 0.3 * dz / 1580 m/s; this build uses c_ref = 1600 m/s, the upper end
  of every configured sound-speed range).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

C_REF = 1600.0  # m/s, reference speed of the k-space operator and the CFL rule
RHO0 = 1000.0   # kg/m^3, homogeneous ambient density (eq. (1) has no density term)
CFL = 0.3


@dataclasses.dataclass(frozen=True)
class Grid:
    """One computational grid (FFT grid, PML counted inside nx, ny)."""
    nx: int
    ny: int
    dx: float          # m, same spacing along x and y
    dt: float          # s
    nt: int            # number of time samples t_n = n*dt, n = 0..nt-1
    pml: int           # PML width in grid points on every side (inside nx, ny)
    pml_alpha: float = 2.0   # PML absorption at the outer edge, nepers per grid point
    c_ref: float = C_REF
    rho0: float = RHO0

    @property
    def npts(self) -> int:
        return self.nx * self.ny


def cfl_dt(dx: float, c: float = C_REF, cfl: float = CFL) -> float:
    """Time step from the CFL number: dt = cfl * dx / c."""
    return cfl * dx / c


def make_grid(n: int, dx: float, nt: int, pml: int, pml_alpha: float = 2.0) -> Grid:
    return Grid(nx=n, ny=n, dx=dx, dt=cfl_dt(dx), nt=nt, pml=pml, pml_alpha=pml_alpha)


def pixel_centres(n: int) -> np.ndarray:
    """Pixel-centre coordinates in units of pixels, origin at the grid centre."""
    return np.arange(n, dtype=np.float64) + 0.5 - n / 2.0


def circle_sensors(m: int, radius: float) -> np.ndarray:
    """``m`` sensors evenly spaced on a circle of ``radius`` metres: ``[m][2]``."""
    th = 2.0 * np.pi * np.arange(m, dtype=np.float64) / m
    return np.stack([radius * np.cos(th), radius * np.sin(th)], axis=1)


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    K: int
    m: int
    sensor_radius_px: float      # in pixels of this grid
    support_radius_px: float     # phantom support / reconstruction mask radius
    phys_px: Optional[int] = None  # side of the physical (non-PML) region if PML is outside

    @property
    def sensors(self) -> np.ndarray:
        return circle_sensors(self.m, self.sensor_radius_px * self.grid.dx)


def sensor_radius_px(n: int) -> int:
    return int(round(0.38 * n))


def pml_for(n: int) -> int:
    return 20 if n >= 512 else 10


def config1() -> Workload:
    """64x64 physical grid at 0.1 mm with a 10-point PML outside (84x84 FFT grid),
    K=1, 64 sensors on a 30-px circle, 600 time samples."""
    g = make_grid(84, 1e-4, 600, 10)
    return Workload("cfg1_84x84_K1_nt600", g, K=1, m=64, sensor_radius_px=30.0,
                    support_radius_px=26.0, phys_px=64)


def config2(n: int = 256, K: int = 4, nt: int = 2000) -> Workload:
    g = make_grid(n, 1e-4, nt, pml_for(n))
    rs = sensor_radius_px(n)
    return Workload(f"cfg2_{n}x{n}_K{K}_nt{nt}", g, K=K, m=n, sensor_radius_px=float(rs),
                    support_radius_px=float(rs - 4))


def config3_level(n: int, K: int = 8, m: int = 512, nt: Optional[int] = None) -> Workload:
    """One multigrid level of the 128 -> 256 -> 512 reconstruction.  Every level
    covers the same 51.2 mm square; the sensors sit at the finest level's radius
    (195 px at 0.1 mm = 19.5 mm) so the levels share one physical geometry."""
    dx = 1e-4 * 512 / n
    if nt is None:
        nt = 4000 * n // 512
    g = make_grid(n, dx, nt, pml_for(n))
    r_phys = sensor_radius_px(512) * 1e-4
    rs = r_phys / dx
    return Workload(f"cfg3_{n}x{n}_K{K}_nt{nt}", g, K=K, m=m, sensor_radius_px=rs,
                    support_radius_px=rs - 4.0)


def w1(K: int = 8, nt: int = 4000) -> Workload:
    """Throughput workload: 512^2 FFT grid (PML 20 inside), 0.1 mm, 18.75 ns,
    K datasets, 512 sensors on a 195-px circle."""
    wl = config3_level(512, K=K, nt=nt)
    wl.name = f"w1_512x512_K{K}_nt{nt}"
    return wl


# ---------------------------------------------------------------------------
# Phantom generators (seeded)
# ---------------------------------------------------------------------------

def _uniform_in_disc(rng: np.random.Generator, radius: float) -> Tuple[float, float]:
    while True:
        x, y = rng.uniform(-radius, radius, size=2)
        if x * x + y * y <= radius * radius:
            return float(x), float(y)


def blob_p0(n: int, rng: np.random.Generator, centre_radius_px: float,
            nblobs: int = 3, sigma_px: float = 2.0, amp: float = 1.0,
            phys_px: Optional[int] = None) -> np.ndarray:
    """Sum of ``nblobs`` isotropic Gaussians (std ``sigma_px``), centres uniform in
    the disc of radius ``centre_radius_px``."""
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    out = np.zeros((n, n))
    for _ in range(nblobs):
        cx, cy = _uniform_in_disc(rng, centre_radius_px)
        out += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma_px ** 2))
    return out


def disc_c(n: int, rng: np.random.Generator, centre_radius_px: float,
           background: float = 1500.0, values=(1450.0, 1600.0), radius_px: float = 8.0) -> np.ndarray:
    """Background speed with non-overlapping discs (rejection-sampled centres)."""
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    c = np.full((n, n), background)
    centres: List[Tuple[float, float]] = []
    for v in values:
        while True:
            cx, cy = _uniform_in_disc(rng, centre_radius_px)
            if all((cx - a) ** 2 + (cy - b) ** 2 > (2 * radius_px) ** 2 for a, b in centres):
                break
        centres.append((cx, cy))
        c[(X - cx) ** 2 + (Y - cy) ** 2 <= radius_px ** 2] = v
    return c


def grf_c(n: int, rng: np.random.Generator, support_radius_px: float, corr_px: float,
          lo: float = 1400.0, hi: float = 1600.0, n_ellipses: int = 3,
          background: float = 1500.0, ramp_px: float = 4.0) -> np.ndarray:
    """Smooth Gaussian random field mapped to [lo, hi], plus random ellipses,
    tapered to ``background`` outside the support disc with a cosine ramp."""
    white = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n) * 2.0 * np.pi
    KX, KY = np.meshgrid(k, k)
    # Gaussian smoothing kernel (periodic) of std corr_px, applied in Fourier space
    field = np.real(np.fft.ifft2(np.fft.fft2(white) * np.exp(-0.5 * corr_px ** 2 * (KX ** 2 + KY ** 2))))
    field = (field - field.min()) / (field.max() - field.min())
    c = lo + (hi - lo) * field
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    s = n / 256.0
    for _ in range(n_ellipses):
        a, b = rng.uniform(8.0, 32.0, size=2) * s
        th = rng.uniform(0.0, np.pi)
        v = rng.uniform(lo, hi)
        cx, cy = _uniform_in_disc(rng, support_radius_px)
        xr = (X - cx) * np.cos(th) + (Y - cy) * np.sin(th)
        yr = -(X - cx) * np.sin(th) + (Y - cy) * np.cos(th)
        c[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] = v
    R = np.sqrt(X ** 2 + Y ** 2)
    t = np.clip((R - (support_radius_px - ramp_px)) / ramp_px, 0.0, 1.0)
    w = 0.5 * (1.0 + np.cos(np.pi * t))     # 1 inside, 0 outside the ramp
    return background + w * (c - background)


def vessel_p0(n: int, rng: np.random.Generator, support_radius_px: float,
              nmin: int = 5, nmax: int = 15, half_width_px: float = 1.0) -> np.ndarray:
    """5-15 random line segments ('vessels') of width 2 px, amplitude U(0.5, 1),
    endpoints uniform in the support disc; overlaps take the maximum."""
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    out = np.zeros((n, n))
    nseg = int(rng.integers(nmin, nmax + 1))
    for _ in range(nseg):
        ax, ay = _uniform_in_disc(rng, support_radius_px)
        bx, by = _uniform_in_disc(rng, support_radius_px)
        amp = rng.uniform(0.5, 1.0)
        dx, dy = bx - ax, by - ay
        L2 = dx * dx + dy * dy
        if L2 == 0.0:
            t = np.zeros_like(X)
        else:
            t = np.clip(((X - ax) * dx + (Y - ay) * dy) / L2, 0.0, 1.0)
        d2 = (X - ax - t * dx) ** 2 + (Y - ay - t * dy) ** 2
        out = np.where(d2 <= half_width_px ** 2, np.maximum(out, amp), out)
    return out


def embed_outside_pml(field: np.ndarray, n_total: int, fill: float) -> np.ndarray:
    """Place a physical-region field in the centre of a larger FFT grid."""
    n = field.shape[-1]
    off = (n_total - n) // 2
    out = np.full(field.shape[:-2] + (n_total, n_total), fill, dtype=field.dtype)
    out[..., off:off + n, off:off + n] = field
    return out


def phantoms(wl: Workload, config: int, case: int = 0, p0_kind: Optional[str] = None,
             c_kind: Optional[str] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Sound speed ``c [ny][nx]`` and initial pressures ``p0 [K][ny][nx]`` (float64).

    Seeds: c uses ``1000*config + case``; dataset k (1-based) uses ``+k``."""
    n = wl.grid.nx
    base = 1000 * config + case
    if p0_kind is None:
        p0_kind = "vessel" if config in (2, 4, 5) else "blob"
    if c_kind is None:
        c_kind = "disc" if config == 1 else "grf"
    nphys = wl.phys_px or n
    rs = wl.sensor_radius_px
    if c_kind == "disc":
        c = disc_c(nphys, np.random.default_rng(base), rs - 12.0)
    else:
        c = grf_c(nphys, np.random.default_rng(base), wl.support_radius_px,
                  corr_px=20.0 * nphys / 256.0)
    p0 = np.zeros((wl.K, nphys, nphys))
    for k in range(wl.K):
        rng = np.random.default_rng(base + k + 1)
        if p0_kind == "blob":
            p0[k] = blob_p0(nphys, rng, rs - 6.0, sigma_px=2.0)
        else:
            p0[k] = vessel_p0(nphys, rng, wl.support_radius_px)
    if nphys != n:
        c = embed_outside_pml(c, n, 1500.0)
        p0 = embed_outside_pml(p0, n, 0.0)
    return c, p0


def add_noise(clean: np.ndarray, seed: int, frac: float = 0.01) -> Tuple[np.ndarray, np.ndarray]:
    """Additive zero-mean Gaussian noise with std ``frac`` of each dataset's
    peak-to-peak clean amplitude (Sec. 4.1.1).  ``clean`` is ``[K][nt][m]``.
    Returns ``(noisy, sigma[K])``."""
    rng = np.random.default_rng(seed)
    K = clean.shape[0]
    sigma = np.array([frac * (clean[k].max() - clean[k].min()) for k in range(K)])
    noisy = clean + sigma[:, None, None] * rng.standard_normal(clean.shape)
    return noisy, sigma


def mask_disc(n: int, radius_px: float) -> np.ndarray:
    xc = pixel_centres(n)
    X, Y = np.meshgrid(xc, xc)
    return (X ** 2 + Y ** 2) <= radius_px ** 2
