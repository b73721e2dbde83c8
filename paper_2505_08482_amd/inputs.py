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
  steps are 0.3 * dz / 1580 m/s; here c_ref = 1600 m/s, the upper end
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
    sensor_xy: Optional[np.ndarray] = None   # explicit sensor positions [m][2] (metres)
    square_half: Optional[float] = None      # half side (metres) of a square reconstruction domain

    @property
    def sensors(self) -> np.ndarray:
        if self.sensor_xy is not None:
            return self.sensor_xy
        return circle_sensors(self.m, self.sensor_radius_px * self.grid.dx)

    def mask(self) -> np.ndarray:
        """Reconstruction domain ``[ny][nx]`` (bool): the square of half side
        ``square_half`` if set, else the disc of radius ``support_radius_px``."""
        g = self.grid
        if self.square_half is not None:
            X, Y = np.meshgrid(pixel_centres(g.nx) * g.dx, pixel_centres(g.ny) * g.dx)
            return (np.abs(X) <= self.square_half) & (np.abs(Y) <= self.square_half)
        return mask_disc(g.nx, self.support_radius_px)


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


def data_grid_768(K: int = 8) -> Workload:
    """A data grid finer than the finest reconstruction level (Sec. 4.1.2
    simulates the data on a grid other than the reconstruction grid): 768^2
    over the same 51.2 mm square (0.0667 mm), a 2 mm PML (30 points), the 512
    sensors at the same physical radius (19.5 mm), and 6000 samples at 12.5 ns
    (the same 75 us as the 512^2 level's 4000 at 18.75 ns)."""
    n = 768
    dx = 51.2e-3 / n
    dt = cfl_dt(dx)
    nt = int(round(4000 * cfl_dt(1e-4) / dt))
    g = Grid(nx=n, ny=n, dx=dx, dt=dt, nt=nt, pml=30)
    rs = sensor_radius_px(512) * 1e-4 / dx
    return Workload(f"data768_K{K}_nt{nt}", g, K=K, m=512, sensor_radius_px=rs, support_radius_px=rs - 6.0)


def data_grid_phantoms(wl: Workload, config: int, case: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """The generators of ``phantoms`` drawn directly on a finer data grid, with
    the lengths in pixels scaled by the grid's refinement over 512 (the same
    physical correlation length, blob width and vessel width).  Seeds as in
    ``phantoms``."""
    n = wl.grid.nx
    f = n / 512.0
    base = 1000 * config + case
    c = grf_c(n, np.random.default_rng(base), wl.support_radius_px, corr_px=40.0 * f)
    p0 = np.zeros((wl.K, n, n))
    for k in range(wl.K):
        rng = np.random.default_rng(base + k + 1)
        if config in (2, 4, 5):
            p0[k] = vessel_p0(n, rng, wl.support_radius_px, half_width_px=1.0 * f)
        else:
            p0[k] = blob_p0(n, rng, wl.sensor_radius_px - 6.0 * f, sigma_px=2.0 * f)
    return c, p0


# ---------------------------------------------------------------------------
# The paper's own geometry (Sec. 4, Table 1)
# ---------------------------------------------------------------------------
# Table 1 rows: pixel size dz (m), target pixels Nz, sensor-layer pixels NzS and
# PML pixels NzPML.  The reconstruction grids add both layers on every side
# (Nz + 2 NzS + 2 NzPML = 81, 125, 125, 175, 243); the data row's Nz = 335
# already holds its two 10-pixel sensor layers, so its FFT grid is
# 335 + 2 * 20 = 375.
TABLE1 = {
    "data": (63.7e-6, 335, 10, 20),
    "mg1": (526.3e-6, 39, 2, 19),
    "mg2": (370.4e-6, 55, 4, 31),
    "mg3": (227.3e-6, 89, 4, 14),
    "mg4": (156.3e-6, 129, 6, 17),
    "mg5": (101.0e-6, 199, 8, 14),
}
PAPER_SIDE = 20e-3          # m, side of the square target domain (Sec. 4)
PAPER_SENSOR_OFFSET = 0.2e-3  # m, distance of the sensors from the domain boundary
PAPER_SENSORS = 236
PAPER_DURATION = 21.15e-6   # s, the common time span Nt * dt of Table 1's grids


def paper_grid(name: str) -> Grid:
    """FFT grid of a Table 1 row; the time step follows the CFL rule above
    (c_ref = 1600 m/s) over the table's common duration."""
    dz, nz, ns, npml = TABLE1[name]
    n = nz + 2 * npml + (0 if name == "data" else 2 * ns)
    dt = cfl_dt(dz)
    return Grid(nx=n, ny=n, dx=dz, dt=dt, nt=int(round(PAPER_DURATION / dt)) + 1, pml=npml)


def square_array(m: int = PAPER_SENSORS, side: float = PAPER_SIDE, offset: float = PAPER_SENSOR_OFFSET) -> np.ndarray:
    """``m`` point sensors evenly spaced along the square of side
    ``side + 2 offset`` centred on the origin (``m/4`` per side, the first half
    a spacing from a corner): the planar detection geometry of Sec. 4."""
    if m % 4:
        raise ValueError("the square array needs a multiple of 4 sensors")
    h = side / 2.0 + offset
    per = m // 4
    s = (np.arange(per, dtype=np.float64) + 0.5) * (2.0 * h / per) - h
    sides = [np.stack([s, np.full(per, -h)], 1), np.stack([np.full(per, h), s], 1),
             np.stack([-s, np.full(per, h)], 1), np.stack([np.full(per, -h), -s], 1)]
    return np.concatenate(sides, axis=0)


def paper_level(name: str, K: int) -> Workload:
    """One Table 1 grid with the 236-sensor square array and the 20 mm target square."""
    g = paper_grid(name)
    return Workload(f"paper_{name}_{g.nx}_K{K}", g, K=K, m=PAPER_SENSORS, sensor_radius_px=0.0,
                    support_radius_px=0.0, sensor_xy=square_array(), square_half=PAPER_SIDE / 2.0)


def nine_disc_phantom(grid: Grid, K: int = 4, background: float = 1430.0, inclusion: float = 1580.0,
                      p0_value: float = 10.0, seed: int = 6000) -> Tuple[np.ndarray, np.ndarray]:
    """A synthetic stand-in of the simple phantom of Sec. 4.1.1: nine discs
    (radius 1.5 mm, on a 3 x 3 lattice of pitch 6 mm) at ``inclusion`` in a
    ``background`` medium, and K initial pressures, each three discs (radius
    1 mm, ``p0_value`` Pa) at seeded positions inside the target square
    (dataset k uses ``seed + k``).  The layout is a stand-in, drawn
    analytically on ``grid`` (a pixel belongs to a disc if its centre does)."""
    X, Y = np.meshgrid(pixel_centres(grid.nx) * grid.dx, pixel_centres(grid.ny) * grid.dx)
    c = np.full((grid.ny, grid.nx), background)
    for cx in (-6e-3, 0.0, 6e-3):
        for cy in (-6e-3, 0.0, 6e-3):
            c[(X - cx) ** 2 + (Y - cy) ** 2 <= (1.5e-3) ** 2] = inclusion
    p0 = np.zeros((K, grid.ny, grid.nx))
    for k in range(K):
        rng = np.random.default_rng(seed + k + 1)
        for _ in range(3):
            cx, cy = rng.uniform(-8.5e-3, 8.5e-3, size=2)
            p0[k][(X - cx) ** 2 + (Y - cy) ** 2 <= (1.0e-3) ** 2] = p0_value
    return c, p0


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
