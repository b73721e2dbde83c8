"""Point sensors (Sec. 2.2): each datum is the pressure read at one sensor
position.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Reading: the pressure at a sensor is the bilinear interpolation of the four
surrounding cell centres; pixel ``i`` of an axis with ``n`` points sits at
``(i + 1/2 - n/2) * dx``.  The sampling operator is an explicit sparse matrix
``S`` (``m x ny*nx``), and the adjoint source of eq. (5)/(6) is injected with
``S^T``.

Pins (tests/test_oracle_sensors.py): weights are non-negative and sum to one;
a sensor on a cell centre samples that pixel; bilinear interpolation is exact
for affine fields; ``<S x, y> = <x, S^T y>``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def sensor_matrix(nx: int, ny: int, dx: float, xy: np.ndarray) -> sp.csr_matrix:
    """Bilinear sampling matrix for sensors at physical ``xy [m][2]`` (metres)."""
    xy = np.asarray(xy, dtype=np.float64)
    m = xy.shape[0]
    fx = xy[:, 0] / dx + nx / 2.0 - 0.5
    fy = xy[:, 1] / dx + ny / 2.0 - 0.5
    i0 = np.floor(fx).astype(np.int64)
    j0 = np.floor(fy).astype(np.int64)
    if (i0 < 0).any() or (j0 < 0).any() or (i0 + 1 > nx - 1).any() or (j0 + 1 > ny - 1).any():
        raise ValueError("sensor outside the interpolation range of the grid")
    tx = fx - i0
    ty = fy - j0
    rows, cols, vals = [], [], []
    for s in range(m):
        for dj, wy in ((0, 1.0 - ty[s]), (1, ty[s])):
            for di, wx in ((0, 1.0 - tx[s]), (1, tx[s])):
                rows.append(s)
                cols.append((j0[s] + dj) * nx + (i0[s] + di))
                vals.append(wx * wy)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, nx * ny))


def sample(S: sp.csr_matrix, p: np.ndarray) -> np.ndarray:
    """``S p`` for fields ``p [..., ny, nx]`` -> ``[..., m]``."""
    lead = p.shape[:-2]
    flat = p.reshape(-1, p.shape[-2] * p.shape[-1])
    return (S @ flat.T).T.reshape(lead + (S.shape[0],))


def inject(S: sp.csr_matrix, r: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """``S^T r`` for sensor values ``r [..., m]`` -> fields ``[..., ny, nx]``."""
    lead = r.shape[:-1]
    flat = r.reshape(-1, r.shape[-1])
    return (S.T @ flat.T).T.reshape(lead + (ny, nx))
