"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
oracle on the same float32-rounded inputs."""
import sys

import numpy as np

from oracle import kspace
from paper_2505_08482_amd import inputs as I

# the oracle's FFTs use this process's CPU share (at most 16 threads)
try:
    import os as _os
    kspace.WORKERS = max(1, min(16, len(_os.sched_getaffinity(0))))
except (AttributeError, OSError):
    kspace.WORKERS = 1


def announce(msg: str) -> None:
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_case(wl, config=2, seed_case=0, c_scale=1.0):
    """float32-rounded c, p0, and a residual from data of a different c."""
    c, p0 = I.phantoms(wl, config, case=seed_case)
    c32 = c.astype(np.float32)
    p032 = p0.astype(np.float32)
    return c32, p032


def gpu_forward_adjoint(wl, c32, p032, resid32=None, ckpt_every=0, torch=None):
    import torch as _t
    from paper_2505_08482_amd import pat
    torch = torch or _t
    g = wl.grid
    plan = pat.Plan(g, wl.K, wl.sensors)
    dev = "cuda"
    c = torch.from_numpy(c32).to(dev)
    p0 = torch.from_numpy(p032).to(dev)
    data = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    ws = plan.workspace(ckpt_every)
    plan.forward(c, p0, data, ws, ckpt_every=ckpt_every, record=True)
    out = {"data": data.cpu().numpy()}
    if resid32 is not None:
        r = torch.from_numpy(np.ascontiguousarray(resid32)).to(dev)
        gp0 = torch.empty(plan.field_shape, dtype=torch.float32, device=dev)
        gc = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)
        plan.adjoint_gradient(c, p0, r, gp0, gc, ws)
        out["g_p0"] = gp0.cpu().numpy()
        out["g_c"] = gc.cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    return out


def oracle_forward_adjoint(wl, c32, p032, y=None, w=None):
    """Oracle data; if ``y`` is given also the misfit residual and gradients."""
    g = wl.grid
    c = c32.astype(np.float64)
    p0 = p032.astype(np.float64)
    data, hist = kspace.forward(g, wl.sensors, c, p0, record=y is not None)
    out = {"data": data}
    if y is not None:
        resid, J = kspace.misfit(data, y, w)
        gp0, gc = kspace.adjoint_gradient(g, wl.sensors, c, p0, resid, hist)
        out.update(resid=resid, J=J, g_p0=gp0, g_c=gc)
    return out


def observed_data(wl, c_true32, p032, noise_seed):
    """Noisy data of the true medium (oracle forward + 1 % noise)."""
    clean, _ = kspace.forward(wl.grid, wl.sensors, c_true32.astype(np.float64), p032.astype(np.float64),
                              record=False)
    y, sigma = I.add_noise(clean, noise_seed)
    return y, 1.0 / sigma


# Bars of the GPU (float32) vs oracle (float64) comparison.  Whole arrays:
# sensor data rel-L2 <= 1e-4, gradients rel-L2 <= 1e-3.  Local checks beside
# them, so that one wrong trace or one wrong band of pixels cannot hide under a
# global norm: every sensor trace whose norm is at least a tenth of the rms
# trace norm within 1e-3 of its own norm, and the largest gradient error
# within 1e-3 of the largest gradient entry (observed float32 errors are
# 1e-6..1e-5 of the whole-array norms, so both leave a factor of 100 or more).
DATA_TOL = 1e-4
GRAD_TOL = 1e-3
TRACE_TOL = 1e-3
MAXABS_TOL = 1e-3


def trace_errors(gpu_data, ora_data):
    """Per-trace relative errors ``|d_gpu - d_ora| / |d_ora|`` over time for the
    traces ``[K][m]`` whose norm is at least 0.1 of the rms trace norm."""
    a = np.asarray(gpu_data, dtype=np.float64)
    b = np.asarray(ora_data, dtype=np.float64)
    nb = np.sqrt(np.sum(b * b, axis=1))              # [K][m]
    ne = np.sqrt(np.sum((a - b) ** 2, axis=1))
    sel = nb >= 0.1 * np.sqrt(np.mean(nb * nb))
    return ne[sel] / nb[sel]


def max_ratio(a, b) -> float:
    """``max |a - b| / max |b|``; for stacked fields ``[K][ny][nx]`` the largest
    of the per-field ratios."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 3:
        return max(max_ratio(a[k], b[k]) for k in range(b.shape[0]))
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check_parity(tag, gpu, ora, keys=("data", "g_p0", "g_c")):
    """Assert the whole-array and the local bars for the given outputs; prints
    every figure first (one line, flushed)."""
    out = {}
    if "data" in keys:
        out["data"] = rel_l2(gpu["data"], ora["data"])
        out["trace_max"] = float(np.max(trace_errors(gpu["data"], ora["data"])))
    for k in ("g_p0", "g_c"):
        if k in keys:
            out[k] = rel_l2(gpu[k], ora[k])
            out[k + "_max"] = max_ratio(gpu[k], ora[k])
    print(f"[parity] {tag}: " + "  ".join(f"{k} {v:.2e}" for k, v in out.items()), flush=True)
    if "data" in keys:
        assert out["data"] <= DATA_TOL, (tag, out)
        assert out["trace_max"] <= TRACE_TOL, (tag, out)
    for k in ("g_p0", "g_c"):
        if k in keys:
            assert out[k] <= GRAD_TOL, (tag, out)
            assert out[k + "_max"] <= MAXABS_TOL, (tag, out)
    return out
