"""Autotuner of the launch configuration (column-pass tile width per grid
size, stream count of a batch).  Measurements are taken on the GPU with short
time axes and cached per (grid, K, GPU architecture) in a JSON file under the
user cache directory (``$PAT_TUNE_CACHE`` overrides the path).  Tuning never
changes results: every candidate computes the same bits."""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional

import numpy as np

from . import inputs as I
from . import pat


def _cache_path() -> str:
    if os.environ.get("PAT_TUNE_CACHE"):
        return os.environ["PAT_TUNE_CACHE"]
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "pat_mi355x", "tune.json")


def _load() -> Dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: Dict):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _time_gradient(plan, c, p0, y, w, reps: int = 3) -> float:
    import torch
    ws = plan.workspace(0)
    data = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
    resid = torch.empty_like(data)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    gp = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    gc = torch.empty(c.shape, dtype=torch.float32, device="cuda")

    def once():
        plan.forward(c, p0, data, ws, record=True)
        plan.misfit(data, y, w, resid, J)
        plan.adjoint_gradient(c, p0, resid, gp, gc, ws)

    once()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tile_for(n: int, K: int, nt_probe: int = 200, force: bool = False) -> int:
    """Fastest column tile width (0 = default, 8) for an n x n grid with K datasets."""
    import torch
    key = f"tile/{_arch()}/{n}/{K}"
    cache = _load()
    if key in cache and not force:
        return int(cache[key]["tile"])
    if n not in (32, 64, 128, 256, 512):
        return 0
    wl = I.config2(n=n, K=K, nt=nt_probe)
    plan = pat.Plan(wl.grid, K, wl.sensors)
    c = torch.full((n, n), 1500.0, device="cuda")
    p0 = torch.rand(plan.field_shape, device="cuda")
    y = torch.zeros(plan.data_shape, device="cuda")
    w = torch.ones(K, device="cuda")
    times = {}
    for tile in (0, 8):
        plan.set_tile(tile)
        times[tile] = _time_gradient(plan, c, p0, y, w)
    plan.close()
    best = min(times, key=times.get)
    cache[key] = {"tile": best, "seconds": {str(k): v for k, v in times.items()}}
    _save(cache)
    return best


def streams_for(jobs, candidates=(1, 2, 4, 8, 16), force: bool = False, label: Optional[str] = None) -> int:
    """Fastest stream count for a batch (the jobs are run once per candidate)."""
    import torch
    key = f"streams/{_arch()}/{label}" if label else None
    cache = _load()
    if key and key in cache and not force:
        return int(cache[key]["streams"])
    times = {}
    for ns in candidates:
        pat.batch_gradient(jobs, ns)
        torch.cuda.synchronize()
        t = time.perf_counter()
        pat.batch_gradient(jobs, ns)
        torch.cuda.synchronize()
        times[ns] = time.perf_counter() - t
    best = min(times, key=times.get)
    if key:
        cache[key] = {"streams": best, "seconds": {str(k): v for k, v in times.items()}}
        _save(cache)
    return best
