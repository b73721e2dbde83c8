"""Autotuner of the launch configuration: per grid size and dataset count, the
column-pass tile width (4 or 8 columns per block) and transform order (a
thread's two transforms together or one after the other, or the two arrays
on two halves of a block); per batch, the
stream count.  Measurements are taken on the GPU with short time axes and
cached per (grid, K, GPU architecture) in a JSON file under the user cache
directory (``$PAT_TUNE_CACHE`` overrides the path); choices measured once per
architecture are committed in ``tune_table.json`` (``python -m
paper_2505_08482_amd.tune``), so that runs on the same hardware take the same
configuration.  Tuning never changes results: every candidate computes the
same bits."""
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


TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")
CANDIDATES = ((0, 0), (8, 0), (0, 1), (8, 1), (0, 2))   # (column tile, column transform order)


def _table() -> Dict:
    """Choices measured on each architecture and committed with the library."""
    try:
        with open(TABLE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def launch_for(n: int, K: int, nt_probe: int = 200, force: bool = False) -> Dict[str, int]:
    """Fastest column-pass configuration for an n x n grid with K datasets:
    ``{"tile": 0 | 8, "seq": 0 | 1 | 2}`` (columns per block, and whether a
    thread's two column transforms run together or one after the other, or
    the two arrays run on two halves of a block of twice the threads).
    Taken from the committed table for this architecture, else from the user
    cache, else measured (every candidate computes the same bits)."""
    import torch
    key = f"launch/{_arch()}/{n}/{K}"
    if not force:
        tab = _table()
        if key in tab:
            return {"tile": int(tab[key]["tile"]), "seq": int(tab[key]["seq"])}
        cache = _load()
        if key in cache:
            return {"tile": int(cache[key]["tile"]), "seq": int(cache[key]["seq"])}
    if n not in (32, 64, 128, 256, 512):
        return {"tile": 0, "seq": 0}
    wl = I.config2(n=n, K=K, nt=nt_probe)
    plan = pat.Plan(wl.grid, K, wl.sensors)
    c = torch.full((n, n), 1500.0, device="cuda")
    p0 = torch.rand(plan.field_shape, device="cuda")
    y = torch.zeros(plan.data_shape, device="cuda")
    w = torch.ones(K, device="cuda")
    times = {}
    for tile, seq in CANDIDATES:
        plan.set_tile(tile)
        plan.set_col_order(seq)
        times[(tile, seq)] = _time_gradient(plan, c, p0, y, w)
    plan.close()
    best = min(times, key=times.get)
    cache = _load()
    cache[key] = {"tile": best[0], "seq": best[1], "seconds": {f"{t}/{q}": v for (t, q), v in times.items()}}
    _save(cache)
    return {"tile": best[0], "seq": best[1]}


def tile_for(n: int, K: int, nt_probe: int = 200, force: bool = False) -> int:
    """Column tile width of ``launch_for``."""
    return launch_for(n, K, nt_probe, force)["tile"]


def apply(plan, n: int, K: int) -> Dict[str, int]:
    """Set a plan to the tuned column-pass configuration for its size."""
    cfg = launch_for(n, K)
    plan.set_tile(cfg["tile"])
    plan.set_col_order(cfg["seq"])
    return cfg


def write_table(sizes=((512, 8), (256, 4), (256, 8), (128, 8), (128, 4)), reps: int = 3, out: str = TABLE) -> Dict:
    """Measure every (size, K) on this GPU and write its table entry to ``out``
    (the most frequent choice of ``reps`` measurements, so that noise between
    near-equal candidates does not decide it)."""
    tab = _table()
    for n, K in sizes:
        picks = [launch_for(n, K, force=True) for _ in range(reps)]
        votes = {}
        for p_ in picks:
            votes[(p_["tile"], p_["seq"])] = votes.get((p_["tile"], p_["seq"]), 0) + 1
        (tile, seq), _ = max(votes.items(), key=lambda kv: kv[1])
        tab[f"launch/{_arch()}/{n}/{K}"] = {"tile": tile, "seq": seq, "votes": {f"{t}/{q}": v for (t, q), v in
                                                                                 votes.items()}}
    with open(out, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return tab


def streams_for(jobs, candidates=(1, 2, 3, 4), force: bool = False, label: Optional[str] = None) -> int:
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


if __name__ == "__main__":
    import sys
    print(json.dumps(write_table(out=sys.argv[1] if len(sys.argv) > 1 else TABLE), indent=1))
