#!/usr/bin/env python3
"""Throughput of the hot path: one objective + gradient evaluation (K recorded
forward solves, the data misfit, K adjoint solves accumulating g_p0 and g_c)
on the 512^2 x 8-dataset workload, 4000 time samples, float32, one GPU.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--nt 4000] [--ckpt S]
                    [--no-cpu] [--cpu-steps 100]

Prints ONE JSON line.  ``value`` is grid-pt-steps/s = K * N^2 * Nt / (seconds
per evaluation), inputs resident in HBM.  ``roofline`` is the dominant fused
pass: algorithmic bytes per launch (bytes per grid point x K N^2) divided by
its average launch duration, timed with start/stop HIP events attached to
sampled dispatches on the launch stream in one evaluation launched kernel by
kernel right after the timed (graph-replayed) ones; ``traffic`` is the measured
HBM bytes per launch (rocprofv3 counters, stored with a digest of the kernel
sources) over the same duration.  ``cpu_baseline`` times the float64 oracle on
this host's cores on a bounded sample of the same workload (100 time samples).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2505_08482_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Bytes per grid point and launch of each fused pass (float32 state, half
# spectra along x count 4 B/pt, c amortised over the K datasets).  Two counts
# differ only in the adjoint density pass:
# * algorithmic (what the method must move): the g_c accumulator is read and
#   written once per time step for all K datasets, 8 / K B/pt;
# * moved by this implementation: its blocks hold ADJ_KB datasets each, so the
#   g_c slice is read and written once per ADJ_KB datasets, 8 / ADJ_KB B/pt.
ADJ_KB = 4      # datasets per block of that pass at K >= 4


def progress(msg: str) -> None:
    """One line per finished step on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def pass_bytes(K: int, moved: bool = False) -> dict:
    """Bytes per grid point of each pass: algorithmic, or (``moved``) what the
    kernels move with their dataset grouping."""
    kb = ADJ_KB if K >= 4 else (2 if K >= 2 else 1)
    gc_rw = 8.0 / kb if moved else 8.0 / K
    c_amort = 4.0 / K
    return {
        # r spectrum 4; w 2 spectra 8
        "fwd_col_grad": 12.0,
        # r 2 spectra 8 + u_x, u_y 8; w u_x, u_y 8 + 2 spectra 8
        "fwd_row_u": 32.0,
        # r 2 spectra 8; w 2 spectra 8
        "fwd_col_div": 16.0,
        # r 2 spectra 8 + rho_x, rho_y 8 + c; w rho_x, rho_y 8 + history p 4 + spectrum of p 4
        "fwd_row_rho": 32.0 + c_amort,
        # r 2 spectra 8; w 1 spectrum 4
        "adj_col_summ": 12.0,
        # r spectrum 4 + rho^ 8 + history p 4 + c + g_c; w rho^ 8 + g_c + 2 spectra 8
        "adj_row_rho": 32.0 + c_amort + gc_rw,
        # r 2 spectra 8; w 2 spectra 8
        "adj_col_grad": 16.0,
        # r 2 spectra 8 + u^ 8; w u^ 8 + 2 spectra 8
        "adj_row_u": 32.0,
    }


PASS_BYTES = pass_bytes(8)
STEP_BYTES = sum(PASS_BYTES.values())   # per grid point and time step, forward + adjoint

# Measured HBM bytes per launch of the pass kinds (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, scaled by what the same counters read for a plain copy of known
# size), valid only for the kernel sources they were taken on.
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2505_08482_amd", "traffic.json")
KERNEL_SOURCES = ("fast_kernels.hpp", "wave_kernels.hpp", "fft_lds.hpp", "vec_kernels.hpp", "pat_api.hip")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(os.path.dirname(TRAFFIC_FILE), "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kind: str, wl_name: str):
    """Bytes per launch of pass ``kind`` at workload ``wl_name`` from the stored
    counter readings, or None when they are missing or the kernels changed."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_digest() or t.get("workload") != wl_name:
        return None
    e = t.get("passes", {}).get(kind)
    if not e:
        return None
    return e["fetch_kib"] * 1024.0 * t["fetch_scale"] + e["write_kib"] * 1024.0 * t["write_scale"]


def cpu_cores() -> int:
    """Threads this process may run: its CPU affinity set, or the thread budget
    the host gives it in OMP_NUM_THREADS if that is smaller (a shared host's
    share of cores; os.cpu_count() counts cores that belong to other jobs)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nt_sample: int, K: int, cores: int = 0) -> dict:
    """The float64 oracle, as it stands, on the W1 grid for nt_sample time samples
    (on ``cores`` threads; 0 = every thread this process may run)."""
    from oracle import kspace
    cores = cores or cpu_cores()
    kspace.WORKERS = cores
    wl = I.w1(K=K, nt=nt_sample)
    c, p0 = I.phantoms(wl, 3)
    rng = np.random.default_rng(3500)
    t0 = time.perf_counter()
    data, hist = kspace.forward(wl.grid, wl.sensors, np.full_like(c, 1500.0), p0)
    resid = rng.standard_normal(data.shape)
    kspace.adjoint_gradient(wl.grid, wl.sensors, np.full_like(c, 1500.0), p0, resid, hist)
    dt = time.perf_counter() - t0
    pts = K * wl.grid.nx * wl.grid.ny * nt_sample
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    # the oracle's cost is linear in the number of time samples: the full
    # 4000-sample evaluation is this sample's time scaled by 4000 / nt_sample
    return {"value": pts / dt, "unit": "grid-pt-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 oracle (numpy + scipy.fft, {cores} threads), forward + adjoint on the "
                      f"512x512 grid, K={K}, {nt_sample} time samples ({dt:.1f} s)",
            "extrapolated_eval_seconds_nt4000": round(dt * 4000.0 / nt_sample, 1),
            "extrapolation": f"linear in the number of time samples, {nt_sample} -> 4000 (extrapolated)",
            "host": {"cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity,
                     "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}}


def forward_only(plan, wl, c, p0, data, ws, reps=2):
    """Rate of the K forward solves alone (store-all recording, as in an evaluation)."""
    import torch
    g = wl.grid
    plan.forward(c, p0, data, ws, record=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        plan.forward(c, p0, data, ws, record=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    return {"value": wl.K * g.nx * g.ny * g.nt / dt, "unit": "grid-pt-steps/s", "ms": round(1000.0 * dt, 2)}


def bandwidth_probe():
    """Achievable memory bandwidth on this GPU for context: device copies and
    fills of buffers that fit the Infinity Cache (64 MB) and that do not (2 GB)."""
    import torch
    out = {}
    for mb in (64, 2048):
        n = mb * (1 << 20) // 4
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        for name, fn, nbytes in (("copy", lambda: y.copy_(x), 2 * 4 * n), ("fill", lambda: y.fill_(1.5), 4 * n)):
            fn()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(20):
                fn()
            e.record()
            torch.cuda.synchronize()
            out[f"{name}_{mb}MB_GBps"] = round(nbytes * 20 / (s.elapsed_time(e) / 1000.0) / 1e9, 1)
        del x, y
        torch.cuda.empty_cache()
    return out


def paper_geometry(iters: int = 40, levels=("mg1", "mg2", "mg3", "mg4")):
    """The paper's own set-up (Sec. 4, Table 1): 236 sensors on the square around
    the 20 mm target, the nine-disc stand-in phantom with four initial pressures,
    data simulated on the 375^2 data grid (not a reconstruction grid) with 1 %
    noise, and multigrid reconstructions over Table 1's grids 1-4 with all four
    datasets (K = 4) and with the first alone (K = 1, the paper's reference
    approach), each with bounds only and with the paper's Ornstein-Uhlenbeck
    prior; c in [1300, 1800] m/s, starting at 1505 m/s, 1430 m/s held outside
    the target square.  E_c and E_p0 of dataset 1 on the finest level."""
    import torch
    from paper_2505_08482_amd import pat, recon
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    wd = I.paper_level("data", K=4)
    cd, p0d = I.nine_disc_phantom(wd.grid, 4)
    plan = pat.Plan(wd.grid, 4, wd.sensors)
    ws = plan.workspace(0)
    data = torch.empty(plan.data_shape, device="cuda")
    t = time.perf_counter()
    plan.forward(T(cd), T(p0d), data, ws, record=False)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t
    plan.close()
    del ws
    noisy, sigma = I.add_noise(data.cpu().numpy().astype(np.float64), seed=6500)
    del data
    torch.cuda.empty_cache()
    out = {"data_grid": wd.grid.nx, "data_nt": wd.grid.nt, "data_seconds": round(t_data, 3),
           "sensors": wd.m, "levels": [I.paper_grid(n).nx for n in levels], "iters_per_level": iters}
    # the paper's prior (Sec. 4.1.2): tau = 1.5 mm, means at the middle and standard
    # deviations a quarter of the true ranges (p0 in [0, 10] Pa, c in [1430, 1580] m/s)
    ou = {"tau": 1.5e-3, "eta_p0": 5.0, "sigma_p0": 2.5, "eta_c": 1505.0, "sigma_c": 37.5}
    for K, use_prior in ((4, False), (1, False), (4, True), (1, True)):
        lv = [I.paper_level(n, K) for n in levels]
        t = time.perf_counter()
        res = recon.multigrid(lv, T(noisy[:K]), wd.grid.dt, T(1.0 / sigma[:K]),
                              lambda wl: T(I.nine_disc_phantom(wl.grid, 1)[0]), c_lo=1300.0, c_hi=1800.0,
                              iters=iters, c_init=1505.0, c_fixed=1430.0, prior=ou if use_prior else None)
        secs = time.perf_counter() - t
        fine = lv[-1]
        p0t = I.nine_disc_phantom(fine.grid, 1)[1][0]
        m = fine.mask()
        p0r = res["p0"][0].cpu().numpy().astype(np.float64)
        e_p0 = 100.0 * float(np.linalg.norm((p0r - p0t)[m]) / np.linalg.norm(p0t[m]))
        out[f"K{K}" + ("_ou_prior" if use_prior else "")] = {"E_c_percent": round(res["E_c"], 3), "E_p0_1_percent": round(e_p0, 2),
                        "seconds": round(secs, 2), "iterations": [r.iters for r in res["levels"]],
                        "evals": [r.evals for r in res["levels"]]}
    return out


def checkpointed(plan, wl, c, p0, y, w, evaluation_ms, s=64):
    """The same evaluation with checkpoints every s steps and segment recompute."""
    import torch
    g = wl.grid
    ws = plan.workspace(s)
    data = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
    resid = torch.empty_like(data)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    gp = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    gc = torch.empty((g.ny, g.nx), dtype=torch.float32, device="cuda")

    def ev():
        plan.forward(c, p0, data, ws, ckpt_every=s, record=True)
        plan.misfit(data, y, w, resid, J)
        plan.adjoint_gradient(c, p0, resid, gp, gc, ws)

    ev()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ev()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    pts = wl.K * g.nx * g.ny * g.nt
    return {"ckpt_every": s, "ms_per_step": 1000.0 * dt, "value": pts / dt, "unit": "grid-pt-steps/s",
            "workspace_GB": round(plan.workspace_size(s) / 1e9, 2),
            "store_all_workspace_GB": round(plan.workspace_size(0) / 1e9, 2),
            "slowdown_vs_store_all": round(1000.0 * dt / evaluation_ms, 3)}


def batch_w3(evals: int):
    """32 independent problems (grids 128/192/256, K 1/2/4, 1000-2000 steps,
    seed 4000), `evals` objective+gradient evaluations each: one batched call
    per round against the same work run problem by problem."""
    import torch
    from paper_2505_08482_amd import pat, tune
    rng = np.random.default_rng(4000)
    jobs = []
    for i in range(32):
        n = int(rng.choice([128, 192, 256]))
        K = int(rng.choice([1, 2, 4]))
        nt = int(rng.integers(1000, 2001))
        wl = I.config2(n=n, K=K, nt=nt)
        c_true, p0 = I.phantoms(wl, 4, case=i)
        plan = pat.Plan(wl.grid, K, wl.sensors)
        tune.apply(plan, n, K)
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
        j = {"plan": plan, "c": T(np.full_like(c_true, 1500.0)), "p0": T(p0), "ws": plan.workspace(0),
             "data": torch.empty(plan.data_shape, device="cuda"), "w": T(np.full(K, 100.0))}
        plan.forward(T(c_true), j["p0"], j["data"], j["ws"], record=False)
        j["y"] = j["data"].clone()
        j["resid"] = torch.empty_like(j["data"])
        j["J"] = torch.zeros(1, dtype=torch.float64, device="cuda")
        j["g_p0"] = torch.empty(plan.field_shape, device="cuda")
        j["g_c"] = torch.empty((n, n), device="cuda")
        jobs.append(j)
    pts = sum(j["plan"].K * j["plan"].grid.nx * j["plan"].grid.ny * j["plan"].grid.nt for j in jobs) * evals

    def sequential():
        for j in jobs:
            p = j["plan"]
            p.forward(j["c"], j["p0"], j["data"], j["ws"], record=True)
            p.misfit(j["data"], j["y"], j["w"], j["resid"], j["J"])
            p.adjoint_gradient(j["c"], j["p0"], j["resid"], j["g_p0"], j["g_c"], j["ws"])

    sequential()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(evals):
        sequential()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    ref = [(j["g_c"].clone(), j["g_p0"].clone(), j["J"].clone()) for j in jobs]
    ns = tune.streams_for(jobs, label="w3_seed4000")
    t = time.perf_counter()
    for _ in range(evals):
        pat.batch_gradient(jobs, ns)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t
    same = all(torch.equal(j["g_c"], r[0]) and torch.equal(j["g_p0"], r[1]) and torch.equal(j["J"], r[2])
               for j, r in zip(jobs, ref))
    classes = sorted({j["plan"].grid.nx for j in jobs})
    for j in jobs:
        j["plan"].close()
    return {"problems": 32, "evals_each": evals, "streams": ns, "classes": classes,
            "batched_value": pts / t_bat, "sequential_value": pts / t_seq, "unit": "grid-pt-steps/s",
            "speedup": round(t_seq / t_bat, 3), "seconds_batched": round(t_bat, 3),
            "seconds_sequential": round(t_seq, 3), "batched_equals_sequential_bitwise": bool(same),
            "schedule": "problems of one grid size share every launch (one launch per pass), forward solves "
                        "aligned at their ends and adjoint solves at their starts, captured step-chunk graphs "
                        "per active set, one stream per grid size"}


def time_to_solution(wl_fine, c_true, y_fine, w, iters: int, target: float = 2.0):
    """Multigrid 128 -> 256 -> 512 reconstruction (K datasets, c in [1400, 1600],
    p0 >= 0): wall time and iterations until E_c over the mask <= target %."""
    import torch
    from paper_2505_08482_amd import recon
    levels = [I.config3_level(128, K=wl_fine.K), I.config3_level(256, K=wl_fine.K), wl_fine]
    log = []
    t0 = time.perf_counter()
    reached = {}

    def cb(msg):
        log.append(msg)

    out = recon.multigrid(levels, y_fine, wl_fine.grid.dt, w, c_true, iters=iters, log=cb)
    total = time.perf_counter() - t0
    # the target is judged on the finest level (E_c of coarse levels is measured
    # against the resampled truth and is only reported); the time is wall clock
    # from the start of the run (level set-up, plans and data resampling included)
    fine = out["levels"][-1]
    its_before = sum(lv.iters for lv in out["levels"][:-1])
    for i, (e, tt) in enumerate(zip(fine.E_c, fine.t)):
        if e <= target:
            reached = {"level": fine.n, "iteration_at_level": i + 1, "iterations_total": its_before + i + 1,
                       "seconds": round(fine.t_start + tt, 2)}
            break
    # the same criterion on any level (E_c of a coarse level against the truth resampled onto it)
    reached_any = {}
    its = 0
    for lv in out["levels"]:
        hit = next((i for i, e in enumerate(lv.E_c) if e <= target), None)
        if hit is not None:
            reached_any = {"level": lv.n, "iteration_at_level": hit + 1, "iterations_total": its + hit + 1,
                           "seconds": round(lv.t_start + lv.t[hit], 2)}
            break
        its += lv.iters
    return {"target_E_c_percent": target, "reached": reached or None, "reached_any_level": reached_any or None,
            "final_E_c_percent": round(out["E_c"], 3),
            "total_seconds": round(total, 2),
            "levels": [{"n": lv.n, "iters": lv.iters, "evals": lv.evals, "seconds": round(lv.seconds, 2),
                        "E_c_first": round(lv.E_c[0], 3) if lv.E_c else None,
                        "E_c_last": round(lv.E_c[-1], 3) if lv.E_c else None} for lv in out["levels"]]}


def time_to_solution_finer_data(K: int, iters: int, target: float = 2.0):
    """The same multigrid reconstruction with data simulated on the finer 768^2
    grid (inputs.data_grid_768: no inverse crime), phantoms of the throughput
    workload's generators drawn on that grid (seeds 3000-3008, noise 3500);
    E_c against the true sound speed interpolated to each level."""
    import torch
    from paper_2505_08482_amd import pat
    dw = I.data_grid_768(K=K)
    c_np, p0_np = I.data_grid_phantoms(dw, 3)
    plan = pat.Plan(dw.grid, K, dw.sensors)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    data = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
    ws = plan.workspace(0)
    t0 = time.perf_counter()
    plan.forward(T(c_np), T(p0_np), data, ws, record=False)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    del ws
    plan.close()
    y_np, sigma = I.add_noise(data.cpu().numpy().astype(np.float64), seed=3500)
    y = T(y_np)
    w = T(1.0 / sigma)
    c_data = T(c_np).reshape(1, dw.grid.ny, dw.grid.nx)

    def truth(level):
        out = torch.empty((1, level.grid.ny, level.grid.nx), dtype=torch.float32, device="cuda")
        pat.prolong_phys(c_data, dw.grid.dx, out, level.grid.dx)
        return out[0]

    from paper_2505_08482_amd import recon
    levels = [I.config3_level(n, K=K) for n in (128, 256, 512)]
    t0 = time.perf_counter()
    out = recon.multigrid(levels, y, dw.grid.dt, w, truth, iters=iters)
    total = time.perf_counter() - t0
    res = {"data_grid": dw.grid.nx, "data_nt": dw.grid.nt, "data_seconds": round(t_data, 2),
           "data_rate_grid_pt_steps_per_s": round(K * dw.grid.nx * dw.grid.ny * dw.grid.nt / t_data, 1),
           "target_E_c_percent": target, "final_E_c_percent": round(out["E_c"], 3),
           "total_seconds": round(total, 2), "reached": None,
           "levels": [{"n": lv.n, "iters": lv.iters, "evals": lv.evals, "seconds": round(lv.seconds, 2),
                       "E_c_first": round(lv.E_c[0], 3) if lv.E_c else None,
                       "E_c_last": round(lv.E_c[-1], 3) if lv.E_c else None} for lv in out["levels"]]}
    its = 0
    for lv in out["levels"]:
        hit = next((i for i, e in enumerate(lv.E_c) if e <= target), None)
        if hit is not None and lv.n == 512:
            res["reached"] = {"level": lv.n, "iteration_at_level": hit + 1, "iterations_total": its + hit + 1,
                              "seconds": round(lv.t_start + lv.t[hit], 2)}
            break
        its += lv.iters
    return res


def network_timing():
    """The learned start's network at the fine-level size (512^2, batch 4):
    forward and training-step times, convolution flop rates, and the forward
    against the sum over its layers of max(flops / MFMA peak, bytes / HBM peak)."""
    from paper_2505_08482_amd import learned
    return learned.time_network(4, 5)


def learned_start(cases, fine_iters: int = 20, targets=(2.0, 1.0), data_grid: int = 512):
    """Held-out phantoms (the 256^2 workload's generators at 512^2, K = 8,
    seeds 5000 + case): plain multigrid 128 -> 256 -> 512 against the coarse
    level followed by the fine level started from the trained network's
    proposal (and, for the gain of the network alone, from the plain
    interpolation of the same coarse iterate).  Iterations and wall time from
    the start of each run to E_c <= each target on the finest grid.
    ``data_grid = 768``: the phantoms and data on the finer 768^2 grid."""
    import os as _os
    from paper_2505_08482_amd import learned
    if not _os.path.exists(learned.DEFAULT_WEIGHTS):
        return {"error": "no trained weights in the package"}
    net = learned.load_weights(learned.DEFAULT_WEIGHTS)
    rows = [learned.evaluate_case(net, c, fine_iters=fine_iters, targets=targets, data_grid=data_grid,
                                  log=lambda m: progress("learned_start " + m)) for c in cases]
    summary = {}
    for run in ("plain_multigrid", "interpolated", "learned"):
        for tg in targets:
            hits = [r[run]["to_target"][f"{tg:g}"] for r in rows]
            ok = [h for h in hits if h is not None]
            summary[f"{run}@{tg:g}%"] = {
                "reached": f"{len(ok)}/{len(rows)}",
                "mean_seconds": round(float(np.mean([h["seconds"] for h in ok])), 2) if ok else None,
                "mean_iterations": round(float(np.mean([h["iterations"] for h in ok])), 1) if ok else None}
    for r in rows:            # keep the JSON line short: trajectories stay in the rows' summaries
        for run in ("plain_multigrid", "interpolated", "learned"):
            r[run].pop("t", None)
    return {"data_grid": data_grid, "targets_E_c_percent": list(targets), "cases": list(cases), "summary": summary,
            "mean_E_c_fine_start": {k: round(float(np.mean([r[k]["E_c_start"] for r in rows])), 3)
                                    for k in ("interpolated", "learned")},
            "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--ckpt", type=int, default=0, help="checkpoint interval (0 = store the whole history)")
    ap.add_argument("--tile", default="auto", choices=("auto", "0", "8"),
                    help="column-pass tile width (auto: the autotuner's choice)")
    ap.add_argument("--col-order", default="auto", choices=("auto", "0", "1", "2"),
                    help="column-pass transform order (0 together, 1 one after the other, 2 split over two "
                         "half-blocks; auto: the autotuner's choice)")
    ap.add_argument("--trace-every", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the checkpointed, batch and time-to-solution measurements")
    ap.add_argument("--batch-evals", type=int, default=5)
    ap.add_argument("--tts-iters", type=int, default=40)
    ap.add_argument("--learned-cases", type=int, default=2,
                    help="held-out phantoms for the learned-start comparison (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the datasets would shard across GPUs with one all-reduce of g_c per gradient, which is not "
              "built here", file=sys.stderr)
        return 2

    import torch
    from paper_2505_08482_amd import pat

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = "cuda"
    wl = I.w1(K=args.K, nt=args.nt)
    g = wl.grid
    c_true, p0 = I.phantoms(wl, 3)
    plan = pat.Plan(g, wl.K, wl.sensors)
    tile, col_seq = 0, 0
    if args.tile == "auto" or args.col_order == "auto":
        from paper_2505_08482_amd import tune
        cfg = tune.launch_for(g.nx, wl.K)    # the committed table for this GPU type, else measured
        tile, col_seq = cfg["tile"], cfg["seq"]
    if args.tile != "auto":
        tile = int(args.tile)
    if args.col_order != "auto":
        col_seq = int(args.col_order)
    plan.set_tile(tile)
    plan.set_col_order(col_seq)
    t_c_true = torch.from_numpy(c_true.astype(np.float32)).to(dev)
    t_p0 = torch.from_numpy(p0.astype(np.float32)).to(dev)
    ws = plan.workspace(args.ckpt)
    data = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    # synthetic observation: data of the true medium + 1 % noise (seed 3500)
    plan.forward(t_c_true, t_p0, data, ws, ckpt_every=args.ckpt, record=False)
    clean = data.cpu().numpy().astype(np.float64)
    y_np, sigma = I.add_noise(clean, seed=3500)
    y = torch.from_numpy(y_np.astype(np.float32)).to(dev)
    w = torch.from_numpy((1.0 / sigma).astype(np.float32)).to(dev)
    # evaluate at the starting guess c = 1500 m/s everywhere
    c = torch.full((g.ny, g.nx), 1500.0, dtype=torch.float32, device=dev)
    resid = torch.empty_like(data)
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    g_p0 = torch.empty(plan.field_shape, dtype=torch.float32, device=dev)
    g_c = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)

    def evaluation():
        plan.forward(c, t_p0, data, ws, ckpt_every=args.ckpt, record=True)
        plan.misfit(data, y, w, resid, J)
        plan.adjoint_gradient(c, t_p0, resid, g_p0, g_c, ws)

    for _ in range(args.warmup):
        evaluation()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        evaluation()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1000.0 * wall / args.steps          # wall clock between the two synchronizations
    progress(f"timed {args.steps} evaluations: {ms:.1f} ms each")
    # Per-pass durations: start/stop HIP events attached to sampled dispatches of
    # every pass kind, on the stream they run on.  Events cannot sit inside the captured
    # step graphs, so this evaluation (right after the timed ones, same inputs
    # and launch shapes) launches its kernels one by one.
    pat.trace_start(args.trace_every)
    evaluation()
    torch.cuda.synchronize()
    pat.trace_stop()
    pts = wl.K * g.nx * g.ny * g.nt
    value = pts / (ms / 1000.0)

    tr = pat.trace_read()
    PB = pass_bytes(wl.K)
    PBM = pass_bytes(wl.K, moved=True)
    # measured bytes of the dominant pass (set below once it is known)
    tb = None
    shares = {k: v[1] / max(v[0], 1) for k, v in tr.items()}   # average launch duration, ms
    # every pass kind runs nt-1 times per evaluation: the longest average is the dominant one
    dom = max(PB, key=lambda k: shares[k])
    tb = measured_traffic(dom, wl.name)
    avg_ms = shares[dom]
    units = wl.K * g.nx * g.ny
    achieved = PB[dom] * units / (avg_ms / 1000.0) / 1e9
    passes = {k: {"avg_us": round(1000.0 * shares[k], 2), "timed_launches": tr[k][0],
                  "alg_GBps": round(PB[k] * units / (shares[k] / 1000.0) / 1e9, 1) if shares[k] > 0 else None}
              for k in PB}
    out = {
        "metric": "grid-pt-steps/s fwd+adjoint at 512^2 x 8 datasets",
        "value": value,
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{g.nx}x{g.ny}", "K": wl.K, "nt": g.nt, "sensors": wl.m,
                   "dx_m": g.dx, "dt_s": g.dt, "pml": g.pml,
                   "history": "store-all" if args.ckpt == 0 else f"checkpoint every {args.ckpt}",
                   "column_tile": tile or "default", "column_order": ("together", "sequential", "split")[col_seq],
                   "step": "recorded forward + misfit + adjoint gradient (g_p0 for all K, g_c)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(tb / (avg_ms / 1000.0) / 1e9, 1) if tb else None,
                     "traffic_bytes_per_launch": tb, "algorithmic_bytes_per_launch": PB[dom] * units,
                     "kernel": dom,
                     "avg_us": round(1000.0 * avg_ms, 2), "bytes_per_point": PB[dom],
                     "bytes_per_point_moved": PBM[dom],
                     "units_per_launch": units,
                     "timing": "HIP start/stop events attached to the kernel dispatch (hipExtLaunchKernelGGL) "
                               "on the launch stream, every %d-th launch of each pass, in one evaluation launched "
                               "kernel by kernel right after the timed (graph-replayed) ones" % args.trace_every,
                     # the whole time step (all eight passes, the figure the 50 % target is about):
                     # algorithmic bytes per grid-point step x grid-point steps per second
                     "step": {"bytes_per_point_step": sum(PB.values()),
                              "achieved": round(sum(PB.values()) * value / 1e9, 1),
                              "frac": round(sum(PB.values()) * value / 1e9 / HBM_PEAK_GBS, 4),
                              "rate_at_half_peak": round(0.5 * HBM_PEAK_GBS * 1e9 / sum(PB.values()), 1)}},
        "step_alg_GBps": round(sum(PB.values()) * pts / (ms / 1000.0) / 1e9, 1),
        "passes": passes,
        "J": float(J.item()),
    }
    if not args.no_extras:
        for name, fn in (("forward_only", lambda: forward_only(plan, wl, c, t_p0, data, ws)),
                         ("bandwidth_probe", bandwidth_probe),
                         ("checkpointed", lambda: checkpointed(plan, wl, c, t_p0, y, w, evaluation_ms=ms)),
                         ("batch", lambda: batch_w3(args.batch_evals)),
                         ("time_to_solution", lambda: time_to_solution(wl, t_c_true, y, w, args.tts_iters)),
                         ("time_to_solution_finer_data", lambda: time_to_solution_finer_data(wl.K, args.tts_iters)),
                         ("paper_geometry", lambda: paper_geometry(args.tts_iters)),
                         ("network", network_timing),
                         ("learned_start", lambda: learned_start(range(args.learned_cases))
                          if args.learned_cases > 0 else {"skipped": True}),
                         ("learned_start_finer_data", lambda: learned_start(range(args.learned_cases),
                                                                            data_grid=768)
                          if args.learned_cases > 0 else {"skipped": True})):
            progress(f"{name} ...")
            try:
                out[name] = fn()
            except Exception as e:   # an extra must never cost the main line
                out[name] = {"error": f"{type(e).__name__}: {e}"}
            progress(f"{name} done")
        if isinstance(out.get("batch"), dict) and "batched_value" in out["batch"]:
            out["batch"]["batched_over_w1_rate"] = round(out["batch"]["batched_value"] / value, 3)
    if not args.no_cpu:
        progress("cpu_baseline ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, wl.K)
        progress("cpu_baseline done")
        if not args.no_extras:
            out["cpu_baseline_single_core"] = cpu_baseline(max(2, args.cpu_steps // 4), wl.K, cores=1)
            progress("cpu_baseline_single_core done")
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
