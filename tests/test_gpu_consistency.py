"""GPU self-consistency of the HIP path (through the C ABI):

* checkpointed history (recompute from checkpoints) gives bit-identical
  gradients to the stored history, including a ragged last segment;
* a batch of K datasets gives bit-identical data and g_p0 to K single runs,
  and g_c equal to their sum up to float32 rounding (also for K not a
  multiple of the datasets per block of the adjoint density pass);
* the W1 launch configuration (512^2, K = 8, 4000 samples) checked by
  properties that hold at any size (linearity in p0, the adjoint dot-product
  identity in p0) and against the oracle on one dataset, g_c included;
* the generic (any radix) kernels and the power-of-two kernels agree.
"""
import dataclasses
import os

import numpy as np
import pytest

from oracle import kspace
from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce, gpu_forward_adjoint, oracle_forward_adjoint, observed_data, rel_l2

pytestmark = pytest.mark.gpu


def _wl(n=128, K=3, nt=203, m=96):
    g = I.make_grid(n, 1e-4 * 256 / n, nt, 10)
    rs = round(0.38 * n)
    return I.Workload(f"c_{n}_K{K}_nt{nt}", g, K=K, m=m, sensor_radius_px=float(rs),
                      support_radius_px=float(rs - 4))


def _inputs(wl, seed=0):
    c, p0 = I.phantoms(wl, 2, case=seed)
    rng = np.random.default_rng(seed + 11)
    resid = rng.standard_normal((wl.K, wl.grid.nt, wl.m)).astype(np.float32)
    return c.astype(np.float32), p0.astype(np.float32), resid


@pytest.mark.parametrize("s", [16, 50, 7])
def test_checkpointed_equals_store_all_bitwise(s):
    wl = _wl()
    c, p0, r = _inputs(wl)
    announce(f"store-all vs ckpt s={s}")
    a = gpu_forward_adjoint(wl, c, p0, resid32=r, ckpt_every=0)
    b = gpu_forward_adjoint(wl, c, p0, resid32=r, ckpt_every=s)
    assert np.array_equal(a["data"], b["data"])
    assert np.array_equal(a["g_p0"], b["g_p0"])
    assert np.array_equal(a["g_c"], b["g_c"])


@pytest.mark.parametrize("K", [4, 6])
def test_batch_equals_single_runs_bitwise(K):
    wl = _wl(K=K, nt=150)
    c, p0, r = _inputs(wl, seed=3)
    announce(f"batch K={K} vs singles")
    full = gpu_forward_adjoint(wl, c, p0, resid32=r)
    w1 = dataclasses.replace(wl, K=1, name=wl.name + "_single")
    gc_sum = np.zeros(full["g_c"].shape, dtype=np.float64)
    for k in range(wl.K):
        one = gpu_forward_adjoint(w1, c, p0[k:k + 1], resid32=np.ascontiguousarray(r[k:k + 1]))
        assert np.array_equal(one["data"][0], full["data"][k])
        assert np.array_equal(one["g_p0"][0], full["g_p0"][k])
        gc_sum = gc_sum + one["g_c"].astype(np.float64)
    # g_c of a batch adds the datasets' terms at every step (in dataset order)
    # before accumulating over time; a single run accumulates over time only, so
    # the float32 sums agree to rounding, not bitwise
    assert rel_l2(full["g_c"], gc_sum) <= 1e-5


def test_w1_full_size_properties():
    """512^2, K = 8, 4000 samples (the benchmark's launch configuration):
    f(a + 2b) = f(a) + 2 f(b) and <f(p0), y> = <p0, f^T y> in float32."""
    import torch
    from paper_2505_08482_amd import pat
    wl = I.w1()
    g = wl.grid
    c_np, p0_np = I.phantoms(wl, 3)
    plan = pat.Plan(g, wl.K, wl.sensors)
    ws = plan.workspace(0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    c = T(c_np)
    rng = np.random.default_rng(9)
    a = T(p0_np)
    b = T(rng.uniform(0, 1, p0_np.shape) * (p0_np > 0.01))
    ab = a + 2.0 * b
    out = {}
    announce("w1 full-size forward x3")
    for name, p in (("a", a), ("b", b), ("ab", ab)):
        d = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
        plan.forward(c, p, d, ws, record=False)
        out[name] = d
    lin = rel_l2((out["a"] + 2.0 * out["b"]).cpu().numpy(), out["ab"].cpu().numpy())
    print(f"[w1] linearity rel {lin:.2e}", flush=True)
    assert lin < 1e-5
    y = T(rng.standard_normal(plan.data_shape))
    d = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
    announce("w1 full-size forward+adjoint")
    plan.forward(c, a, d, ws, record=True)
    gp0 = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    gc = torch.empty((g.ny, g.nx), dtype=torch.float32, device="cuda")
    plan.adjoint_gradient(c, a, y, gp0, gc, ws)
    lhs = float((d.double() * y.double()).sum())
    rhs = float((a.double() * gp0.double()).sum())
    print(f"[w1] dot test {lhs:.6e} {rhs:.6e} rel {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    assert torch.isfinite(gc).all()
    plan.close()


def test_w1_full_size_dataset_vs_oracle():
    """The benchmark's launch configuration itself (512^2, K = 8, 4000 samples,
    the true heterogeneous c) against the float64 oracle.  The adjoint source
    is nonzero for dataset 5 only (the second dataset of the second group of
    four in the grouped g_c reduction): the datasets are independent given c and
    a zero residual gives a zero adjoint field, so g_c of the K = 8 launch must
    equal the oracle's g_c of dataset 5 alone, g_p0 of the other datasets must
    be exactly zero, and dataset 5's traces and g_p0 must match its oracle run."""
    from gpu_helpers import check_parity
    wl = I.w1()
    g = wl.grid
    j = 5
    c_np, p0_np = I.phantoms(wl, 3)
    c32 = c_np.astype(np.float32)
    p032 = p0_np.astype(np.float32)
    rng = np.random.default_rng(31)
    r32 = np.zeros((wl.K, g.nt, wl.m), dtype=np.float32)
    r32[j] = rng.standard_normal((g.nt, wl.m)).astype(np.float32)
    announce("w1 full size gpu K=8")
    gpu = gpu_forward_adjoint(wl, c32, p032, resid32=r32)
    for k in range(wl.K):
        if k != j:
            assert not np.any(gpu["g_p0"][k]), k
    announce(f"w1 full size oracle dataset {j}")
    data, hist = kspace.forward(g, wl.sensors, c32.astype(np.float64), p032[j:j + 1].astype(np.float64))
    gp0, gc = kspace.adjoint_gradient(g, wl.sensors, c32.astype(np.float64), p032[j:j + 1].astype(np.float64),
                                      r32[j:j + 1].astype(np.float64), hist)
    del hist
    check_parity(f"w1 full size, dataset {j}",
                 {"data": gpu["data"][j:j + 1], "g_p0": gpu["g_p0"][j:j + 1], "g_c": gpu["g_c"]},
                 {"data": data, "g_p0": gp0, "g_c": gc})


def test_generic_and_power_of_two_kernels_agree():
    """The same 128^2 problem through both kernel families agrees to float32
    rounding (the family is fixed when a plan is created: PAT_GENERIC_KERNELS
    set -> the any-radix kernels)."""
    wl = _wl(K=2, nt=120)
    c, p0, r = _inputs(wl, seed=5)
    outs = []
    try:
        for generic in (False, True):
            if generic:
                os.environ["PAT_GENERIC_KERNELS"] = "1"
            else:
                os.environ.pop("PAT_GENERIC_KERNELS", None)
            announce(f"kernel family generic={generic}")
            outs.append(gpu_forward_adjoint(wl, c, p0, resid32=r))
    finally:
        os.environ.pop("PAT_GENERIC_KERNELS", None)
    for key in ("data", "g_p0", "g_c"):
        e = rel_l2(outs[0][key], outs[1][key])
        print(f"[families] {key} {e:.2e}", flush=True)
        assert e < 1e-5, (key, e)


@pytest.mark.parametrize("ckpt", [0, 24])
def test_graph_replay_equals_eager_bitwise(ckpt):
    """Time-step chunks replayed from captured graphs give the same bits as the
    same kernels launched one by one, on every replay (four evaluations in a
    row on one plan and workspace, with eager work in between)."""
    import torch
    from paper_2505_08482_amd import pat
    wl = _wl(K=2, nt=150)
    c_np, p0_np, r_np = _inputs(wl, seed=7)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()

    def evaluate(plan, ws, c, p0, r):
        d = torch.empty(plan.data_shape, dtype=torch.float32, device="cuda")
        gp = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
        gc = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.float32, device="cuda")
        plan.forward(c, p0, d, ws, ckpt_every=ckpt, record=True)
        plan.adjoint_gradient(c, p0, r, gp, gc, ws)
        torch.cuda.synchronize()
        return d.cpu().numpy(), gp.cpu().numpy(), gc.cpu().numpy()

    c, p0, r = T(c_np), T(p0_np), T(r_np)
    os.environ["PAT_NO_GRAPHS"] = "1"
    try:
        plan = pat.Plan(wl.grid, wl.K, wl.sensors)
        ws = plan.workspace(ckpt)
        announce(f"eager reference ckpt={ckpt}")
        ref = evaluate(plan, ws, c, p0, r)
    finally:
        os.environ.pop("PAT_NO_GRAPHS", None)
    for rep in range(4):
        announce(f"graph replay {rep} ckpt={ckpt}")
        out = evaluate(plan, ws, c, p0, r)
        for a, b in zip(out, ref):
            assert np.array_equal(a, b), rep
        _ = (c * 1.0).sum().item()   # unrelated eager work and a synchronisation between replays
    plan.close()


def test_traced_launches_equal_plain_and_time_every_pass():
    """Sampled launches carry dispatch events (extended launch); the results
    must not change and every pass kind must report a positive duration."""
    from paper_2505_08482_amd import pat
    wl = _wl(n=128, K=3, nt=60)
    c, p0, r = _inputs(wl, seed=5)
    announce("traced vs plain launches")
    plain = gpu_forward_adjoint(wl, c, p0, resid32=r)
    pat.trace_start(3)
    try:
        traced = gpu_forward_adjoint(wl, c, p0, resid32=r)
    finally:
        pat.trace_stop()
    tr = pat.trace_read()
    for key in ("data", "g_p0", "g_c"):
        assert np.array_equal(plain[key], traced[key])
    for kind, (n, ms) in tr.items():
        print(f"[trace] {kind}: {n} launches, {ms / max(n, 1) * 1000:.2f} us")
        assert n > 0 and ms > 0.0


def test_graph_cache_eviction_keeps_results():
    """One plan driven through many distinct step-run shapes (checkpoint
    intervals) overflows its cache of captured graphs; evicted graphs are
    destroyed only after their launches finished and every result stays
    bit-identical to store-all."""
    import torch
    from paper_2505_08482_amd import pat
    wl = _wl(n=64, K=2, nt=97, m=32)
    c, p0, r = _inputs(wl, seed=9)
    announce("graph cache eviction")
    plan = pat.Plan(wl.grid, wl.K, wl.sensors)
    dev = "cuda"
    tc, tp0, tr = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (c, p0, r))
    outs = []
    for s in (0, 3, 5, 6, 7, 9, 10, 11, 13, 3, 0):
        ws = plan.workspace(s)
        data = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
        gp0 = torch.empty(plan.field_shape, dtype=torch.float32, device=dev)
        gc = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.float32, device=dev)
        plan.forward(tc, tp0, data, ws, ckpt_every=s, record=True)
        plan.adjoint_gradient(tc, tp0, tr, gp0, gc, ws)
        torch.cuda.synchronize()
        outs.append((s, data.cpu().numpy(), gp0.cpu().numpy(), gc.cpu().numpy()))
        del ws
    plan.close()
    ref = outs[0]
    for s, d, gp, gcc in outs[1:]:
        assert np.array_equal(d, ref[1]), s
        assert np.array_equal(gp, ref[2]), s
        assert np.array_equal(gcc, ref[3]), s


def test_error_paths_through_the_abi():
    """The library refuses, without launching anything: an adjoint before any
    recorded forward, with another workspace, other c / p0 buffers, or a
    workspace too small; a forward into a too-small workspace.  A refused call
    leaves the recorded state usable."""
    import torch
    from paper_2505_08482_amd import pat
    wl = _wl(n=64, K=2, nt=40, m=16)
    c, p0, r = _inputs(wl, seed=2)
    announce("error paths")
    plan = pat.Plan(wl.grid, wl.K, wl.sensors)
    dev = "cuda"
    tc, tp0, tr = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (c, p0, r))
    data = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    gp0 = torch.empty(plan.field_shape, dtype=torch.float32, device=dev)
    gc = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.float32, device=dev)
    ws = plan.workspace(0)
    ws2 = plan.workspace(0)

    def status(fn):
        try:
            fn()
        except pat.PatError as e:
            return e.status
        return pat.PAT_OK

    EW = pat.PAT_EWORKSPACE
    assert status(lambda: plan.adjoint_gradient(tc, tp0, tr, gp0, gc, ws)) == EW
    small = torch.empty(plan.workspace_size(0) - 256, dtype=torch.uint8, device=dev)
    assert status(lambda: plan.forward(tc, tp0, data, small, record=True)) == EW
    plan.forward(tc, tp0, data, ws, record=True)
    assert status(lambda: plan.adjoint_gradient(tc, tp0, tr, gp0, gc, ws2)) == EW
    assert status(lambda: plan.adjoint_gradient(tc.clone(), tp0, tr, gp0, gc, ws)) == EW
    assert status(lambda: plan.adjoint_gradient(tc, tp0.clone(), tr, gp0, gc, ws)) == EW
    plan.adjoint_gradient(tc, tp0, tr, gp0, gc, ws)   # the recorded state survived the refusals
    ref = gpu_forward_adjoint(wl, c, p0, resid32=r)
    torch.cuda.synchronize()
    assert np.array_equal(gp0.cpu().numpy(), ref["g_p0"]) and np.array_equal(gc.cpu().numpy(), ref["g_c"])
    plan.close()
