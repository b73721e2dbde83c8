"""Uneven batches and launch tuning (GPU): pat_batch_gradient gives every
problem exactly the bits it gets alone, for problems of different grid sizes
(power-of-two and mixed-radix), dataset counts and time axes, with any stream
count; the column tile width changes no bit.  Problems of one transform
family and grid size advance in shared launches (one launch per pass for
all of them)."""
import numpy as np
import pytest

from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _job(n, K, nt, seed):
    import torch
    from paper_2505_08482_amd import pat
    wl = I.config2(n=n, K=K, nt=nt)
    c_true, p0 = I.phantoms(wl, 4, case=seed)
    plan = pat.Plan(wl.grid, K, wl.sensors)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    rng = np.random.default_rng(seed)
    job = {"plan": plan, "c": T(np.full_like(c_true, 1500.0)), "p0": T(p0),
           "y": T(rng.standard_normal(plan.data_shape) * 0.01), "w": T(rng.uniform(50, 100, K)),
           "data": torch.empty(plan.data_shape, device="cuda"), "ws": plan.workspace(0)}
    job["resid"] = torch.empty_like(job["data"])
    job["J"] = torch.zeros(1, dtype=torch.float64, device="cuda")
    job["g_p0"] = torch.empty(plan.field_shape, device="cuda")
    job["g_c"] = torch.empty((n, n), device="cuda")
    return job


def _single(job):
    import torch
    p = job["plan"]
    p.forward(job["c"], job["p0"], job["data"], job["ws"], record=True)
    p.misfit(job["data"], job["y"], job["w"], job["resid"], job["J"])
    p.adjoint_gradient(job["c"], job["p0"], job["resid"], job["g_p0"], job["g_c"], job["ws"])
    torch.cuda.synchronize()
    return {k: job[k].cpu().numpy().copy() for k in ("data", "resid", "J", "g_p0", "g_c")}


def _check_batch(jobs, ref, ns, what):
    import torch
    from paper_2505_08482_amd import pat
    for j in jobs:
        j["g_c"].fill_(7.0); j["g_p0"].fill_(7.0); j["data"].fill_(7.0); j["J"].fill_(7.0)
    announce(f"batch nstreams={ns} {what}")
    pat.batch_gradient(jobs, ns)
    torch.cuda.synchronize()
    for j, r in zip(jobs, ref):
        for k in r:
            assert np.array_equal(j[k].cpu().numpy(), r[k]), (ns, what, j["plan"].grid.nx, j["plan"].K, k)


def test_batch_equals_single_runs_bitwise():
    """Problems sharing launches (same family and grid size) with different
    dataset counts (datasets per block of the adjoint density pass 1, 2, 4)
    and time axes (the forward solves aligned at their ends, the adjoint
    solves at their starts), including single-sample and two-sample problems;
    batches replayed from their captured step graphs, and a different batch
    in between (new slot tables)."""
    from paper_2505_08482_amd import pat
    specs = [(128, 2, 120, 1), (192, 1, 90, 2), (256, 4, 70, 3), (64, 1, 150, 4), (128, 1, 41, 5),
             (128, 4, 77, 6), (192, 2, 2, 7), (128, 2, 1, 8), (192, 3, 131, 9)]
    jobs = [_job(*s) for s in specs]
    announce("single runs")
    ref = [_single(j) for j in jobs]
    for ns in (1, 3, 8):
        _check_batch(jobs, ref, ns, "first")
    _check_batch(jobs, ref, 3, "again (replayed graphs)")
    _check_batch(jobs[:4], ref[:4], 3, "another batch")
    _check_batch(jobs, ref, 3, "the first batch again")
    pat.batch_release()
    _check_batch(jobs, ref, 2, "after releasing the streams")
    for j in jobs:
        j["plan"].close()


@pytest.mark.parametrize("n, K", [(256, 2), (512, 8), (128, 3)])
def test_column_launch_configuration_changes_no_bit(n, K):
    """Every candidate of the tuner (column tile 4 or 8, the two transforms of
    a thread together or one after the other, the two arrays on two halves of
    a block) gives the same bits."""
    job = _job(n, K, 60, 9)
    announce(f"column configurations {n} K={K}")
    ref = _single(job)
    for tile, seq in ((8, 0), (0, 1), (8, 1), (0, 2)):
        job["plan"].set_tile(tile)
        job["plan"].set_col_order(seq)
        out = _single(job)
        for k in ref:
            assert np.array_equal(ref[k], out[k]), (tile, seq, k)
    job["plan"].close()
