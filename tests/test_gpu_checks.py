"""Failure handling through the C ABI and in the reconstruction driver:

* the check mode of a plan (PAT_CHECK_FINITE at plan creation) returns
  PAT_ENONFINITE when a forward or adjoint output holds a NaN or an infinity,
  and OK otherwise; without it the same call returns OK;
* the projected L-BFGS driver rejects line-search trials whose objective is
  not finite (it halves the step until the trial is finite and satisfies the
  Armijo test), so no non-finite value ever enters the iterate or the pairs.
"""
import os

import numpy as np
import pytest

from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _plan_and_buffers(wl, check: bool):
    import torch
    from paper_2505_08482_amd import pat
    if check:
        os.environ["PAT_CHECK_FINITE"] = "1"
    try:
        plan = pat.Plan(wl.grid, wl.K, wl.sensors)
    finally:
        os.environ.pop("PAT_CHECK_FINITE", None)
    g = wl.grid
    bufs = {"data": torch.empty(plan.data_shape, dtype=torch.float32, device="cuda"),
            "gp0": torch.empty(plan.field_shape, dtype=torch.float32, device="cuda"),
            "gc": torch.empty((g.ny, g.nx), dtype=torch.float32, device="cuda"),
            "ws": plan.workspace(0)}
    return plan, bufs


def test_check_mode_reports_nonfinite_outputs():
    import torch
    from paper_2505_08482_amd import pat
    wl = I.config2(n=64, K=2, nt=60)
    c_np, p0_np = I.phantoms(wl, 2)
    c = torch.from_numpy(c_np.astype(np.float32)).cuda()
    p0 = torch.from_numpy(p0_np.astype(np.float32)).cuda()
    r = torch.from_numpy(np.random.default_rng(4).standard_normal((wl.K, wl.grid.nt, wl.m)).astype(np.float32)).cuda()
    c_bad = c.clone()
    c_bad[32, 30] = float("nan")
    announce("check mode: finite inputs")
    plan, b = _plan_and_buffers(wl, check=True)
    plan.forward(c, p0, b["data"], b["ws"], record=True)
    plan.adjoint_gradient(c, p0, r, b["gp0"], b["gc"], b["ws"])
    torch.cuda.synchronize()
    announce("check mode: a NaN in c")
    with pytest.raises(pat.PatError) as e:
        plan.forward(c_bad, p0, b["data"], b["ws"], record=True)
    assert e.value.status == pat.PAT_ENONFINITE
    plan.close()
    announce("no check mode: a NaN in c")
    plan, b = _plan_and_buffers(wl, check=False)
    plan.forward(c_bad, p0, b["data"], b["ws"], record=True)     # no check: OK, NaN data
    torch.cuda.synchronize()
    assert not torch.isfinite(b["data"]).all()
    plan.close()
    assert pat.status_string(pat.PAT_ENONFINITE).startswith("non-finite")


class _Quadratic:
    """J(z) = 1/2 |z - t|^2 with t outside the region z < 3, where J is NaN
    (a stand-in for a forward solve that blows up); bounds [-10, 10]."""

    def __init__(self, n):
        import torch
        self.n = n
        self.t = torch.full((n,), 5.0, device="cuda")
        self.lo_z = torch.full((n,), -10.0, device="cuda")
        self.hi_z = torch.full((n,), 10.0, device="cuda")
        self.evals = 0
        self.trials = []

    def objective(self, z):
        self.evals += 1
        self.z = z.clone()
        J = 0.5 * float(((z - self.t) ** 2).sum().item())
        if float(z.max().item()) >= 3.0:
            J = float("nan")
        self.trials.append(J)
        return J

    def gradient(self):
        return self.z - self.t

    def dot(self, a, b):
        return float((a.double() * b.double()).sum().item())


def test_lbfgs_rejects_nonfinite_trials():
    import torch
    from paper_2505_08482_amd import recon
    announce("projected L-BFGS with non-finite trials")
    prob = _Quadratic(64)
    z0 = torch.linspace(-1.0, 1.0, 64, device="cuda")
    hist = []
    z, J, Js, nit = recon.projected_lbfgs(prob, z0, iters=12, callback=lambda it, z, J: hist.append(J) and False)
    assert any(np.isnan(t) for t in prob.trials), "the test must produce non-finite trials"
    assert np.all(np.isfinite(Js)) and np.all(np.diff(Js) <= 0.0), Js
    assert torch.isfinite(z).all() and float(z.max().item()) < 3.0
    assert J < Js[0]
