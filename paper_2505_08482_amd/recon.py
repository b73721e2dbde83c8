"""Joint reconstruction of the K initial pressures and the shared sound speed
(Sec. 3, Sec. 3.1) on top of the C ABI.

* objective and gradient: ``pat_forward`` (recorded) + ``pat_misfit`` +
  ``pat_adjoint_gradient`` (eq. (4) data term, eqs. (5)-(9));
* optional prior terms of eq. (4) (Ornstein-Uhlenbeck, Sec. 4.1.2) through
  ``pat_ou_prior``, added to J and to the gradient;
* step: eq. (10) ``x <- P(x - alpha H g)`` with ``pat_lbfgs_direction``
  (Alg. 1, memory l) and ``pat_project_update`` (eq. (11)), backtracking
  (Armijo) line search with trial forward solves only;
* multigrid continuation (Sec. 3.1): coarse-to-fine levels, the converged
  iterate carried to the next level with ``pat_prolong_phys`` (same physical
  positions, levels of any extent) and the data
  resampled onto each level's time grid with ``pat_time_interp`` (Sec. 4.1.2).

The optimiser works on scaled variables ``z = x / scale`` (per block: p0 and c).
Its decisions (active set, direction safeguards, Armijo test, pair filter) are
the ones of the float64 reference driver.  Every vector operation of an
iteration runs in the library (``pat_free_part``, ``pat_axpby``, ``pat_mul``,
``pat_absmax``, ``pat_dot``); the host keeps the scalars and the decisions.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import inputs as I
from . import pat


@dataclasses.dataclass
class LevelResult:
    n: int
    iters: int
    evals: int
    J: List[float]
    seconds: float
    E_c: List[float]
    t: List[float]          # seconds since the start of the level, per iteration
    t_start: float = 0.0    # seconds from the start of the multigrid run to the start of the level


class Problem:
    """One grid level: K datasets, observed traces y, weights w, bounds."""

    def __init__(self, wl: I.Workload, y: torch.Tensor, w: torch.Tensor, c_lo: float, c_hi: float,
                 c_fixed: float = 1500.0, ckpt_every: int = 0, device="cuda", prior: Optional[Dict] = None):
        self.wl = wl
        g = wl.grid
        self.plan = pat.Plan(g, wl.K, wl.sensors)
        self.ws = self.plan.workspace(ckpt_every, device=device)
        self.ckpt = ckpt_every
        self.y = y.contiguous()
        self.w = w.contiguous()
        self.N = g.nx * g.ny
        self.K = wl.K
        self.n = (self.K + 1) * self.N
        mask = torch.from_numpy(wl.mask().astype(np.bool_)).to(device)
        # bounds (eq. (11)): p0 >= 0, c in [c_lo, c_hi]; outside the mask both are pinned
        lo = torch.empty(self.n, dtype=torch.float32, device=device)
        hi = torch.empty_like(lo)
        lo[: self.K * self.N] = 0.0
        hi[: self.K * self.N] = float("inf")
        lo[self.K * self.N:] = c_lo
        hi[self.K * self.N:] = c_hi
        outside = ~mask.reshape(-1)
        for k in range(self.K + 1):
            sl = slice(k * self.N, (k + 1) * self.N)
            fixed = c_fixed if k == self.K else 0.0
            lo[sl][outside] = fixed
            hi[sl][outside] = fixed
        self.scale = torch.empty_like(lo)
        self.scale[: self.K * self.N] = 0.25
        self.scale[self.K * self.N:] = (c_hi - c_lo) / 4.0
        self.inv_scale = 1.0 / self.scale
        self.lo_z = lo * self.inv_scale
        self.hi_z = hi * self.inv_scale
        self.mask = mask
        self.data = torch.empty(self.plan.data_shape, dtype=torch.float32, device=device)
        self.resid = torch.empty_like(self.data)
        self.J = torch.zeros(1, dtype=torch.float64, device=device)
        # the physical point of the last objective call and the physical gradient,
        # each one vector [K*N + N] whose blocks are the p0 and c fields
        self.x = torch.empty(self.n, dtype=torch.float32, device=device)
        self.g_all = torch.empty(self.n, dtype=torch.float32, device=device)
        self.gp0 = self.g_all[: self.K * self.N].view(self.plan.field_shape)
        self.gc = self.g_all[self.K * self.N:].view(g.ny, g.nx)
        self.dot_scratch = torch.empty(pat.lbfgs_scratch_bytes(0), dtype=torch.uint8, device=device)
        self.dot_out = torch.zeros(1, dtype=torch.float64, device=device)
        self.evals = 0
        # eq. (4) prior terms (Ornstein-Uhlenbeck, Sec. 4.1.2): one operator over the
        # reconstruction domain, a mean and a standard deviation per distribution
        self.ou = None
        if prior is not None:
            self.ou = pat.OuPrior(g.ny, g.nx, g.dx, prior["tau"], mask.cpu().numpy())
            eta = [prior["eta_p0"]] * self.K + [prior["eta_c"]]
            sig = [prior["sigma_p0"]] * self.K + [prior["sigma_c"]]
            self.eta = torch.tensor(eta, dtype=torch.float32, device=device)
            self.inv_var = torch.tensor([1.0 / s_ ** 2 for s_ in sig], dtype=torch.float32, device=device)
            self.g_prior = torch.empty((self.K + 1, g.ny, g.nx), dtype=torch.float32, device=device)
            self.J_prior = torch.zeros(1, dtype=torch.float64, device=device)
            self.prior_tol = prior.get("tol", 1e-6)
            self.cg_iters = []

    def split(self, x: torch.Tensor):
        """Physical (p0 [K][ny][nx], c [ny][nx]) views of a physical stacked vector."""
        g = self.wl.grid
        return x[: self.K * self.N].view(self.K, g.ny, g.nx), x[self.K * self.N:].view(g.ny, g.nx)

    def objective(self, z: torch.Tensor) -> float:
        """J at scaled point z (recorded forward solve + misfit, plus the prior
        terms when configured)."""
        pat.mul(z, self.scale, self.x)     # kept: the adjoint reads the same buffers
        p0, c = self.split(self.x)
        self.plan.forward(c, p0, self.data, self.ws, ckpt_every=self.ckpt, record=True)
        self.plan.misfit(self.data, self.y, self.w, self.resid, self.J)
        self.evals += 1
        J = float(self.J.item())
        if self.ou is not None:
            g = self.wl.grid
            self.cg_iters.append(self.ou.prior(self.x.view(self.K + 1, g.ny, g.nx), self.eta, self.inv_var,
                                               self.g_prior, self.J_prior, tol=self.prior_tol))
            J += float(self.J_prior.item())
        return J

    def gradient(self) -> torch.Tensor:
        """Scaled gradient at the point of the last ``objective`` call (a new vector)."""
        p0, c = self.split(self.x)
        self.plan.adjoint_gradient(c, p0, self.resid, self.gp0, self.gc, self.ws)
        if self.ou is not None:
            pat.axpby(1.0, self.g_all, 1.0, self.g_prior.reshape(-1), self.g_all)
        out = torch.empty_like(self.g_all)
        pat.mul(self.g_all, self.scale, out)
        return out

    def dot(self, a, b) -> float:
        pat.dot(a, b, self.dot_out, self.dot_scratch)
        return float(self.dot_out.item())

    def close(self):
        self.plan.close()
        if self.ou is not None:
            self.ou.close()


def projected_lbfgs(prob: Problem, z0: torch.Tensor, iters: int, memory: int = 20, c1: float = 1e-4,
                    max_halvings: int = 20, callback: Optional[Callable] = None, state: Optional[Dict] = None,
                    log: Optional[Callable] = None):
    """Eq. (10) iterations on scaled variables (see the module docstring).

    ``state`` (optional): a dict from ``lbfgs_state`` (the iterate and the
    stored pairs of an interrupted run) to resume from; ``z0`` is then
    ignored.  ``log`` (optional): called after every accepted step with a dict
    of the iteration's figures (J, projected-gradient max norm, step length,
    trials, whether the step was quasi-Newton)."""
    dev = z0.device
    if state is not None:
        z = state["z"].to(dev).clone()
        S = [t.to(dev).clone() for t in state["S"]]
        Y = [t.to(dev).clone() for t in state["Y"]]
    else:
        z = z0.clone()
        S, Y = [], []
    pat.project_update(z, torch.zeros_like(z), 0.0, prob.lo_z, prob.hi_z)
    J = prob.objective(z)
    g = prob.gradient()
    scratch = torch.empty(pat.lbfgs_scratch_bytes(memory), dtype=torch.uint8, device=dev)
    red = torch.empty(pat.lbfgs_scratch_bytes(0), dtype=torch.uint8, device=dev)
    dmax = torch.zeros(1, dtype=torch.float64, device=dev)
    hist = [J]
    d = torch.empty_like(z)
    gf = torch.empty_like(z)
    step = torch.empty_like(z)

    def steepest() -> bool:
        """d = gf / max |gf| (the norm of this iteration); False if gf is zero."""
        if gnorm == 0.0:
            return False
        pat.axpby(1.0 / gnorm, gf, 0.0, None, d)
        return True

    gnorm = 0.0
    it = 0
    for it in range(iters):
        pat.free_part(z, g, prob.lo_z, prob.hi_z, g, gf)
        pat.absmax(gf, dmax, red)
        gnorm = float(dmax.item())
        use_qn = bool(S)
        if use_qn:
            pat.lbfgs_direction(gf, S, Y, d, scratch)
            pat.free_part(z, g, prob.lo_z, prob.hi_z, d, d)
            if prob.dot(d, gf) <= 0.0:
                S.clear(); Y.clear()
                use_qn = False
        if not use_qn and not steepest():
            break
        accepted = False
        zt = torch.empty_like(z)
        trials = 0
        for attempt in range(2):
            alpha = 1.0
            for _ in range(max_halvings):
                pat.axpby(1.0, z, 0.0, None, zt)
                pat.project_update(zt, d, alpha, prob.lo_z, prob.hi_z)
                Jt = prob.objective(zt)
                trials += 1
                pat.axpby(1.0, zt, -1.0, z, step)
                if np.isfinite(Jt) and Jt <= J + c1 * prob.dot(g, step):
                    accepted = True
                    break
                alpha *= 0.5
            if accepted or not use_qn:
                break
            S.clear(); Y.clear()
            use_qn = False
            if not steepest():
                break
        if not accepted:
            break
        gt = prob.gradient()    # adjoint of the accepted trial's recorded forward solve
        s_ = torch.empty_like(z)
        y_ = torch.empty_like(z)
        pat.axpby(1.0, zt, -1.0, z, s_)
        pat.axpby(1.0, gt, -1.0, g, y_)
        ys = prob.dot(y_, s_)
        if ys > 1e-10 * np.sqrt(max(prob.dot(y_, y_), 0.0)) * np.sqrt(max(prob.dot(s_, s_), 0.0)):
            S.append(s_); Y.append(y_)
            if len(S) > memory:
                S.pop(0); Y.pop(0)
        z, J, g = zt, Jt, gt
        hist.append(J)
        prob.last_state = {"z": z, "S": list(S), "Y": list(Y)}
        if log is not None:
            log({"iter": it + 1, "J": J, "proj_grad_max": gnorm, "alpha": alpha, "trials": trials,
                 "quasi_newton": use_qn, "pairs": len(S)})
        if callback is not None and callback(it, z, J):
            break            # the caller's stopping rule (e.g. a target error reached)
    prob.last_state = {"z": z, "S": list(S), "Y": list(Y)}
    return z, J, hist, it + 1


class _Lane:
    """State of one problem in the lockstep driver (the same decisions, in the
    same order, as ``projected_lbfgs``)."""

    def __init__(self, prob: Problem, z0: torch.Tensor, iters: int, memory: int):
        self.prob, self.iters, self.memory = prob, iters, memory
        self.z = z0.clone()
        pat.project_update(self.z, torch.zeros_like(self.z), 0.0, prob.lo_z, prob.hi_z)
        self.zt = self.z            # the point to evaluate next
        self.S, self.Y = [], []
        self.J = None
        self.g = None
        self.hist = []
        self.it = 0
        self.done = False
        self.d = torch.empty_like(self.z)
        self.gf = torch.empty_like(self.z)
        self.step = torch.empty_like(self.z)
        self.red = torch.empty(pat.lbfgs_scratch_bytes(0), dtype=torch.uint8, device=z0.device)
        self.dmax = torch.zeros(1, dtype=torch.float64, device=z0.device)
        self.scratch = torch.empty(pat.lbfgs_scratch_bytes(memory), dtype=torch.uint8, device=z0.device)

    def job(self) -> Dict:
        p = self.prob
        p0, c = p.split(p.x)
        return {"plan": p.plan, "c": c, "p0": p0, "y": p.y, "w": p.w, "data": p.data, "resid": p.resid,
                "J": p.J, "g_p0": p.gp0, "g_c": p.gc, "ws": p.ws}

    def load(self):
        pat.mul(self.zt, self.prob.scale, self.prob.x)

    def _start_iteration(self):
        """Direction and the first trial of iteration self.it (True), or stop (False)."""
        p = self.prob
        pat.free_part(self.z, self.g, p.lo_z, p.hi_z, self.g, self.gf)
        pat.absmax(self.gf, self.dmax, self.red)
        self.gnorm = float(self.dmax.item())
        self.use_qn = bool(self.S)
        if self.use_qn:
            pat.lbfgs_direction(self.gf, self.S, self.Y, self.d, self.scratch)
            pat.free_part(self.z, self.g, p.lo_z, p.hi_z, self.d, self.d)
            if p.dot(self.d, self.gf) <= 0.0:
                self.S.clear(); self.Y.clear()
                self.use_qn = False
        if not self.use_qn and not self._steepest():
            return False
        self.attempt, self.alpha, self.halvings = 0, 1.0, 0
        self._propose()
        return True

    def _steepest(self) -> bool:
        if self.gnorm == 0.0:
            return False
        pat.axpby(1.0 / self.gnorm, self.gf, 0.0, None, self.d)
        return True

    def _propose(self):
        self.zt = torch.empty_like(self.z)
        pat.axpby(1.0, self.z, 0.0, None, self.zt)
        pat.project_update(self.zt, self.d, self.alpha, self.prob.lo_z, self.prob.hi_z)

    def evaluated(self, c1: float, max_halvings: int):
        """Take the objective and gradient just computed at self.zt."""
        p = self.prob
        p.evals += 1
        Jt = float(p.J.item())
        gt = torch.empty_like(p.g_all)
        pat.mul(p.g_all, p.scale, gt)
        if self.J is None:                       # the starting point
            self.J, self.g = Jt, gt
            self.hist.append(Jt)
            if self.iters <= 0 or not self._start_iteration():
                self.done = True
            return
        pat.axpby(1.0, self.zt, -1.0, self.z, self.step)
        if np.isfinite(Jt) and Jt <= self.J + c1 * p.dot(self.g, self.step):
            s_ = torch.empty_like(self.z)
            y_ = torch.empty_like(self.z)
            pat.axpby(1.0, self.zt, -1.0, self.z, s_)
            pat.axpby(1.0, gt, -1.0, self.g, y_)
            ys = p.dot(y_, s_)
            if ys > 1e-10 * np.sqrt(max(p.dot(y_, y_), 0.0)) * np.sqrt(max(p.dot(s_, s_), 0.0)):
                self.S.append(s_); self.Y.append(y_)
                if len(self.S) > self.memory:
                    self.S.pop(0); self.Y.pop(0)
            self.z, self.J, self.g = self.zt, Jt, gt
            self.hist.append(Jt)
            self.it += 1
            if self.it >= self.iters or not self._start_iteration():
                self.done = True
            return
        self.alpha *= 0.5
        self.halvings += 1
        if self.halvings < max_halvings:
            self._propose()
            return
        if self.use_qn and self.attempt == 0:    # restart with steepest descent
            self.S.clear(); self.Y.clear()
            self.use_qn = False
            self.attempt, self.alpha, self.halvings = 1, 1.0, 0
            if self._steepest():
                self._propose()
                return
        self.done = True                         # no acceptable step


def batched_projected_lbfgs(probs: List[Problem], z0s: List[torch.Tensor], iters: int, memory: int = 20,
                            c1: float = 1e-4, max_halvings: int = 20, nstreams: int = 4):
    """``projected_lbfgs`` on many independent problems in lockstep: every
    round evaluates one point of every problem (its next line-search trial, or
    its last point again once it has finished) with one ``pat_batch_gradient``
    call, so problems of one grid size share every launch.  Each problem takes
    exactly the iterates it takes alone (an evaluation is bit-identical in a
    batch and alone; a trial's gradient is kept only when the trial is
    accepted).  Returns one ``(z, J, hist, iterations)`` per problem."""
    if any(p.ou is not None for p in probs):
        raise ValueError("batched_projected_lbfgs: the prior terms are not supported")
    lanes = [_Lane(p, z0, iters, memory) for p, z0 in zip(probs, z0s)]
    jobs = [ln.job() for ln in lanes]
    while True:
        for ln in lanes:
            ln.load()
        pat.batch_gradient(jobs, nstreams)
        for ln in lanes:
            if not ln.done:
                ln.evaluated(c1, max_halvings)
        if all(ln.done for ln in lanes):
            break
        for ln in lanes:
            if ln.done:
                ln.zt = ln.z                     # re-evaluate the final point (keeps the batch fixed)
    if any(ln.zt is not ln.z for ln in lanes):
        # a lane that ended on a rejected trial: evaluate every final point
        # once more, so that each problem's buffers (p0 gradient, data,
        # residual) hold its final iterate's values, as after the one-problem
        # driver
        for ln in lanes:
            ln.zt = ln.z
            ln.load()
        pat.batch_gradient(jobs, nstreams)
    # iterations as ``projected_lbfgs`` counts them (a final iteration that
    # found no acceptable step counts)
    return [(ln.z, ln.J, ln.hist, ln.it if ln.it >= ln.iters else ln.it + 1) for ln in lanes]


def lbfgs_state(prob) -> Dict:
    """The iterate and the stored pairs after the last ``projected_lbfgs`` run
    on ``prob`` (device tensors; for ``save_state`` and resuming)."""
    return prob.last_state


def relative_error_c(prob: Problem, z: torch.Tensor, c_true: torch.Tensor) -> float:
    """Eq. (12) for c over the reconstruction mask, in percent."""
    x = torch.empty_like(z)
    pat.mul(z, prob.scale, x)
    _, c = prob.split(x)
    m = prob.mask
    return 100.0 * float(torch.linalg.vector_norm((c - c_true)[m]) / torch.linalg.vector_norm(c_true[m]))


def save_state(path: str, level: int, iters_done: int, prob: Problem, levels_n: List[int]) -> None:
    """Write the reconstruction's resumable state (``.npz``, no pickles): the
    level index, the iterations done on it, the iterate (scaled, as the
    optimiser holds it, and physical) and the stored L-BFGS pairs of the last
    ``projected_lbfgs`` run on ``prob``."""
    st = prob.last_state
    x = torch.empty_like(st["z"])
    pat.mul(st["z"], prob.scale, x)
    S = torch.stack(st["S"]).cpu().numpy() if st["S"] else np.zeros((0, prob.n), np.float32)
    Y = torch.stack(st["Y"]).cpu().numpy() if st["Y"] else np.zeros((0, prob.n), np.float32)
    tmp = path + ".tmp.npz"
    np.savez(tmp, level=np.array([level]), iters_done=np.array([iters_done]), x=x.cpu().numpy(),
             z=st["z"].cpu().numpy(), S=S, Y=Y, levels=np.array(levels_n))
    import os
    os.replace(tmp, path)


def _truth_at(c_true, wl: I.Workload, levels: List[I.Workload]) -> torch.Tensor:
    """The true sound speed on level ``wl``: a callable's value there, or a
    tensor covering the finest level's physical extent (on that level's grid or
    a finer one), resampled at the same physical positions."""
    if callable(c_true):
        return c_true(wl)
    g = wl.grid
    if c_true.shape[-1] == g.nx and c_true.shape[-2] == g.ny:
        return c_true
    fg = levels[-1].grid
    dx_t = fg.dx * fg.nx / c_true.shape[-1]       # the tensor's spacing over the finest level's extent
    out = torch.empty((1, g.ny, g.nx), dtype=torch.float32, device=c_true.device)
    pat.prolong_phys(c_true.reshape(1, *c_true.shape).contiguous(), dx_t, out, g.dx)
    return out[0]


def multigrid(levels: List[I.Workload], y_fine: torch.Tensor, dt_fine: float, w: torch.Tensor, c_true_fine,
              c_lo: float = 1400.0, c_hi: float = 1600.0, iters: int = 40, memory: int = 20,
              ckpt_every: int = 0, target_Ec: Optional[float] = None, log: Optional[Callable] = None,
              c_init: Optional[float] = None, c_fixed: float = 1500.0, prior: Optional[Dict] = None,
              log_path: Optional[str] = None, save_path: Optional[str] = None, save_every: int = 10,
              resume: Optional[str] = None):
    """Coarse-to-fine reconstruction (Sec. 3.1).  ``c_true_fine`` only measures
    E_c and never enters the optimisation: a tensor over the finest level's
    physical extent (on its grid or a finer one; resampled to each level), or a
    callable ``level workload -> tensor``.
    Levels may differ in physical extent (Table 1); the converged iterate is
    carried to the next level at the same physical positions.  ``c_init``: the
    starting sound speed inside the mask (default: the middle of the bounds);
    ``c_fixed``: the sound speed held outside the mask.  ``prior``: the
    Ornstein-Uhlenbeck prior terms of eq. (4) (keys tau, eta_p0, sigma_p0,
    eta_c, sigma_c, optional tol), or None for bounds only.

    ``log_path``: one JSON line per iteration (level, iteration, J, max |projected
    gradient|, step length, line-search trials, E_c, seconds).  ``save_path``:
    the resumable state (``save_state``) every ``save_every`` iterations and at
    the end of every level; ``resume``: such a file, to continue an interrupted
    run (the same levels and settings) where it stopped, with the same results.
    ``target_Ec`` (percent): stop on the finest level at the first iteration
    whose E_c is at or below it (coarser levels always run ``iters``)."""
    import json
    device = y_fine.device
    results: List[LevelResult] = []
    z_prev = None
    prev = None
    t_all = time.perf_counter()
    start_level, done_iters, saved = 0, 0, None
    levels_n = [wl.grid.nx for wl in levels]
    if resume is not None:
        with np.load(resume, allow_pickle=False) as f:
            saved = {k: f[k] for k in f.files}
        if [int(v) for v in saved["levels"]] != levels_n:
            raise ValueError("resume: the saved run used other levels")
        start_level, done_iters = int(saved["level"][0]), int(saved["iters_done"][0])
    logf = open(log_path, "a") if log_path else None
    try:
        for li, wl in enumerate(levels):
            if li < start_level:
                continue
            g = wl.grid
            y = torch.empty((wl.K, g.nt, wl.m), dtype=torch.float32, device=device)
            pat.time_interp(y_fine, dt_fine, y, g.dt)
            prob = Problem(wl, y, w, c_lo, c_hi, c_fixed=c_fixed, ckpt_every=ckpt_every, prior=prior)
            state = None
            level_iters = iters
            if saved is not None and li == start_level:
                x0 = torch.from_numpy(saved["x"]).to(device)
                state = {"z": torch.from_numpy(saved["z"]).to(device),
                         "S": [torch.from_numpy(v).to(device) for v in saved["S"]],
                         "Y": [torch.from_numpy(v).to(device) for v in saved["Y"]]}
                level_iters = iters - done_iters
            elif z_prev is None:
                x0 = torch.empty(prob.n, dtype=torch.float32, device=device)
                x0[: prob.K * prob.N] = 0.0
                x0[prob.K * prob.N:] = 0.5 * (c_lo + c_hi) if c_init is None else c_init
            else:
                pg = prev.wl.grid
                xc = torch.empty_like(z_prev)
                pat.mul(z_prev, prev.scale, xc)
                xc = xc.view(prev.K + 1, pg.ny, pg.nx)
                xf = torch.empty((prob.K + 1, g.ny, g.nx), dtype=torch.float32, device=device)
                pat.prolong_phys(xc, pg.dx, xf, g.dx)
                x0 = xf.reshape(-1)
                prev.close()
            z0 = torch.empty_like(x0)
            pat.mul(x0, prob.inv_scale, z0)
            ct = _truth_at(c_true_fine, wl, levels)
            Ec = []
            Ts = []
            figures = {}
            first = iters - level_iters
            t0 = time.perf_counter()

            def cb(it, z, J):
                Ec.append(relative_error_c(prob, z, ct))
                Ts.append(time.perf_counter() - t0)
                if log:
                    log(f"level {g.nx}: iter {first + it + 1} J {J:.6e} E_c {Ec[-1]:.3f} %")
                if logf:
                    rec = dict(figures, level=g.nx, iter=first + it + 1, E_c=Ec[-1], t=round(Ts[-1], 4))
                    logf.write(json.dumps(rec) + "\n")
                    logf.flush()
                if save_path and (first + it + 1) % save_every == 0:
                    save_state(save_path, li, first + it + 1, prob, levels_n)
                # the caller's target on the finest level ends the run there
                return target_Ec is not None and li == len(levels) - 1 and Ec[-1] <= target_Ec

            z, J, hist, nit = projected_lbfgs(prob, z0, level_iters, memory=memory, callback=cb, state=state,
                                              log=figures.update)
            torch.cuda.synchronize()
            if save_path:
                if li + 1 < len(levels):
                    prob.last_state = {"z": z, "S": [], "Y": []}   # a finished level: no pairs carried
                    save_state(save_path, li, iters, prob, levels_n)
                else:
                    save_state(save_path, li, first + nit, prob, levels_n)
            results.append(LevelResult(g.nx, nit, prob.evals, hist, time.perf_counter() - t0, Ec, Ts, t0 - t_all))
            z_prev, prev = z, prob
    finally:
        if logf:
            logf.close()
    x = torch.empty_like(z_prev)
    pat.mul(z_prev, prev.scale, x)
    p0, c = prev.split(x)
    ct = _truth_at(c_true_fine, levels[-1], levels)
    out = {"levels": results, "p0": p0.clone(), "c": c.clone(), "seconds": time.perf_counter() - t_all,
           "E_c": relative_error_c(prev, z_prev, ct)}
    prev.close()
    return out
