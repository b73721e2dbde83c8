"""GPU tests of the torch.autograd wrapper and of the reconstruction driver.

* autograd: the backward of WaveOperator equals the library adjoint (up to
  the rounding of the residual that torch forms), matches the float64 oracle
  gradient (rel-L2 <= 1e-3), and matches
  central finite differences of the float32 forward along smooth directions;
* projected L-BFGS (eq. (10)-(11), Alg. 1): the first iterate equals the
  oracle driver's first iterate (rel-L2 <= 1e-3); J decreases monotonically
  over several iterations; the multigrid driver runs coarse -> fine.
"""
import dataclasses

import numpy as np
import pytest

from oracle import kspace, optim
from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce, rel_l2

pytestmark = pytest.mark.gpu


def _small(n=64, K=2, nt=160):
    wl = I.config2(n=n, K=K, nt=nt)
    c_true, p0 = I.phantoms(wl, 2, case=3)
    c_true = c_true.astype(np.float32)
    p0 = p0.astype(np.float32)
    clean, _ = kspace.forward(wl.grid, wl.sensors, c_true.astype(np.float64), p0.astype(np.float64), record=False)
    y, sigma = I.add_noise(clean, seed=2503)
    return wl, c_true, p0, y.astype(np.float32), (1.0 / sigma).astype(np.float32)


def test_autograd_matches_adjoint_oracle_and_fd():
    import torch
    from paper_2505_08482_amd import pat
    from paper_2505_08482_amd.autograd import WaveOperator
    wl, c_true, p0_np, y_np, w_np = _small()
    g = wl.grid
    dev = "cuda"
    plan = pat.Plan(g, wl.K, wl.sensors)
    op = WaveOperator(plan)
    # a heterogeneous iterate: midway between the true medium and 1510 m/s
    c0 = (0.5 * (c_true.astype(np.float64) + 1510.0)).astype(np.float32)
    assert np.ptp(c0) > 10.0
    p0 = torch.from_numpy(p0_np).to(dev).requires_grad_(True)
    c = torch.from_numpy(c0).to(dev).requires_grad_(True)
    y = torch.from_numpy(y_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)

    def loss_fn(p0_, c_):
        d = op(p0_, c_)
        r = (d - y) * w[:, None, None]
        return 0.5 * (r.double() ** 2).sum()

    announce("autograd backward")
    L = loss_fn(p0, c)
    L.backward()
    gp0 = p0.grad.detach().cpu().numpy()
    gc = c.grad.detach().cpu().numpy()
    # oracle gradient of the same objective
    data, hist = kspace.forward(g, wl.sensors, c0.astype(np.float64), p0_np.astype(np.float64))
    resid, J = kspace.misfit(data, y_np.astype(np.float64), w_np.astype(np.float64))
    ogp0, ogc = kspace.adjoint_gradient(g, wl.sensors, c0.astype(np.float64), p0_np.astype(np.float64), resid, hist)
    print(f"[autograd] J gpu {L.item():.9e} oracle {J:.9e}; g_p0 {rel_l2(gp0, ogp0):.2e} g_c {rel_l2(gc, ogc):.2e}")
    assert abs(L.item() - J) <= 1e-5 * J
    assert rel_l2(gp0, ogp0) <= 1e-3
    assert rel_l2(gc, ogc) <= 1e-3
    # finite differences of the float32 forward along smooth directions
    xs = I.pixel_centres(g.nx)
    X, Y = np.meshgrid(xs, xs)
    dc = (np.exp(-((X - 6) ** 2 + (Y + 4) ** 2) / 60.0)).astype(np.float32)
    dp = np.stack([np.exp(-((X + 3) ** 2 + (Y - 5) ** 2) / 30.0)] * wl.K).astype(np.float32)
    with torch.no_grad():
        for name, direction, h, grad in (("c", dc, 2.0, gc), ("p0", dp, 0.05, gp0)):
            dt = torch.from_numpy(direction).to(dev)
            if name == "c":
                Jp = loss_fn(p0.detach(), c.detach() + h * dt).item()
                Jm = loss_fn(p0.detach(), c.detach() - h * dt).item()
            else:
                Jp = loss_fn(p0.detach() + h * dt, c.detach()).item()
                Jm = loss_fn(p0.detach() - h * dt, c.detach()).item()
            fd = (Jp - Jm) / (2 * h)
            an = float(np.sum(grad.astype(np.float64) * direction))
            print(f"[fd] {name}: fd {fd:.6e} adjoint {an:.6e}")
            assert abs(fd - an) <= 2e-2 * abs(an)
    # backward == library adjoint driven by the same residual
    d = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    plan.forward(c.detach(), p0.detach(), d, op.ws, record=True)
    r = ((d - y) * w[:, None, None] ** 2).contiguous()
    g2p = torch.empty_like(p0.detach())
    g2c = torch.empty_like(c.detach())
    plan.adjoint_gradient(c.detach(), p0.detach(), r, g2p, g2c, op.ws)
    np.testing.assert_allclose(g2p.cpu().numpy(), gp0, rtol=1e-5, atol=1e-6 * np.abs(gp0).max())
    plan.close()


def _oracle_problem(wl, y, w, c_lo=1400.0, c_hi=1600.0):
    g = wl.grid
    N, K = g.nx * g.ny, wl.K
    mask = I.mask_disc(g.nx, wl.support_radius_px).reshape(-1)
    lo = np.concatenate([np.zeros(K * N), np.full(N, c_lo)])
    hi = np.concatenate([np.full(K * N, np.inf), np.full(N, c_hi)])
    for k in range(K + 1):
        sl = slice(k * N, (k + 1) * N)
        fixed = 1500.0 if k == K else 0.0
        lo[sl][~mask] = fixed
        hi[sl][~mask] = fixed
    scale = np.concatenate([np.full(K * N, 0.25), np.full(N, (c_hi - c_lo) / 4.0)])

    def fun(x):
        p0 = x[: K * N].reshape(K, g.ny, g.nx)
        c = x[K * N:].reshape(g.ny, g.nx)
        data, hist = kspace.forward(g, wl.sensors, c, p0)
        resid, J = kspace.misfit(data, y, w)
        gp0, gc = kspace.adjoint_gradient(g, wl.sensors, c, p0, resid, hist)
        return J, np.concatenate([gp0.ravel(), gc.ravel()])

    x0 = np.concatenate([np.zeros(K * N), np.full(N, 1500.0)])
    return fun, x0, lo, hi, scale


def test_first_projected_lbfgs_iterate_matches_oracle():
    import torch
    from paper_2505_08482_amd import recon
    wl, c_true, p0, y_np, w_np = _small(nt=140)
    fun, x0, lo, hi, scale = _oracle_problem(wl, y_np.astype(np.float64), w_np.astype(np.float64))
    announce("oracle first iterate")
    x_o, J_o, hist_o = optim.projected_lbfgs(fun, x0, lo, hi, scale=scale, iters=2)
    announce("gpu first iterate")
    prob = recon.Problem(wl, torch.from_numpy(y_np).cuda(), torch.from_numpy(w_np).cuda(), 1400.0, 1600.0)
    z0 = torch.from_numpy(x0.astype(np.float32)).cuda() / prob.scale
    z, J, hist, nit = recon.projected_lbfgs(prob, z0, iters=2)
    x = (z * prob.scale).cpu().numpy()
    print(f"[lbfgs] J oracle {hist_o} gpu {hist}; x rel {rel_l2(x, x_o):.2e}")
    assert len(hist) == len(hist_o)
    np.testing.assert_allclose(hist, hist_o, rtol=1e-4)
    assert rel_l2(x, x_o) <= 1e-3
    prob.close()


def test_reconstruction_decreases_J_and_runs_multigrid():
    import torch
    from paper_2505_08482_amd import recon
    wl, c_true, p0, y_np, w_np = _small(nt=200)
    prob = recon.Problem(wl, torch.from_numpy(y_np).cuda(), torch.from_numpy(w_np).cuda(), 1400.0, 1600.0)
    x0 = torch.cat([torch.zeros(prob.K * prob.N), torch.full((prob.N,), 1500.0)]).cuda()
    announce("gpu 8 iterations")
    z, J, hist, nit = recon.projected_lbfgs(prob, x0 / prob.scale, iters=8)
    print(f"[lbfgs] J {hist}")
    assert nit >= 4
    assert all(b <= a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
    prob.close()
    # two-level multigrid on one physical domain (12.8 mm: 64 px at 0.2 mm -> 128 px at 0.1 mm)
    def level(n, nt, pml):
        dx = 12.8e-3 / n
        g = I.Grid(nx=n, ny=n, dx=dx, dt=I.cfl_dt(dx), nt=nt, pml=pml)
        rs = 5.0e-3 / dx
        return I.Workload(f"mg_{n}", g, K=2, m=48, sensor_radius_px=rs, support_radius_px=rs - 4.0 * n / 128)
    fine, coarse = level(128, 241, 10), level(64, 121, 6)
    c_t, p_t = I.phantoms(fine, 2, case=4)
    clean, _ = kspace.forward(fine.grid, fine.sensors, c_t, p_t, record=False)
    y, sigma = I.add_noise(clean, seed=77)
    announce("gpu multigrid 64 -> 128")
    out = recon.multigrid([coarse, fine], torch.from_numpy(y.astype(np.float32)).cuda(), fine.grid.dt,
                          torch.from_numpy((1.0 / sigma).astype(np.float32)).cuda(),
                          torch.from_numpy(c_t.astype(np.float32)).cuda(), iters=4)
    for lv in out["levels"]:
        print(f"[multigrid] level {lv.n}: iters {lv.iters} J {lv.J[0]:.4e} -> {lv.J[-1]:.4e} E_c {lv.E_c}")
        assert lv.J[-1] <= lv.J[0]
    assert np.isfinite(out["E_c"])


def test_resume_gives_the_uninterrupted_result(tmp_path):
    """A two-level reconstruction stopped in the middle of its first level and
    resumed from the saved state (iterate and L-BFGS pairs), and one stopped
    after its first level, both end with exactly the iterate of the
    uninterrupted run; the JSON-lines log holds one record per iteration."""
    import json
    import torch
    from paper_2505_08482_amd import recon

    def level(n, nt, pml):
        dx = 12.8e-3 / n
        g = I.Grid(nx=n, ny=n, dx=dx, dt=I.cfl_dt(dx), nt=nt, pml=pml)
        rs = 5.0e-3 / dx
        return I.Workload(f"mg_{n}", g, K=2, m=48, sensor_radius_px=rs, support_radius_px=rs - 4.0 * n / 128)
    fine, coarse = level(128, 161, 10), level(64, 81, 6)
    c_t, p_t = I.phantoms(fine, 2, case=5)
    clean, _ = kspace.forward(fine.grid, fine.sensors, c_t, p_t, record=False)
    y, sigma = I.add_noise(clean, seed=78)
    args = (torch.from_numpy(y.astype(np.float32)).cuda(), fine.grid.dt,
            torch.from_numpy((1.0 / sigma).astype(np.float32)).cuda(), torch.from_numpy(c_t.astype(np.float32)).cuda())
    announce("multigrid uninterrupted, 6 + 6 iterations")
    log = tmp_path / "log.jsonl"
    ref = recon.multigrid([coarse, fine], *args, iters=6, log_path=str(log))
    recs = [json.loads(line) for line in open(log)]
    assert len(recs) == sum(lv.iters for lv in ref["levels"])
    assert {"level", "iter", "J", "proj_grad_max", "alpha", "trials", "E_c", "t"} <= set(recs[0])
    st = tmp_path / "state.npz"
    announce("multigrid stopped after 3 iterations of the first level, resumed")
    # an interrupted run: the first level alone for 3 of its 6 iterations, saving its state
    recon.multigrid([coarse], *args, iters=3, save_path=str(st), save_every=3)
    with np.load(st, allow_pickle=False) as f:
        saved = {k: f[k] for k in f.files}
    # the same state as a file of the two-level run
    np.savez(st, level=saved["level"], iters_done=saved["iters_done"], x=saved["x"], z=saved["z"], S=saved["S"],
             Y=saved["Y"], levels=np.array([coarse.grid.nx, fine.grid.nx]))
    res = recon.multigrid([coarse, fine], *args, iters=6, resume=str(st))
    assert torch.equal(res["c"], ref["c"]) and torch.equal(res["p0"], ref["p0"])
    announce("multigrid stopped after the first level, resumed")
    st2 = tmp_path / "state2.npz"
    recon.multigrid([coarse], *args, iters=6, save_path=str(st2), save_every=100)
    with np.load(st2, allow_pickle=False) as f:
        saved = {k: f[k] for k in f.files}
    np.savez(st2, level=saved["level"], iters_done=saved["iters_done"], x=saved["x"], z=saved["z"], S=saved["S"],
             Y=saved["Y"], levels=np.array([coarse.grid.nx, fine.grid.nx]))
    res2 = recon.multigrid([coarse, fine], *args, iters=6, resume=str(st2))
    assert torch.equal(res2["c"], ref["c"]) and torch.equal(res2["p0"], ref["p0"])


@pytest.mark.parametrize("max_halvings", [20, 1])
def test_batched_lbfgs_equals_one_problem_at_a_time(max_halvings):
    """Several reconstructions in lockstep (one batched evaluation per round,
    shared launches) take exactly the iterates each takes alone, and leave
    each problem's p0 gradient at its final iterate; with one trial per line
    search some problems stop early on a rejected trial."""
    import torch
    from paper_2505_08482_amd import pat, recon
    specs = [(64, 2, 90, 1), (64, 1, 70, 2), (96, 2, 80, 3)]
    probs, z0s, ref = [], [], []
    for n, K, nt, case in specs:
        wl = I.config2(n=n, K=K, nt=nt)
        c_t, p_t = I.phantoms(wl, 2, case=case)
        clean, _ = kspace.forward(wl.grid, wl.sensors, c_t, p_t, record=False)
        y, sigma = I.add_noise(clean, seed=90 + case)
        yt = torch.from_numpy(y.astype(np.float32)).cuda()
        wt = torch.from_numpy((1.0 / sigma).astype(np.float32)).cuda()
        prob = recon.Problem(wl, yt, wt, 1400.0, 1600.0)
        x0 = torch.zeros(prob.n, dtype=torch.float32, device="cuda")
        x0[prob.K * prob.N:] = 1500.0
        z0 = torch.empty_like(x0)
        pat.mul(x0, prob.inv_scale, z0)
        announce(f"alone {n} K={K} max_halvings={max_halvings}")
        z, J, hist, nit = recon.projected_lbfgs(prob, z0, iters=6, max_halvings=max_halvings)
        ref.append((z.clone(), list(hist), nit, prob.gp0.clone()))
        probs.append(prob)
        z0s.append(z0)
    announce("lockstep")
    out = recon.batched_projected_lbfgs(probs, z0s, iters=6, max_halvings=max_halvings)
    for (z, J, hist, nit), (zr, hr, nr, gr), p in zip(out, ref, probs):
        assert nit == nr and hist == hr, (hist, hr)
        assert torch.equal(z, zr)
        assert torch.equal(p.gp0, gr)       # the final iterate's p0 gradient
    for p in probs:
        p.close()
