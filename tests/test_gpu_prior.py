"""GPU parity of the Ornstein-Uhlenbeck prior terms of eq. (4) (Sec. 4.1.2)
against the dense float64 oracle (oracle/prior.py), through the C ABI:
the exact product Xi v, and the prior value and gradient from the
conjugate-gradient solve, on a disc mask and on Table 1's target squares."""
import numpy as np
import pytest

from oracle import prior
from paper_2505_08482_amd import inputs as I
from gpu_helpers import announce, rel_l2

pytestmark = pytest.mark.gpu


def _disc(ny, nx, r):
    Y, X = np.meshgrid(np.arange(ny) - (ny - 1) / 2, np.arange(nx) - (nx - 1) / 2, indexing="ij")
    return X ** 2 + Y ** 2 <= r * r


def test_exact_product_on_a_disc_mask():
    import torch
    from paper_2505_08482_amd import pat
    ny, nx, dx, tau = 30, 26, 0.2e-3, 1.5e-3
    mask = _disc(ny, nx, 11.5)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((2, ny, nx)).astype(np.float32)
    announce("ou product 30x26 disc")
    ou = pat.OuPrior(ny, nx, dx, tau, mask)
    out = torch.empty((2, ny, nx), dtype=torch.float32, device="cuda")
    ou.apply(torch.from_numpy(v).cuda(), out)
    Xi = prior.ou_correlation(ny, nx, dx, tau, mask)
    for k in range(2):
        ref = np.zeros((ny, nx))
        ref[mask] = Xi @ v[k][mask].astype(np.float64)
        got = out[k].cpu().numpy()
        assert np.all(got[~mask] == 0.0)
        assert rel_l2(got, ref) <= 2e-6, rel_l2(got, ref)
    ou.close()


@pytest.mark.parametrize("level", ["mg1", "mg3"])
def test_prior_value_and_gradient_on_table1_target(level):
    import torch
    from paper_2505_08482_amd import pat
    wl = I.paper_level(level, K=2)
    g = wl.grid
    mask = wl.mask()
    rng = np.random.default_rng(5)
    # two initial pressures and a sound speed, each with its own mean and sigma
    z = np.stack([10.0 * rng.uniform(0, 1, (g.ny, g.nx)), 10.0 * rng.uniform(0, 1, (g.ny, g.nx)),
                  1505.0 + 40.0 * rng.standard_normal((g.ny, g.nx))]).astype(np.float32)
    eta = np.array([5.0, 5.0, 1505.0], dtype=np.float32)
    sig = np.array([2.5, 2.5, 37.5])
    tau = 1.5e-3
    announce(f"ou prior {level} box {int(mask.any(1).sum())}")
    ou = pat.OuPrior(g.ny, g.nx, g.dx, tau, mask)
    grad = torch.empty((3, g.ny, g.nx), dtype=torch.float32, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    it = ou.prior(torch.from_numpy(z).cuda(), torch.from_numpy(eta).cuda(),
                  torch.from_numpy((1.0 / sig ** 2).astype(np.float32)).cuda(), grad, J, tol=1e-7, maxit=2000)
    Jo, go = 0.0, []
    for k in range(3):
        j, gk = prior.ou_prior(z[k].astype(np.float64), float(eta[k]), sig[k], g.dx, tau, mask)
        Jo += j
        go.append(gk)
    go = np.stack(go)
    e_g = rel_l2(grad.cpu().numpy(), go)
    print(f"[ou] {level}: CG iterations {it}, J {J.item():.9e} vs {Jo:.9e}, grad rel {e_g:.2e}", flush=True)
    assert it < 2000
    assert abs(J.item() - Jo) <= 1e-4 * Jo
    assert e_g <= 1e-4
    ou.close()
