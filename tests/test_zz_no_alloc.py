"""The allocation-free two-loop recursion (pat_lbfgs_direction_noalloc, whose
scratch is the library's static per-GPU array) against pat_lbfgs_direction
with a caller-owned scratch buffer, through the C ABI: bit-identical
directions on two calls in a row, the second with a smaller vector and fewer
pairs (the static array keeps the first call's contents), and a clear
refusal above the array's size."""
import ctypes

import numpy as np
import pytest

from paper_2505_08482_amd import pat
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _pairs(rng, n, npairs, device):
    import torch
    s = [torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(device) for _ in range(npairs)]
    # y_j = A s_j + noise for an SPD diagonal A: positive curvature y^T s > 0
    a = torch.from_numpy(rng.uniform(0.5, 2.0, n).astype(np.float32)).to(device)
    y = [a * sj + 0.01 * torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(device) for sj in s]
    g = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(device)
    return g, s, y


def test_noalloc_equals_scratch_version_two_calls():
    import torch
    dev = "cuda"
    rng = np.random.default_rng(123)
    for n, npairs in ((1_000_003, 20), (4099, 3)):
        announce(f"lbfgs noalloc n={n} pairs={npairs}")
        g, s, y = _pairs(rng, n, npairs, dev)
        ref = torch.empty_like(g)
        scratch = torch.empty(pat.lbfgs_scratch_bytes(npairs), dtype=torch.uint8, device=dev)
        pat.lbfgs_direction(g, s, y, ref, scratch)
        out = torch.full_like(g, float("nan"))
        pat.lbfgs_direction_noalloc(g, s, y, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        print(f"[noalloc] n={n} pairs={npairs}: equal={np.array_equal(a, b)} "
              f"max|diff|={np.max(np.abs(a - b)):.3e}", flush=True)
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)


def test_noalloc_refuses_too_many_pairs():
    import torch
    n = 64
    npairs = pat.LBFGS_NOALLOC_MAX_PAIRS + 1
    g = torch.zeros(n, dtype=torch.float32, device="cuda")
    vecs = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(npairs)]
    with pytest.raises(pat.PatError) as e:
        pat.lbfgs_direction_noalloc(g, vecs, vecs, torch.empty_like(g))
    assert e.value.status == pat.PAT_EUNSUPPORTED
    L = pat.lib()
    assert L.pat_lbfgs_direction_noalloc(0, None, 0, None, None, None, None) == pat.PAT_EINVAL
