"""What the trained network gains over the method without it: on held-out
phantoms (the 256^2 workload's generators at 512^2, seeds 5000 + case, never
used in training), the fine level is started from the network's proposal and
from the plain interpolation of the same coarse iterate (Sec. 3.1); plain
gradient iterations then run from both."""
import os

import numpy as np
import pytest

from tests.gpu_helpers import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_08482_amd import learned  # noqa: E402

WEIGHTS = learned.DEFAULT_WEIGHTS


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights in the package")
def test_learned_start_beats_interpolation_on_held_out_phantom():
    announce("learned start, held-out case 0 (512^2, K = 8)")
    net = learned.load_weights(WEIGHTS)
    res = learned.evaluate_case(net, case=0, fine_iters=3, targets=(), plain_multigrid=False,
                                log=lambda s: print("[learned]", s, flush=True))
    e_int = res["interpolated"]["E_c_start"]
    e_net = res["learned"]["E_c_start"]
    print(f"[learned] E_c at the fine start: interpolated {e_int:.3f} %, learned {e_net:.3f} %; after 3 fine "
          f"iterations: {res['interpolated']['E_c_last']:.3f} % vs {res['learned']['E_c_last']:.3f} %", flush=True)
    assert e_net < 0.9 * e_int
    assert res["learned"]["E_c_last"] <= res["interpolated"]["E_c_last"]
