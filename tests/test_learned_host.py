"""Host-side logic of the learned start (no GPU): the layer table agrees with
the oracle's architecture, the parameter layout keeps every bf16 weight block
16-byte aligned, and stored weights (if present) have the table's shapes."""
import os

import numpy as np
import pytest

from oracle import unet as U
from paper_2505_08482_amd import learned


def test_layer_table_matches_oracle_architecture():
    for cin, base in ((8, 32), (8, 8), (16, 16)):
        assert learned.layer_table(cin, base) == U.layer_shapes(cin, base)


def test_parameter_layout_alignment_and_size():
    off, n_params = 0, 0
    for name, ci, co in learned.layer_table(8, 32):
        assert off % 8 == 0, name            # weight block starts on 8 bf16 = 16 bytes
        off += co * 9 * ci + co
        n_params += co * 9 * ci + co
    assert off % 8 == 0                      # the head's weights too
    n_params += 32 + 1
    assert 1.9e6 < n_params < 2.0e6


@pytest.mark.skipif(not os.path.exists(learned.DEFAULT_WEIGHTS), reason="no trained weights in the package")
def test_stored_weights_have_the_table_shapes():
    with np.load(learned.DEFAULT_WEIGHTS, allow_pickle=False) as f:
        base, cin = int(f["base"][0]), int(f["cin"][0])
        for name, ci, co in learned.layer_table(cin, base):
            w = f[name + ".w"]
            assert w.shape == (co, 9, ci) and f[name + ".b"].shape == (co,)
            if w.dtype == np.uint16:                   # bfloat16 bit patterns
                w = (w.astype(np.uint32) << 16).view(np.float32)
            assert np.all(np.isfinite(w))
            # trained from He-normal initialisation (std sqrt(2 / (9 cin))): the scale stays of that order
            assert 0.1 < w.std() / np.sqrt(2.0 / (9 * ci)) < 10.0, name
        assert f["head.w"].shape == (base,) and f["head.b"].shape == (1,)
