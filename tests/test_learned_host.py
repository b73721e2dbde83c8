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


def test_evaluation_summary_counts_and_means():
    """The held-out summary counts each start's cases that reach a target and
    averages time and iterations over those only; the plain multigrid run's
    fine-start error is its first fine-level iterate."""
    rows = [
        {"plain_multigrid": {"E_c": [1.5, 1.2], "to_target": {"2": {"iterations": 81, "seconds": 8.0}, "1": None}},
         "interpolated": {"E_c_start": 2.5, "to_target": {"2": None, "1": None}},
         "learned": {"E_c_start": 0.8, "to_target": {"2": {"iterations": 40, "seconds": 2.0},
                                                    "1": {"iterations": 40, "seconds": 2.0}}}},
        {"plain_multigrid": {"E_c": [0.9], "to_target": {"2": {"iterations": 81, "seconds": 10.0},
                                                         "1": {"iterations": 81, "seconds": 10.0}}},
         "interpolated": {"E_c_start": 1.5, "to_target": {"2": {"iterations": 40, "seconds": 3.0}, "1": None}},
         "learned": {"E_c_start": 1.2, "to_target": {"2": {"iterations": 40, "seconds": 2.2},
                                                    "1": {"iterations": 42, "seconds": 4.0}}}},
    ]
    fig, table = learned.summarize(rows)
    assert fig["cases"] == 2
    pm, it, ln = fig["plain_multigrid"], fig["interpolated"], fig["learned"]
    assert pm["E_c_start_mean"] == 1.2 and pm["2"]["reached"] == 2 and pm["2"]["seconds_mean"] == 9.0
    assert pm["1"]["reached"] == 1 and pm["1"]["seconds_mean"] == 10.0
    assert it["2"]["reached"] == 1 and it["2"]["seconds_mean"] == 3.0 and it["1"]["reached"] == 0
    assert it["1"]["seconds_mean"] is None
    assert ln["1"]["reached"] == 2 and ln["1"]["iterations_mean"] == 41.0 and ln["E_c_start_median"] == 1.0
    assert table.count("\n") == 4 and "0/2" in table
