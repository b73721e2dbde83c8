"""The C-ABI library loads and exports every entry point declared in
include/pat.h and include/pat_nn.h (no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

from paper_2505_08482_amd import nn, pat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header=None):
    names = set()
    for h in ([header] if header else ["pat.h", "pat_nn.h"]):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(pat_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_and_binding_agree():
    assert _declared("pat.h") == sorted(pat.EXPORTS)
    assert _declared("pat_nn.h") == sorted(nn.EXPORTS)


@pytest.mark.skipif(not os.path.exists(pat.LIB_PATH), reason="libpat.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pat.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(pat.LIB_PATH), reason="libpat.so not built")
def test_host_side_argument_checks():
    """Invalid arguments are rejected before anything touches a device."""
    L = pat.lib()
    assert L.pat_plan_create(None, 1, 1, None, None) == pat.PAT_EINVAL
    g = pat.pat_grid(100, 100, 10, 10, 1e-4, 1e-8, 1600.0, 1000.0, 2.0)   # 100 has no radix plan
    xy = (ctypes.c_double * 2)(0.0, 0.0)
    h = ctypes.c_void_p()
    assert L.pat_plan_create(ctypes.byref(g), 1, 1, xy, ctypes.byref(h)) == pat.PAT_EUNSUPPORTED
    g = pat.pat_grid(64, 64, 0, 10, 1e-4, 1e-8, 1600.0, 1000.0, 2.0)      # nt = 0
    assert L.pat_plan_create(ctypes.byref(g), 1, 1, xy, ctypes.byref(h)) == pat.PAT_EINVAL
    assert L.pat_project_update(-1, None, None, 1.0, None, None, 0.0, 1.0, None) == pat.PAT_EINVAL
    assert L.pat_prolong(0, None, 1, 1, None, 1, 1, None) == pat.PAT_EINVAL
    assert pat.status_string(pat.PAT_EWORKSPACE).startswith("workspace")
    g = pat.pat_grid(64, 64, 10, 8, 1e-4, 1e-8, 1600.0, 1000.0, 2.0)
    assert L.pat_plan_create(ctypes.byref(g), 65, 1, xy, ctypes.byref(h)) == pat.PAT_EUNSUPPORTED   # K > 64
    far = (ctypes.c_double * 2)(0.0, 40e-4)                                                     # off the grid
    assert L.pat_plan_create(ctypes.byref(g), 1, 1, far, ctypes.byref(h)) == pat.PAT_EINVAL
    nan = (ctypes.c_double * 2)(float("nan"), 0.0)
    assert L.pat_plan_create(ctypes.byref(g), 1, 1, nan, ctypes.byref(h)) == pat.PAT_EINVAL
    g = pat.pat_grid(64, 64, 10, 32, 1e-4, 1e-8, 1600.0, 1000.0, 2.0)     # PML covers the grid
    assert L.pat_plan_create(ctypes.byref(g), 1, 1, xy, ctypes.byref(h)) == pat.PAT_EINVAL
    assert L.pat_prolong_phys(1, None, 4, 4, 1e-4, None, 8, 8, 5e-5, None) == pat.PAT_EINVAL
    dummy = ctypes.c_void_p(1)
    assert L.pat_prolong_phys(1, dummy, 4, 4, 0.0, dummy, 8, 8, 5e-5, None) == pat.PAT_EINVAL
    assert L.pat_batch_gradient(0, None, 1, None) == pat.PAT_EINVAL
    out = ctypes.c_void_p()
    assert L.pat_history_field(None, dummy, 0, ctypes.byref(out)) == pat.PAT_EINVAL
    assert L.pat_batch_gradient(1, dummy, 17, None) == pat.PAT_EINVAL
    assert L.pat_trace_start(0) == pat.PAT_EINVAL
    assert L.pat_plan_set_tile(None, 0) == pat.PAT_EINVAL
    # prior operator: refused before any device allocation
    oh = ctypes.c_void_p()
    assert L.pat_ou_create(0, 8, 1e-4, 1e-3, None, ctypes.byref(oh)) == pat.PAT_EINVAL
    assert L.pat_ou_create(8, 8, 1e-4, 0.0, None, ctypes.byref(oh)) == pat.PAT_EINVAL
    empty = (ctypes.c_uint8 * 64)()
    assert L.pat_ou_create(8, 8, 1e-4, 1e-3, empty, ctypes.byref(oh)) == pat.PAT_EINVAL   # empty mask
    assert L.pat_ou_create(300, 300, 1e-4, 1e-3, None, ctypes.byref(oh)) == pat.PAT_EUNSUPPORTED   # L > 512


@pytest.mark.skipif(not os.path.exists(pat.LIB_PATH), reason="libpat.so not built")
def test_nn_host_side_argument_checks():
    """The learned-start layers refuse bad shapes, misaligned pointers and short
    scratch before launching anything."""
    L = nn.lib()
    d16 = ctypes.c_void_p(1 << 20)        # 16-byte aligned stand-in, never dereferenced
    odd = ctypes.c_void_p((1 << 20) + 2)  # misaligned
    # cin not a multiple of 8, ld below the channel count, misaligned input
    assert L.pat_nn_conv3x3(1, 8, 8, d16, 12, 12, d16, None, d16, 32, 32, 1, 0, None, 0, None) == pat.PAT_EINVAL
    assert L.pat_nn_conv3x3(1, 8, 8, d16, 8, 16, d16, None, d16, 32, 32, 1, 0, None, 0, None) == pat.PAT_EINVAL
    assert L.pat_nn_conv3x3(1, 8, 8, odd, 16, 16, d16, None, d16, 32, 32, 1, 0, None, 0, None) == pat.PAT_EINVAL
    assert L.pat_nn_conv3x3(0, 8, 8, d16, 16, 16, d16, None, d16, 32, 32, 1, 0, None, 0, None) == pat.PAT_EINVAL
    size = ctypes.c_size_t(0)
    assert L.pat_nn_wgrad_scratch_bytes(2, 16, 16, 32, 64, ctypes.byref(size)) == pat.PAT_OK and size.value > 0
    need = size.value
    assert L.pat_nn_conv3x3_wgrad(2, 16, 16, d16, 32, 32, d16, 64, 64, d16, None, d16, need - 4,
                                  None) == pat.PAT_EWORKSPACE
    assert L.pat_nn_conv3x3_wgrad(2, 16, 16, d16, 32, 32, d16, 64, 60, d16, None, d16, need, None) == pat.PAT_EINVAL
    assert L.pat_nn_avgpool2(1, 7, 8, 8, d16, 8, d16, 8, None) == pat.PAT_EINVAL          # odd height
    assert L.pat_nn_upsample2(1, 8, 8, 12, d16, 16, d16, 16, None) == pat.PAT_EINVAL      # C % 8
    assert L.pat_nn_head_backward(10, 24, d16, 24, d16, d16, d16, 24, d16, d16, d16, 1 << 20,
                                  None) == pat.PAT_EINVAL                                # 24 does not divide 256
    assert L.pat_nn_masked_mse(1, 16, d16, d16, d16, d16, d16, d16, 8, None) == pat.PAT_EWORKSPACE
    assert L.pat_nn_adam(10, d16, d16, d16, d16, None, 0, 1e-3, 0.9, 0.999, 1e-8, None) == pat.PAT_EINVAL
    assert L.pat_nn_pack_input(8, 16, 1, d16, d16, None, 4, 1500.0, 100.0, d16, d16, None, d16, 1 << 12,
                               None) == pat.PAT_EINVAL                                   # transpose of a non-square
    assert L.pat_nn_pack_input(8, 8, 1, d16, d16, None, 0, 1500.0, 100.0, d16, d16, d16, d16, 1 << 12,
                               None) == pat.PAT_EINVAL                                   # target without c_true


@pytest.mark.skipif(not os.path.exists(pat.LIB_PATH), reason="libpat.so not built")
def test_library_and_oracle_accept_the_same_sensor_positions():
    """A sensor is accepted where its four bilinear taps lie on the grid
    (fractional cell-centre index in [0, n - 1) on each axis), by the library
    and by the oracle alike; the spacing is a power of two, so the positions
    are exact.  Without a GPU an accepted plan fails at its first device
    allocation (PAT_EHIP), after every host table has been built."""
    import numpy as np
    from oracle import sensors as osens
    L = pat.lib()
    nx, ny, dx = 64, 48, 1.0 / 8192
    g = pat.pat_grid(nx, ny, 10, 4, dx, 1e-8, 1600.0, 1000.0, 2.0)
    fx_cases = [0.0, 1e-9, 31.5, nx - 1 - 1e-9, nx - 1.0, -1e-9, nx + 3.0]
    fy_cases = [0.0, ny - 1 - 1e-9, ny - 1.0, -1e-9]
    for fx in fx_cases:
        for fy in fy_cases:
            x, y = (fx + 0.5 - nx / 2) * dx, (fy + 0.5 - ny / 2) * dx
            xy = (ctypes.c_double * 2)(x, y)
            h = ctypes.c_void_p()
            st = L.pat_plan_create(ctypes.byref(g), 1, 1, xy, ctypes.byref(h))
            if st == pat.PAT_OK:
                L.pat_plan_destroy(h)
            assert st in (pat.PAT_OK, pat.PAT_EHIP, pat.PAT_EINVAL), st
            try:
                osens.sensor_matrix(nx, ny, dx, np.array([[x, y]]))
                oracle_ok = True
            except ValueError:
                oracle_ok = False
            inside = 0 <= fx < nx - 1 and 0 <= fy < ny - 1
            assert oracle_ok == inside, (fx, fy)
            assert (st != pat.PAT_EINVAL) == inside, (fx, fy, st)
