"""Pins of the learned-start network oracle (oracle/unet.py)."""
import numpy as np
import scipy.signal

from oracle import unet as U


def test_conv_matches_library_correlation():
    """Zero-padded 3x3 cross-correlation per (output, input) channel pair,
    summed over inputs, plus the bias: ``scipy.signal.correlate2d``."""
    rng = np.random.default_rng(0)
    B, H, W, Ci, Co = 2, 7, 5, 3, 4
    x = rng.standard_normal((B, H, W, Ci))
    w = rng.standard_normal((Co, 9, Ci))
    b = rng.standard_normal(Co)
    y = U.conv3x3(x, w, b)
    for bb in range(B):
        for o in range(Co):
            ref = np.full((H, W), b[o])
            for c in range(Ci):
                ker = w[o, :, c].reshape(3, 3)      # tap t = 3 (di+1) + (dj+1)
                ref += scipy.signal.correlate2d(x[bb, :, :, c], ker, mode="same", boundary="fill")
            assert np.allclose(y[bb, :, :, o], ref, rtol=0, atol=1e-12)


def test_conv_identity_and_shift_kernels():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 6, 6, 2))
    w = np.zeros((2, 9, 2))
    w[:, 4, :] = np.eye(2)                      # centre tap: identity
    assert np.array_equal(U.conv3x3(x, w, np.zeros(2)), x)
    w = np.zeros((2, 9, 2))
    w[:, 5, :] = np.eye(2)                      # tap (0, +1): y[i, j] = x[i, j + 1]
    y = U.conv3x3(x, w, np.zeros(2))
    assert np.array_equal(y[:, :, :-1], x[:, :, 1:]) and np.all(y[:, :, -1] == 0)
    w = np.zeros((2, 9, 2))
    w[:, 0, :] = np.eye(2)                      # tap (-1, -1): y[i, j] = x[i - 1, j - 1]
    y = U.conv3x3(x, w, np.zeros(2))
    assert np.array_equal(y[:, 1:, 1:], x[:, :-1, :-1]) and np.all(y[:, 0] == 0) and np.all(y[:, :, 0] == 0)


def test_conv_backward_adjoint_identities():
    rng = np.random.default_rng(2)
    B, H, W, Ci, Co = 2, 6, 9, 3, 5
    x = rng.standard_normal((B, H, W, Ci))
    w = rng.standard_normal((Co, 9, Ci))
    dy = rng.standard_normal((B, H, W, Co))
    dx, dw, db = U.conv3x3_backward(x, w, dy)
    zero = np.zeros(Co)
    # <A x, dy> = <x, A^T dy> for the linear map x -> conv(x, w, 0)
    assert np.isclose(np.sum(U.conv3x3(x, w, zero) * dy), np.sum(x * dx), rtol=1e-12)
    # <dw, v> = <conv(x, v, 0), dy> for the linear map w -> conv(x, w, 0)
    v = rng.standard_normal(w.shape)
    assert np.isclose(np.sum(dw * v), np.sum(U.conv3x3(x, v, zero) * dy), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_pool_and_upsample():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 6, 3))
    y = rng.standard_normal((2, 8, 12, 3))
    assert np.array_equal(U.avgpool2(U.upsample2(x)), x)
    # up and pool are adjoint up to the factor 4: <up x, y> = <x, up^T y> = 4 <x, pool y>
    assert np.isclose(np.sum(U.upsample2(x) * y), np.sum(x * U.upsample2_backward(y)), rtol=1e-12)
    assert np.isclose(np.sum(U.upsample2(x) * y), 4.0 * np.sum(x * U.avgpool2(y)), rtol=1e-12)
    assert np.isclose(np.sum(U.avgpool2(y) * x), np.sum(y * U.avgpool2_backward(x)), rtol=1e-12)
    # a constant stays constant
    assert np.allclose(U.upsample2(np.full((1, 2, 2, 1), 3.5)), 3.5)


def _loss(p, x, t, mask):
    r, _ = U.unet_forward(p, x)
    return U.masked_mse(r, t, mask)[0]


def test_network_gradient_matches_finite_differences():
    """Tiny network (base 2 channels, 16 x 16 input, batch 2), every layer
    perturbed; the head starts non-zero so that all layers receive gradient."""
    rng = np.random.default_rng(4)
    cin, base = 3, 2
    p = U.init_params(cin, base, seed=5)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["head.w"] = rng.standard_normal(base)
    x = rng.standard_normal((2, 16, 16, cin))
    t = rng.standard_normal((2, 16, 16))
    mask = np.ones((16, 16), dtype=bool)
    mask[:3] = False
    r, cache = U.unet_forward(p, x)
    L, dr = U.masked_mse(r, t, mask)
    g = U.unet_backward(p, cache, dr)
    assert set(g) == set(p) | {"input"}
    h = 1e-6
    checked = 0
    for name in list(p) + ["input"]:
        arr = x if name == "input" else p[name]
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp = _loss(p, x, t, mask)
            flat[idx] = old - h
            Lm = _loss(p, x, t, mask)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (name, idx, fd, an)
            checked += 1
    assert checked >= 3 * 15


def test_masked_mse_gradient_and_adam_first_step():
    rng = np.random.default_rng(6)
    r = rng.standard_normal((2, 4, 4))
    t = rng.standard_normal((2, 4, 4))
    mask = rng.random((4, 4)) > 0.3
    L, dr = U.masked_mse(r, t, mask)
    n = 2 * mask.sum()
    assert np.isclose(L, 0.5 * np.sum(((r - t) * mask) ** 2) / n)
    assert np.allclose(dr, (r - t) * mask / n)
    # Adam at t = 1 from zero moments: the step is lr * g / (|g| + eps)
    w = rng.standard_normal(10)
    g = rng.standard_normal(10)
    w1, m, v = U.adam_step(w, g, np.zeros(10), np.zeros(10), 1, lr=1e-3)
    assert np.allclose(w - w1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    # exactly representable values are kept; halfway cases go to the even neighbour
    assert U.bf16_round(np.array([1.0, -2.5, 0.0]))[1] == -2.5
    one_ulp = 2.0 ** -7                                 # spacing of bf16 at 1.0
    assert U.bf16_round(np.array([1.0 + one_ulp / 2]))[0] == 1.0          # tie -> even (1.0)
    assert U.bf16_round(np.array([1.0 + 1.5 * one_ulp]))[0] == 1.0 + 2 * one_ulp
    assert U.bf16_round(np.array([1.0 + 0.49 * one_ulp]))[0] == 1.0
    x = np.random.default_rng(7).standard_normal(1000)
    assert np.max(np.abs(U.bf16_round(x) - x) / np.abs(x)) <= 2.0 ** -8


def test_storage_rounding_mode():
    """``store`` is applied to every tensor kept between layers: with
    bf16_round every cached value is a bfloat16 number, the identity reproduces
    the full-precision run bit for bit, and the rounded run stays within a few
    bfloat16 roundings of it."""
    rng = np.random.default_rng(8)
    p = U.init_params(8, 8, seed=9)
    p["head.w"] = rng.standard_normal(8)
    x = U.bf16_round(rng.standard_normal((2, 16, 16, 8)))
    r0, c0 = U.unet_forward(p, x)
    r1, c1 = U.unet_forward(p, x, store=lambda a: a)
    assert np.array_equal(r0, r1)
    rb, cb = U.unet_forward(p, x, store=U.bf16_round)
    for k, v in cb.items():
        assert np.array_equal(U.bf16_round(v), v), k
    assert np.linalg.norm(rb - r0) / np.linalg.norm(r0) < 2e-2
    dr = rng.standard_normal(r0.shape)
    g0 = U.unet_backward(p, c0, dr)
    g1 = U.unet_backward(p, c0, dr, store=lambda a: a)
    assert all(np.array_equal(g0[k], g1[k]) for k in g0)
    gb = U.unet_backward(p, cb, dr, store=U.bf16_round)
    num = sum(np.sum((gb[k] - g0[k]) ** 2) for k in g0 if k != "input")
    den = sum(np.sum(g0[k] ** 2) for k in g0 if k != "input")
    assert np.sqrt(num / den) < 0.1
