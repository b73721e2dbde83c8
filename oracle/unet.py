"""Learned fine-level start for the sound speed: a 4-level U-Net, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
The multigrid continuation of Sec. 3.1 starts each finer level from the
coarse iterate, linearly interpolated.  The learned start replaces that
interpolation for the sound speed: a small convolutional network reads the
coarse sound speed and the summed initial-pressure gradient (both interpolated
onto the fine grid) and proposes a correction added to the interpolated sound
speed.  The network and its training rule are not part of the paper; they are
the plain textbook definitions written out:

* 3 x 3 convolution with zero padding ("same" size), channels last:
  ``y[b,i,j,o] = bias[o] + sum_{t,c} x[b, i+di_t, j+dj_t, c] * w[o,t,c]``,
  tap ``t = 3 (di+1) + (dj+1)`` for ``di, dj`` in {-1, 0, 1};
* ReLU ``max(v, 0)`` with derivative ``[v > 0]``;
* 2 x 2 average pooling and 2 x 2 nearest-neighbour upsampling;
* a 1 x 1 output head ``r[b,i,j] = bias + sum_c w[c] x[b,i,j,c]``;
* loss ``L = 1/(2 n) sum_{masked pixels} (r - t)^2`` (n = masked pixels x batch);
* Adam (Kingma & Ba, 2015) with bias correction.

Architecture (``base`` channels ``C_l = base 2^l``, l = 0..3, resolutions
``H / 2^l``): encoder ``e_l = relu(conv(relu(conv(in_l))))`` with
``in_0`` = the input and ``in_{l+1} = avgpool(e_l)``; decoder from the bottom
``d_3 = e_3``: ``cat_l = [e_l, up(d_{l+1})]`` (skip channels first),
``d_l = relu(conv(relu(conv(cat_l))))``; output ``head(d_0)``.  Layer names:
``e{l}a, e{l}b`` (l = 0..3), ``d{l}a, d{l}b`` (l = 2, 1, 0), ``head``.  Weights
``w [C_out][9][C_in]``, biases ``b [C_out]``; the head has ``w [C]`` and a
scalar ``b``.

Every backward function is the derivative of its forward written out from the
definition (no automatic differentiation).

Pins (tests/test_oracle_unet.py)
--------------------------------
* the convolution equals ``scipy.signal.correlate2d`` (zero fill) summed over
  input channels, and special kernels give the identity and pure shifts;
* its backward satisfies the adjoint identities ``<conv(x), dy> = <x, dx>``
  (no bias) and ``<dw, v> = <conv_v(x), dy>``, and ``db = sum dy``;
* pooling and upsampling are adjoint up to the factor 4 and
  ``avgpool(up(x)) = x``;
* the whole network's gradient equals central finite differences of the loss
  (weights, biases and the input);
* Adam's first step moves each parameter by ``lr g / (|g| + eps)``.

With ``store=bf16_round`` the forward and backward round every tensor kept
between layers to bfloat16 (the storage precision of the GPU layers), so that
ReLU decisions are taken on the same values as there; the full-precision
default is what the pins above check, and the gap between the two is the cost
of bfloat16 storage.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

LEVELS = 4


def _shift(x: np.ndarray, di: int, dj: int) -> np.ndarray:
    """``s[b,i,j,:] = x[b, i+di, j+dj, :]`` with zeros outside the image."""
    B, H, W, C = x.shape
    s = np.zeros_like(x)
    i0, i1 = max(0, -di), min(H, H - di)
    j0, j1 = max(0, -dj), min(W, W - dj)
    s[:, i0:i1, j0:j1, :] = x[:, i0 + di:i1 + di, j0 + dj:j1 + dj, :]
    return s


TAPS = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """``x [B][H][W][Ci]``, ``w [Co][9][Ci]``, ``b [Co]`` -> ``[B][H][W][Co]``."""
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (di, dj) in enumerate(TAPS):
        y += _shift(x, di, dj) @ w[:, t, :].T
    return y + b


def conv3x3_data_gradient(w: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """``dx`` of ``sum(dy * conv3x3(x, w, b))``: y[p] gathers x[p + d], so
    x[q] receives from y[q - d] through tap d."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (di, dj) in enumerate(TAPS):
        dx += _shift(dy @ w[:, t, :], -di, -dj)
    return dx


def conv3x3_weight_gradient(x: np.ndarray, dy: np.ndarray):
    """``(dw, db)`` of ``sum(dy * conv3x3(x, w, b))``: the sum over pixels of
    ``dy[p][o] x[p + d][c]`` for every tap d (one matrix product per tap)."""
    cout, cin = dy.shape[-1], x.shape[-1]
    dw = np.zeros((cout, 9, cin))
    d2 = dy.reshape(-1, cout)
    for t, (di, dj) in enumerate(TAPS):
        dw[:, t, :] = d2.T @ _shift(x, di, dj).reshape(-1, cin)
    return dw, dy.sum(axis=(0, 1, 2))


def conv3x3_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients ``(dx, dw, db)`` of ``sum(dy * conv3x3(x, w, b))``."""
    dw, db = conv3x3_weight_gradient(x, dy)
    return conv3x3_data_gradient(w, dy), dw, db


def relu(v: np.ndarray) -> np.ndarray:
    return np.maximum(v, 0.0)


def relu_backward(y: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """``dy * [v > 0]`` written with the output ``y = relu(v)`` (``v > 0`` iff ``y > 0``)."""
    return dy * (y > 0.0)


def avgpool2(x: np.ndarray) -> np.ndarray:
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(dy: np.ndarray) -> np.ndarray:
    return 0.25 * upsample2(dy)


def upsample2(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dy: np.ndarray) -> np.ndarray:
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def head(x: np.ndarray, w: np.ndarray, b: float) -> np.ndarray:
    return x @ w + b


def head_backward(x: np.ndarray, w: np.ndarray, dr: np.ndarray):
    return dr[..., None] * w, np.einsum("bij,bijc->c", dr, x), float(dr.sum())


def layer_shapes(cin: int, base: int) -> List[Tuple[str, int, int]]:
    """``(name, C_in, C_out)`` of every 3 x 3 convolution, in forward order."""
    C = [base * 2 ** l for l in range(LEVELS)]
    out = []
    prev = cin
    for l in range(LEVELS):
        out += [(f"e{l}a", prev, C[l]), (f"e{l}b", C[l], C[l])]
        prev = C[l]
    for l in range(LEVELS - 2, -1, -1):
        out += [(f"d{l}a", C[l] + C[l + 1], C[l]), (f"d{l}b", C[l], C[l])]
    return out


def init_params(cin: int, base: int, seed: int) -> Dict[str, np.ndarray]:
    """He-normal convolution weights, zero biases, zero head (the untrained
    network proposes no correction)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in layer_shapes(cin, base):
        p[name + ".w"] = rng.standard_normal((co, 9, ci)) * np.sqrt(2.0 / (9 * ci))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = np.zeros(base)
    p["head.b"] = np.zeros(1)
    return p


def _same(a: np.ndarray) -> np.ndarray:
    return a


def unet_forward(p: Dict[str, np.ndarray], x: np.ndarray, store=None):
    """Output ``r [B][H][W]`` and the cache of every layer output.

    ``store`` (optional) is applied to every tensor the network keeps between
    layers (layer outputs, pooled maps), e.g. ``bf16_round`` to take every
    stored value, and so every ReLU decision downstream, in the precision of
    a bfloat16-storage implementation; the default keeps full precision."""
    keep = store or _same
    cache = {"in0": x}
    h = x
    for l in range(LEVELS):
        if l > 0:
            h = keep(avgpool2(cache[f"e{l - 1}b"]))
            cache[f"in{l}"] = h
        a = keep(relu(conv3x3(h, p[f"e{l}a.w"], p[f"e{l}a.b"])))
        cache[f"e{l}a"] = a
        h = keep(relu(conv3x3(a, p[f"e{l}b.w"], p[f"e{l}b.b"])))
        cache[f"e{l}b"] = h
    d = cache[f"e{LEVELS - 1}b"]
    for l in range(LEVELS - 2, -1, -1):
        cat = np.concatenate([cache[f"e{l}b"], upsample2(d)], axis=-1)
        cache[f"cat{l}"] = cat
        a = keep(relu(conv3x3(cat, p[f"d{l}a.w"], p[f"d{l}a.b"])))
        cache[f"d{l}a"] = a
        d = keep(relu(conv3x3(a, p[f"d{l}b.w"], p[f"d{l}b.b"])))
        cache[f"d{l}b"] = d
    r = head(d, p["head.w"], float(p["head.b"][0]))
    return r, cache


def unet_backward(p: Dict[str, np.ndarray], cache, dr: np.ndarray, store=None):
    """Gradients of ``sum(dr * r)`` wrt every parameter and the input.

    ``store`` as in ``unet_forward``, applied to every gradient tensor kept
    between layers (the gradient wrt each layer output and each concatenation,
    and the running sum of a skip connection's two contributions)."""
    keep = store or _same
    g: Dict[str, np.ndarray] = {}
    dd, g["head.w"], hb = head_backward(cache["d0b"], p["head.w"], dr)
    g["head.b"] = np.array([hb])
    d_out = {}          # gradient wrt each layer output (post-activation)
    d_out["d0b"] = keep(dd)
    for l in range(LEVELS - 1):
        d_out[f"e{l}b"] = np.zeros_like(cache[f"e{l}b"])

    def conv_back(name, x_key):
        pre = relu_backward(cache[name], d_out[name])
        dx, g[name + ".w"], g[name + ".b"] = conv3x3_backward(cache[x_key], p[name + ".w"], pre)
        return keep(dx)

    for l in range(LEVELS - 1):
        d_out[f"d{l}a"] = conv_back(f"d{l}b", f"d{l}a")
        dcat = conv_back(f"d{l}a", f"cat{l}")
        C = cache[f"e{l}b"].shape[-1]
        d_out[f"e{l}b"] += dcat[..., :C]
        below = f"d{l + 1}b" if l + 1 < LEVELS - 1 else f"e{LEVELS - 1}b"
        d_out[below] = keep(upsample2_backward(dcat[..., C:]))
    for l in range(LEVELS - 1, -1, -1):
        d_out[f"e{l}a"] = conv_back(f"e{l}b", f"e{l}a")
        x_key = f"in{l}"
        dx = conv_back(f"e{l}a", x_key)
        if l > 0:
            d_out[f"e{l - 1}b"] = keep(d_out[f"e{l - 1}b"] + avgpool2_backward(dx))
        else:
            g["input"] = dx
    return g


def masked_mse(r: np.ndarray, t: np.ndarray, mask: np.ndarray):
    """``L = 1/(2n) sum_mask (r - t)^2`` over a batch (mask ``[H][W]`` shared),
    and ``dL/dr``."""
    m = np.broadcast_to(np.asarray(mask, dtype=bool), r.shape)
    n = int(m.sum())
    e = np.where(m, r - t, 0.0)
    return 0.5 * float((e ** 2).sum()) / n, e / n


def adam_step(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step ``t >= 1``; returns ``(w, m, v)``."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64: the precision in which the network's weights and activations are
    stored (8 significant bits)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
