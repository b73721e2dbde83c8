"""Thin binding of the learned-start layers in ``include/pat_nn.h``.

Argument marshalling only: each function checks shapes, passes device pointers
and enqueues the library call on torch's current stream.  Activations are
channels-last ``torch.bfloat16`` tensors ``[B][H][W][ld]`` (a channel slice is
a view ``t[..., c0:c0 + C]``; its leading dimension is ``t.shape[-1]``);
weights ``[cout][9][cin]`` bfloat16; gradients of weights float32.
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import pat

EXPORTS = (
    "pat_nn_conv3x3", "pat_nn_conv3x3_flip", "pat_nn_wgrad_scratch_bytes", "pat_nn_conv3x3_wgrad",
    "pat_nn_avgpool2", "pat_nn_avgpool2_backward", "pat_nn_upsample2", "pat_nn_upsample2_backward",
    "pat_nn_head", "pat_nn_head_scratch_bytes", "pat_nn_head_backward", "pat_nn_mse_scratch_bytes",
    "pat_nn_masked_mse", "pat_nn_adam", "pat_nn_to_bf16", "pat_nn_pack_scratch_bytes", "pat_nn_pack_input",
)

_ready = False


def lib() -> ctypes.CDLL:
    global _ready
    L = pat.lib()
    if _ready:
        return L
    vp, i32, i64, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    L.pat_nn_conv3x3.argtypes = [i32, i32, i32, vp, i32, i32, vp, vp, vp, i32, i32, i32, i32, vp, i32, vp]
    L.pat_nn_conv3x3_flip.argtypes = [i32, i32, vp, vp, vp]
    L.pat_nn_wgrad_scratch_bytes.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.pat_nn_conv3x3_wgrad.argtypes = [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, vp, vp, sz, vp]
    L.pat_nn_avgpool2.argtypes = [i32, i32, i32, i32, vp, i32, vp, i32, vp]
    L.pat_nn_avgpool2_backward.argtypes = [i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp]
    L.pat_nn_upsample2.argtypes = [i32, i32, i32, i32, vp, i32, vp, i32, vp]
    L.pat_nn_upsample2_backward.argtypes = [i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, vp]
    L.pat_nn_head.argtypes = [i64, i32, vp, i32, vp, vp, vp, vp]
    L.pat_nn_head_scratch_bytes.argtypes = [i32]
    L.pat_nn_head_scratch_bytes.restype = sz
    L.pat_nn_head_backward.argtypes = [i64, i32, vp, i32, vp, vp, vp, i32, vp, vp, vp, sz, vp]
    L.pat_nn_mse_scratch_bytes.argtypes = []
    L.pat_nn_mse_scratch_bytes.restype = sz
    L.pat_nn_masked_mse.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.pat_nn_adam.argtypes = [i64, vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
    L.pat_nn_to_bf16.argtypes = [i64, vp, vp, vp]
    L.pat_nn_pack_scratch_bytes.argtypes = []
    L.pat_nn_pack_scratch_bytes.restype = sz
    L.pat_nn_pack_input.argtypes = [i32, i32, i32, vp, vp, vp, i32, f32, f32, vp, vp, vp, vp, sz, vp]
    for name in EXPORTS:
        if not name.endswith("_scratch_bytes") or name == "pat_nn_wgrad_scratch_bytes":
            getattr(L, name).restype = ctypes.c_int
    _ready = True
    return L


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _act(t, name: str):
    """(pointer, B, H, W, C, ld) of a channels-last bf16 activation (or slice)."""
    import torch
    if t.dtype != torch.bfloat16 or not t.is_cuda or t.dim() != 4:
        raise ValueError(f"{name}: expected a 4-D bfloat16 GPU tensor [B][H][W][C]")
    B, H, W, C = t.shape
    ld = t.stride(2)
    if t.stride(3) != 1 or t.stride(1) != W * ld or t.stride(0) != H * W * ld:
        raise ValueError(f"{name}: expected a channel slice of a contiguous [B][H][W][ld] buffer")
    return t.data_ptr(), B, H, W, C, ld


def _dev(t, dtype, name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def conv3x3(x, w, bias, y, relu: bool = False, accumulate: bool = False, mask=None) -> None:
    """``y = conv3x3(x, w) (+bias) (relu) (+y) (masked)``, see ``pat_nn_conv3x3``."""
    import torch
    xp, B, H, W, cin, ldx = _act(x, "x")
    yp, B2, H2, W2, cout, ldy = _act(y, "y")
    if (B2, H2, W2) != (B, H, W):
        raise ValueError("x and y differ in B, H, W")
    wp = _dev(w, torch.bfloat16, "w", cout * 9 * cin)
    bp = _dev(bias, torch.float32, "bias", cout)
    mp, ldm = None, 0
    if mask is not None:
        mp, B3, H3, W3, C3, ldm = _act(mask, "mask")
        if (B3, H3, W3, C3) != (B, H, W, cout):
            raise ValueError("mask must match y")
    pat._check(lib().pat_nn_conv3x3(B, H, W, xp, ldx, cin, wp, bp, yp, ldy, cout, int(relu), int(accumulate),
                                    mp, ldm, _stream()), "pat_nn_conv3x3")


def conv3x3_flip(w, wt) -> None:
    import torch
    cout, nine, cin = w.shape
    if nine != 9 or tuple(wt.shape) != (cin, 9, cout):
        raise ValueError("w [cout][9][cin] -> wt [cin][9][cout]")
    pat._check(lib().pat_nn_conv3x3_flip(cout, cin, _dev(w, torch.bfloat16, "w"), _dev(wt, torch.bfloat16, "wt"),
                                         _stream()), "pat_nn_conv3x3_flip")


def wgrad_scratch_bytes(B: int, H: int, W: int, cin: int, cout: int) -> int:
    out = ctypes.c_size_t(0)
    pat._check(lib().pat_nn_wgrad_scratch_bytes(B, H, W, cin, cout, ctypes.byref(out)), "pat_nn_wgrad_scratch_bytes")
    return int(out.value)


def conv3x3_wgrad(x, dy, dw, db, scratch) -> None:
    import torch
    xp, B, H, W, cin, ldx = _act(x, "x")
    dp, B2, H2, W2, cout, ldy = _act(dy, "dy")
    if (B2, H2, W2) != (B, H, W):
        raise ValueError("x and dy differ in B, H, W")
    pat._check(lib().pat_nn_conv3x3_wgrad(B, H, W, xp, ldx, cin, dp, ldy, cout,
                                          _dev(dw, torch.float32, "dw", cout * 9 * cin),
                                          _dev(db, torch.float32, "db", cout),
                                          _dev(scratch, torch.uint8, "scratch"), scratch.numel(), _stream()),
               "pat_nn_conv3x3_wgrad")


def avgpool2(x, y) -> None:
    xp, B, H, W, C, ldx = _act(x, "x")
    yp, B2, H2, W2, C2, ldy = _act(y, "y")
    if (B2, 2 * H2, 2 * W2, C2) != (B, H, W, C):
        raise ValueError("y must be [B][H/2][W/2][C]")
    pat._check(lib().pat_nn_avgpool2(B, H, W, C, xp, ldx, yp, ldy, _stream()), "pat_nn_avgpool2")


def avgpool2_backward(dy, dx, mask=None, accumulate: bool = False) -> None:
    dyp, B, Hc, Wc, C, ldy = _act(dy, "dy")
    dxp, B2, H, W, C2, ldx = _act(dx, "dx")
    if (B2, H, W, C2) != (B, 2 * Hc, 2 * Wc, C):
        raise ValueError("dx must be [B][2H][2W][C]")
    mp, ldm = None, 0
    if mask is not None:
        mp, *shape, ldm = _act(mask, "mask")
        if tuple(shape) != (B, H, W, C):
            raise ValueError("mask must match dx")
    pat._check(lib().pat_nn_avgpool2_backward(B, H, W, C, dyp, ldy, dxp, ldx, mp, ldm, int(accumulate), _stream()),
               "pat_nn_avgpool2_backward")


def upsample2(x, y) -> None:
    xp, B, Hc, Wc, C, ldx = _act(x, "x")
    yp, B2, H, W, C2, ldy = _act(y, "y")
    if (B2, H, W, C2) != (B, 2 * Hc, 2 * Wc, C):
        raise ValueError("y must be [B][2H][2W][C]")
    pat._check(lib().pat_nn_upsample2(B, H, W, C, xp, ldx, yp, ldy, _stream()), "pat_nn_upsample2")


def upsample2_backward(dy, dx, mask=None) -> None:
    dyp, B, H, W, C, ldy = _act(dy, "dy")
    dxp, B2, Hc, Wc, C2, ldx = _act(dx, "dx")
    if (B2, 2 * Hc, 2 * Wc, C2) != (B, H, W, C):
        raise ValueError("dx must be [B][H/2][W/2][C]")
    mp, ldm = None, 0
    if mask is not None:
        mp, *shape, ldm = _act(mask, "mask")
        if tuple(shape) != (B, Hc, Wc, C):
            raise ValueError("mask must match dx")
    pat._check(lib().pat_nn_upsample2_backward(B, H, W, C, dyp, ldy, dxp, ldx, mp, ldm, _stream()),
               "pat_nn_upsample2_backward")


def head(x, w, b, r) -> None:
    import torch
    xp, B, H, W, C, ldx = _act(x, "x")
    P = B * H * W
    pat._check(lib().pat_nn_head(P, C, xp, ldx, _dev(w, torch.bfloat16, "w", C), _dev(b, torch.float32, "b", 1),
                                 _dev(r, torch.float32, "r", P), _stream()), "pat_nn_head")


def head_scratch_bytes(C: int) -> int:
    return int(lib().pat_nn_head_scratch_bytes(C))


def head_backward(x, w, dr, dx, dw, db, scratch) -> None:
    import torch
    xp, B, H, W, C, ldx = _act(x, "x")
    dxp, *shape, lddx = _act(dx, "dx")
    if tuple(shape) != (B, H, W, C):
        raise ValueError("dx must match x")
    P = B * H * W
    pat._check(lib().pat_nn_head_backward(P, C, xp, ldx, _dev(w, torch.bfloat16, "w", C),
                                          _dev(dr, torch.float32, "dr", P), dxp, lddx,
                                          _dev(dw, torch.float32, "dw", C), _dev(db, torch.float32, "db", 1),
                                          _dev(scratch, torch.uint8, "scratch"), scratch.numel(), _stream()),
               "pat_nn_head_backward")


def mse_scratch_bytes() -> int:
    return int(lib().pat_nn_mse_scratch_bytes())


def masked_mse(r, t, mask, dr, out, scratch) -> None:
    """``r, t, dr [B][H][W]`` float32, ``mask [H][W]`` uint8, ``out [2]`` float64."""
    import torch
    B = r.shape[0]
    hw = r.numel() // B
    pat._check(lib().pat_nn_masked_mse(B, hw, _dev(r, torch.float32, "r"), _dev(t, torch.float32, "t", r.numel()),
                                       _dev(mask, torch.uint8, "mask", hw), _dev(dr, torch.float32, "dr", r.numel()),
                                       _dev(out, torch.float64, "out", 2), _dev(scratch, torch.uint8, "scratch"),
                                       scratch.numel(), _stream()), "pat_nn_masked_mse")


def adam(w, g, m, v, w_bf16, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
    import torch
    n = w.numel()
    pat._check(lib().pat_nn_adam(n, _dev(w, torch.float32, "w"), _dev(g, torch.float32, "g", n),
                                 _dev(m, torch.float32, "m", n), _dev(v, torch.float32, "v", n),
                                 _dev(w_bf16, torch.bfloat16, "w_bf16", n), int(step), lr, b1, b2, eps, _stream()),
               "pat_nn_adam")


def to_bf16(a, b) -> None:
    import torch
    pat._check(lib().pat_nn_to_bf16(a.numel(), _dev(a, torch.float32, "a"), _dev(b, torch.bfloat16, "b", a.numel()),
                                    _stream()), "pat_nn_to_bf16")


def pack_scratch_bytes() -> int:
    return int(lib().pat_nn_pack_scratch_bytes())


def pack_input(c_up, g_up, c_true, sym: int, shift: float, scale: float, x, base, target, scratch) -> None:
    """One image: ``c_up [H][W]``, ``g_up [K][H][W]``, ``c_true [H][W]`` or None
    (float32) -> ``x [1][H][W][8]`` bf16, ``base``, ``target`` ``[H][W]`` float32."""
    import torch
    H, W = c_up.shape
    K = g_up.numel() // (H * W)
    pat._check(lib().pat_nn_pack_input(H, W, K, _dev(c_up, torch.float32, "c_up"),
                                       _dev(g_up, torch.float32, "g_up", K * H * W),
                                       _dev(c_true, torch.float32, "c_true", H * W), int(sym), shift, scale,
                                       _dev(x, torch.bfloat16, "x", H * W * 8), _dev(base, torch.float32, "base", H * W),
                                       _dev(target, torch.float32, "target", H * W),
                                       _dev(scratch, torch.uint8, "scratch"), scratch.numel(), _stream()),
               "pat_nn_pack_input")
