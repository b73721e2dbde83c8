// nn_api.hip — C ABI of the learned fine-level start (include/pat_nn.h):
// argument checks, launch shapes and scratch layouts of nn_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/pat.h"
#include "../../include/pat_nn.h"
#include "nn_kernels.hpp"

using namespace pat::nn;

namespace {

int nn_blocks(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 16384) b = 16384;
  return (int)std::max<int64_t>(b, 1);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int launched() { return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// pixel-split of the weight gradient: enough blocks to fill the chip, whole chunks per split
struct WgradSplit {
  int rows;                // input channels per block of the halo-staged kernel (0: not used)
  int ct, ntiles, cotiles;
  int64_t nchunks, per, nsplit, ngroups;
};

// Layers of at most 32 output and 16 or 32 input channels on rows of 64-pixel
// multiples use the halo-staged kernel (32 output x 16 input channels x 9 taps
// per block; wider inputs re-stage dY per channel group and lose to the tiles); otherwise the output-channel tile is 32, 64 or 128 (at most
// 32, 64, or more channels) with 128 (tap, ci) columns per block.  Enough pixel
// splits to fill the chip, at least 16 chunks of 64 pixels per split.
WgradSplit wgrad_split(int64_t P, int W, int cin, int cout) {
  WgradSplit s;
  s.rows = cout <= 32 && W % 64 == 0 && cin % 16 == 0 && cin <= 32 ? 16 : 0;
  s.ct = cout <= 32 ? 32 : cout <= 64 ? 64 : 128;
  s.ntiles = s.rows ? cin / s.rows : (9 * cin + 127) / 128;
  s.cotiles = (cout + s.ct - 1) / s.ct;
  s.nchunks = (P + WG_CHUNK - 1) / WG_CHUNK;
  const int64_t tiles = (int64_t)s.ntiles * s.cotiles;
  int64_t want = (2048 + tiles - 1) / tiles;
  want = std::min<int64_t>(want, (s.nchunks + 15) / 16);
  want = std::max<int64_t>(1, std::min<int64_t>(want, s.nchunks));
  s.per = (s.nchunks + want - 1) / want;
  s.nsplit = (s.nchunks + s.per - 1) / s.per;
  s.ngroups = (s.nsplit + WG_GROUP - 1) / WG_GROUP;
  return s;
}

// scratch: partials [nsplit][cout * 9 cin], bias partials [nsplit][cout], group sums [ngroups][cout * 9 cin + cout]
size_t wgrad_bytes(const WgradSplit& s, int cin, int cout) {
  const size_t row = (size_t)cout * 9 * cin + cout;
  return ((size_t)s.nsplit + (size_t)s.ngroups) * row * sizeof(float);
}

}  // namespace

extern "C" {

int pat_nn_conv3x3(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t ldx, int32_t cin, const uint16_t* w,
                   const float* bias, uint16_t* y, int32_t ldy, int32_t cout, int32_t relu, int32_t accumulate,
                   const uint16_t* mask, int32_t ldm, void* stream) {
  if (!x || !w || !y || B < 1 || H < 1 || W < 1 || cin < 8 || cin % 8 || cout < 1 || ldx < cin || ldx % 8 ||
      ldy < cout)
    return PAT_EINVAL;
  if (!aligned16(x) || !aligned16(w)) return PAT_EINVAL;
  if (mask && ldm < cout) return PAT_EINVAL;
  const int64_t P = (int64_t)B * H * W;
  if (P > (int64_t)1 << 31 || (int64_t)B * H > INT32_MAX) return PAT_EINVAL;
  ConvArgs a{x, w, bias, y, mask, B, H, W, cin, cout, ldx, ldy, ldm, relu ? 1 : 0, accumulate ? 1 : 0};
  hipStream_t st = as_stream(stream);
  // block tiles (pixels x output channels): 256 x 32, 256 x 64 or 128 x 128; a wave
  // holds up to 4 x 4 accumulator tiles, so each operand load feeds up to 4 MFMAs.
  // Rows of 64-pixel multiples with 32-channel multiples stage their input in LDS.
  const int bm = cout <= 32 || (cout % 128 != 0 && cout % 64 == 0) ? 4 : 2;
  if (cin % 32 == 0 && W % 64 == 0 && H % bm == 0) {
    const unsigned nblk = (unsigned)((int64_t)B * (H / bm) * (W / 64));
    if (cout <= 32) {
      hipLaunchKernelGGL((k_conv3x3_rows<2, 4>), dim3(nblk, (unsigned)((cout + 31) / 32)), dim3(256), 0, st, a);
    } else if (bm == 4) {
      hipLaunchKernelGGL((k_conv3x3_rows<4, 4>), dim3(nblk, (unsigned)(cout / 64)), dim3(256), 0, st, a);
    } else {
      hipLaunchKernelGGL((k_conv3x3_rows<4, 2>), dim3(nblk, (unsigned)((cout + 127) / 128)), dim3(256), 0, st, a);
    }
    return launched();
  }
  if (cout <= 32) {
    dim3 grid((unsigned)((P + 255) / 256), (unsigned)((cout + 31) / 32));
    hipLaunchKernelGGL((k_conv3x3<4, 2, 4>), grid, dim3(256), 0, st, a);
  } else if (cout % 128 != 0 && cout % 64 == 0) {
    dim3 grid((unsigned)((P + 255) / 256), (unsigned)(cout / 64));
    hipLaunchKernelGGL((k_conv3x3<4, 4, 4>), grid, dim3(256), 0, st, a);
  } else {
    dim3 grid((unsigned)((P + 127) / 128), (unsigned)((cout + 127) / 128));
    hipLaunchKernelGGL((k_conv3x3<4, 4, 2>), grid, dim3(256), 0, st, a);
  }
  return launched();
}

int pat_nn_conv3x3_flip(int32_t cout, int32_t cin, const uint16_t* w, uint16_t* wt, void* stream) {
  if (!w || !wt || cout < 1 || cin < 1 || w == wt) return PAT_EINVAL;
  const int64_t n = (int64_t)cout * 9 * cin;
  hipLaunchKernelGGL(k_flip, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), cout, cin, w, wt);
  return launched();
}

int pat_nn_wgrad_scratch_bytes(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout, size_t* bytes) {
  if (!bytes || B < 1 || H < 1 || W < 1 || cin < 8 || cout < 8) return PAT_EINVAL;
  const WgradSplit s = wgrad_split((int64_t)B * H * W, W, cin, cout);
  *bytes = wgrad_bytes(s, cin, cout);
  return PAT_OK;
}

int pat_nn_conv3x3_wgrad(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t ldx, int32_t cin,
                         const uint16_t* dy, int32_t ldy, int32_t cout, float* dw, float* db, void* scratch,
                         size_t scratch_bytes, void* stream) {
  if (!x || !dy || !dw || !scratch || B < 1 || H < 1 || W < 1 || cin < 8 || cin % 8 || cout < 8 || cout % 8 ||
      ldx < cin || ldx % 8 || ldy < cout || ldy % 8)
    return PAT_EINVAL;
  if (!aligned16(x) || !aligned16(dy)) return PAT_EINVAL;
  const int64_t P = (int64_t)B * H * W;
  if (P > (int64_t)1 << 31) return PAT_EINVAL;
  const WgradSplit s = wgrad_split(P, W, cin, cout);
  if (scratch_bytes < wgrad_bytes(s, cin, cout)) return PAT_EWORKSPACE;
  float* part = static_cast<float*>(scratch);
  float* partb = part + (size_t)s.nsplit * cout * 9 * cin;
  WgradArgs a{x, dy, part, partb, B, H, W, cin, cout, ldx, ldy, s.per};
  hipStream_t st = as_stream(stream);
  const dim3 grid((unsigned)s.ntiles, (unsigned)s.cotiles, (unsigned)s.nsplit);
  if (s.rows == 16)
    hipLaunchKernelGGL((k_wgrad_rows<16>), grid, dim3(256), 0, st, a);
  else if (s.ct == 32)
    hipLaunchKernelGGL((k_wgrad<32, 128>), grid, dim3(256), 0, st, a);
  else if (s.ct == 64)
    hipLaunchKernelGGL((k_wgrad<64, 128>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_wgrad<128, 128>), grid, dim3(256), 0, st, a);
  const int64_t nw = (int64_t)cout * 9 * cin;
  float* part2 = partb + (size_t)s.nsplit * cout;
  hipLaunchKernelGGL(k_wgrad_reduce1, dim3((unsigned)((nw + cout + 255) / 256), (unsigned)s.ngroups), dim3(256), 0,
                     st, (int)s.nsplit, nw, cout, part, partb, part2);
  hipLaunchKernelGGL(k_wgrad_reduce2, dim3(nn_blocks(nw + cout)), dim3(256), 0, st, (int)s.ngroups, nw, cout, part2,
                     dw, db);
  return launched();
}

int pat_nn_avgpool2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* x, int32_t ldx, uint16_t* y,
                    int32_t ldy, void* stream) {
  if (!x || !y || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 8 || C % 8 || ldx < C || ldx % 8 || ldy < C ||
      ldy % 8 || !aligned16(x) || !aligned16(y))
    return PAT_EINVAL;
  const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (C / 8);
  hipLaunchKernelGGL(k_avgpool2, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), B, H, W, C, x, ldx, y, ldy);
  return launched();
}

int pat_nn_avgpool2_backward(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* dy, int32_t ldy,
                             uint16_t* dx, int32_t ldx, const uint16_t* mask, int32_t ldm, int32_t accumulate,
                             void* stream) {
  if (!dy || !dx || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 8 || C % 8 || ldx < C || ldx % 8 || ldy < C ||
      ldy % 8 || !aligned16(dy) || !aligned16(dx))
    return PAT_EINVAL;
  if (mask && (ldm < C || ldm % 8 || !aligned16(mask))) return PAT_EINVAL;
  const int64_t n = (int64_t)B * H * W * (C / 8);
  hipLaunchKernelGGL(k_avgpool2_bwd, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), B, H, W, C, dy, ldy, dx,
                     ldx, mask, ldm, accumulate ? 1 : 0);
  return launched();
}

int pat_nn_upsample2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* x, int32_t ldx, uint16_t* y,
                     int32_t ldy, void* stream) {
  if (!x || !y || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 8 || C % 8 || ldx < C || ldx % 8 || ldy < C ||
      ldy % 8 || !aligned16(x) || !aligned16(y))
    return PAT_EINVAL;
  const int64_t n = (int64_t)B * H * W * (C / 8);
  hipLaunchKernelGGL(k_upsample2, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), B, H, W, C, x, ldx, y, ldy);
  return launched();
}

int pat_nn_upsample2_backward(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* dy, int32_t ldy,
                              uint16_t* dx, int32_t ldx, const uint16_t* mask, int32_t ldm, void* stream) {
  if (!dy || !dx || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 8 || C % 8 || ldx < C || ldx % 8 || ldy < C ||
      ldy % 8 || !aligned16(dy) || !aligned16(dx))
    return PAT_EINVAL;
  if (mask && (ldm < C || ldm % 8 || !aligned16(mask))) return PAT_EINVAL;
  const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (C / 8);
  hipLaunchKernelGGL(k_upsample2_bwd, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), B, H, W, C, dy, ldy, dx,
                     ldx, mask, ldm);
  return launched();
}

int pat_nn_head(int64_t P, int32_t C, const uint16_t* x, int32_t ldx, const uint16_t* w, const float* b, float* r,
                void* stream) {
  if (!x || !w || !b || !r || P < 1 || C < 8 || C % 8 || ldx < C || ldx % 8 || !aligned16(x) || !aligned16(w))
    return PAT_EINVAL;
  hipLaunchKernelGGL(k_head, dim3(nn_blocks(P)), dim3(256), 0, as_stream(stream), P, C, x, ldx, w, b, r);
  return launched();
}

size_t pat_nn_head_scratch_bytes(int32_t C) { return C < 1 ? 0 : (size_t)HEAD_BLOCKS * (C + 1) * sizeof(float); }

int pat_nn_head_backward(int64_t P, int32_t C, const uint16_t* x, int32_t ldx, const uint16_t* w, const float* dr,
                         uint16_t* dx, int32_t lddx, float* dw, float* db, void* scratch, size_t scratch_bytes,
                         void* stream) {
  if (!x || !w || !dr || !dx || !dw || !db || !scratch || P < 1 || C < 8 || C % 8 || 256 % C || ldx < C ||
      ldx % 8 || lddx < C || lddx % 8 || !aligned16(x) || !aligned16(w) || !aligned16(dx))
    return PAT_EINVAL;
  if (scratch_bytes < pat_nn_head_scratch_bytes(C)) return PAT_EWORKSPACE;
  hipStream_t st = as_stream(stream);
  float* part = static_cast<float*>(scratch);
  hipLaunchKernelGGL(k_head_bwd_dx, dim3(nn_blocks(P)), dim3(256), 0, st, P, C, x, ldx, w, dr, dx, lddx);
  hipLaunchKernelGGL(k_head_wgrad, dim3(HEAD_BLOCKS), dim3(256), 0, st, P, C, x, ldx, dr, part);
  hipLaunchKernelGGL(k_head_wgrad_final, dim3(C + 1), dim3(256), 0, st, HEAD_BLOCKS, C, part, dw, db);
  return launched();
}

size_t pat_nn_mse_scratch_bytes(void) { return (size_t)MSE_BLOCKS * 2 * sizeof(double); }

int pat_nn_masked_mse(int32_t B, int64_t hw, const float* r, const float* t, const uint8_t* mask, float* dr,
                      double* out, void* scratch, size_t scratch_bytes, void* stream) {
  if (!r || !t || !mask || !dr || !out || !scratch || B < 1 || hw < 1) return PAT_EINVAL;
  if (scratch_bytes < pat_nn_mse_scratch_bytes()) return PAT_EWORKSPACE;
  hipStream_t st = as_stream(stream);
  const int64_t n = (int64_t)B * hw;
  double* part = static_cast<double*>(scratch);
  hipLaunchKernelGGL(k_mse_partial, dim3(MSE_BLOCKS), dim3(256), 0, st, n, hw, r, t, mask, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, MSE_BLOCKS, part, out);
  hipLaunchKernelGGL(k_mse_grad, dim3(nn_blocks(n)), dim3(256), 0, st, n, hw, r, t, mask, out, dr);
  return launched();
}

int pat_nn_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, int32_t step, float lr,
                float b1, float b2, float eps, void* stream) {
  if (!w || !g || !m || !v || n < 1 || step < 1 || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f))
    return PAT_EINVAL;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
  hipLaunchKernelGGL(k_adam, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), n, w, g, m, v, w_bf16, lr, b1, b2,
                     eps, c1, c2);
  return launched();
}

int pat_nn_to_bf16(int64_t n, const float* a, uint16_t* b, void* stream) {
  if (!a || !b || n < 1) return PAT_EINVAL;
  hipLaunchKernelGGL(k_to_bf16, dim3(nn_blocks(n)), dim3(256), 0, as_stream(stream), n, a, b);
  return launched();
}

size_t pat_nn_pack_scratch_bytes(void) { return (size_t)PACK_BLOCKS * sizeof(float); }

int pat_nn_pack_input(int32_t H, int32_t W, int32_t K, const float* c_up, const float* g_up, const float* c_true,
                      int32_t sym, float shift, float scale, uint16_t* x, float* base, float* target, void* scratch,
                      size_t scratch_bytes, void* stream) {
  if (!c_up || !g_up || !x || !base || !scratch || H < 1 || W < 1 || K < 1 || sym < 0 || sym > 7 ||
      !(scale > 0.f) || !aligned16(x))
    return PAT_EINVAL;
  if ((sym & 4) && H != W) return PAT_EINVAL;
  if (target && !c_true) return PAT_EINVAL;
  if (scratch_bytes < pat_nn_pack_scratch_bytes()) return PAT_EWORKSPACE;
  hipStream_t st = as_stream(stream);
  const int64_t hw = (int64_t)H * W;
  float* part = static_cast<float*>(scratch);
  hipLaunchKernelGGL(k_gsum_absmax, dim3(PACK_BLOCKS), dim3(256), 0, st, hw, K, g_up, part);
  hipLaunchKernelGGL(k_pack_input, dim3(nn_blocks(hw)), dim3(256), 0, st, H, W, K, c_up, g_up, c_true, sym, shift,
                     1.f / scale, part, PACK_BLOCKS, x, base, target);
  return launched();
}

}  // extern "C"
