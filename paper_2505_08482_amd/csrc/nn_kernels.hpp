// nn_kernels.hpp — the learned fine-level start of the sound speed (a U-Net
// proposing the starting c of the next multigrid level, Sec. 3.1) on gfx950.
//
// Activations are channels-last bfloat16, [pixels][ld] with the channel slice
// at a pointer offset (concatenations are channel slices of one buffer, so no
// copy kernel exists).  bfloat16 values are stored as uint16_t: the upper half
// of a float32, rounded to nearest even.
//
// Dense contractions run on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation):
//  * k_conv3x3: implicit GEMM  Y[p][o] = sum_k A[p][k] Wt[o][k], k = (tap, ci),
//    A[p][(t,c)] = X[p + offset_t][c] (zero outside the image), operands
//    gathered straight from memory (any shape with cin % 8 == 0);
//    k_conv3x3_rows: the same GEMM for rows of 64-pixel multiples and
//    32-channel chunks, with the block's input rows (plus halo) and weights
//    staged in LDS and the next stage prefetched into registers.  Both are
//    the data gradient of a convolution when given the flipped weights
//    (k_flip) and the gradient of the layer above.
//  * k_wgrad: dW[o][(t,c)] = sum_p dY[p][o] X[p + offset_t][c] with the pixel
//    sum split over blocks (partials reduced in a fixed order, k_wgrad_reduce1/2).
// MFMA operand layout (16x16x32): lane l supplies row (l mod 16) of A and
// column (l mod 16) of B, each with 8 consecutive k; the accumulator holds
// D[4 (l / 16) + r][l mod 16], r = 0..3.  The k order inside a step only has
// to agree between A and B.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pat {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ u16x8 load8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// 3x3 convolution, zero padding, as implicit GEMM
// ---------------------------------------------------------------------------
struct ConvArgs {
  const uint16_t* x;     // [B*H*W][ldx] (channel slice of cin)
  const uint16_t* w;     // [cout][9][cin]
  const float* bias;     // [cout] or null
  uint16_t* y;           // [B*H*W][ldy] (channel slice of cout)
  const uint16_t* mask;  // [B*H*W][ldm] or null: zero where mask <= 0
  int B, H, W, cin, cout, ldx, ldy, ldm;
  int relu, accum;
};

// Block: 4 waves, BM along the pixels and 4 / BM along the output channels; a
// wave owns WM x WN MFMA tiles (16 pixels x 16 output channels each).  Block
// tile: 16 WM BM pixels x 16 WN (4 / BM) output channels.
template <int WM, int WN, int BM>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
  constexpr int BN = 4 / BM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % BM, wn = wave / BM;
  const int r = lane & 15, kg = lane >> 4;
  const int64_t P = (int64_t)a.B * a.H * a.W;
  const int64_t m0 = (int64_t)blockIdx.x * (16 * WM * BM) + wm * (16 * WM);
  const int n0 = blockIdx.y * (16 * WN * BN) + wn * (16 * WN);
  const int ktot = 9 * a.cin;

  int pb[WM], py[WM], px[WM];
  bool pv[WM];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    int64_t p = m0 + 16 * i + r;
    pv[i] = p < P;
    if (!pv[i]) p = 0;
    px[i] = (int)(p % a.W);
    const int64_t t = p / a.W;
    py[i] = (int)(t % a.H);
    pb[i] = (int)(t / a.H);
  }
  const uint16_t* wrow[WN];
  bool cv[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int co = n0 + 16 * j + r;
    cv[j] = co < a.cout;
    wrow[j] = a.w + (size_t)(cv[j] ? co : 0) * ktot;
  }
  f32x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  if (a.cin % 32 == 0) {
    // a 32-wide k step never crosses a tap: walk taps, then channel chunks
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      const uint16_t* src[WM];
      bool ok[WM];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int yy = py[i] + dy, xx = px[i] + dx;
        ok[i] = pv[i] && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        src[i] = a.x + ((int64_t)(pb[i] * a.H + (ok[i] ? yy : 0)) * a.W + (ok[i] ? xx : 0)) * a.ldx + 8 * kg;
      }
      const int kt = tap * a.cin + 8 * kg;
      for (int c0 = 0; c0 < a.cin; c0 += 32) {
        bf16x8 A[WM], Bv[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i) A[i] = as_bf16x8(ok[i] ? load8(src[i] + c0) : zero8);
#pragma unroll
        for (int j = 0; j < WN; ++j) Bv[j] = as_bf16x8(cv[j] ? load8(wrow[j] + kt + c0) : zero8);
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = mfma(A[i], Bv[j], acc[i][j]);
      }
    }
  } else {
    // cin a multiple of 8: each lane's 8 consecutive k stay inside one tap
    for (int kc = 0; kc < ktot; kc += 32) {
      const int k = kc + 8 * kg;
      const bool kv = k < ktot;
      const int tap = kv ? k / a.cin : 0;
      const int ci = k - tap * a.cin;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      bf16x8 A[WM], Bv[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int yy = py[i] + dy, xx = px[i] + dx;
        const bool ok = kv && pv[i] && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        A[i] = as_bf16x8(ok ? load8(a.x + ((int64_t)(pb[i] * a.H + yy) * a.W + xx) * a.ldx + ci) : zero8);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) Bv[j] = as_bf16x8(kv && cv[j] ? load8(wrow[j] + k) : zero8);
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = mfma(A[i], Bv[j], acc[i][j]);
    }
  }

  // epilogue: lane holds output channel n0 + 16 j + r of pixels m0 + 16 i + 4 kg + q
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int co = n0 + 16 * j + r;
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t p = m0 + 16 * i + 4 * kg + q;
        if (p >= P) continue;
        float v = acc[i][j][q] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        uint16_t* dst = a.y + p * a.ldy + co;
        if (a.accum) v += bf2f(*dst);
        if (a.mask && !(bf2f(a.mask[p * a.ldm + co]) > 0.f)) v = 0.f;
        *dst = f2bf(v);
      }
  }
}

// Row-tiled variant for cin % 32 == 0, W % 64 == 0 and H % BM == 0: a block
// covers BM image rows x 64 pixels (wave row wm = image row y0 + wm, its 4 MFMA
// pixel tiles = 64 consecutive pixels) x 16 WN (4 / BM) output channels.  Per
// 32-channel chunk the block stages its input rows with a one-pixel halo in LDS
// once; every tap then reads its operand from LDS, so the input is fetched
// once per chunk instead of once per tap.  The weights of each row of 3 taps
// are staged beside it, so both MFMA operands come from LDS.
constexpr int ROWS_HALO_W = 66;

template <int WN, int BM>
__global__ __launch_bounds__(256) void k_conv3x3_rows(ConvArgs a) {
  constexpr int BN = 4 / BM, HR = BM + 2, CT = 16 * WN * BN;
  __shared__ __attribute__((aligned(16))) uint16_t sX[HR][ROWS_HALO_W][32];
  __shared__ __attribute__((aligned(16))) uint16_t sW[3][CT][32];   // one row of 3 taps of the chunk
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % BM, wn = wave / BM;
  const int r = lane & 15, kg = lane >> 4;
  const int tiles_x = a.W / 64, tiles_y = a.H / BM;
  int bid = blockIdx.x;
  const int tx = bid % tiles_x;
  bid /= tiles_x;
  const int ty = bid % tiles_y;
  const int b = bid / tiles_y;
  const int x0 = tx * 64, y0 = ty * BM;
  const int cb0 = blockIdx.y * CT;
  const int nl = wn * (16 * WN);                  // the wave's first channel inside the block tile
  const int ktot = 9 * a.cin;
  f32x4 acc[4][WN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};

  // Staging through registers: the global loads of the next stage (the next
  // tap row's weights, or the next chunk's input rows) are issued right after
  // a barrier, so they are in flight while the current stage's MFMAs run.
  constexpr int XG = HR * ROWS_HALO_W * 4, WG = 3 * CT * 4;        // 16-byte groups per stage
  constexpr int NXG = (XG + 255) / 256, NWG = (WG + 255) / 256;    // per thread
  u16x8 rx[NXG], rw[NWG];
  auto load_x = [&](int c0) {
#pragma unroll
    for (int k = 0; k < NXG; ++k) {
      const int g = threadIdx.x + 256 * k;
      rx[k] = zero8;
      if (g < XG) {
        const int row = g / (ROWS_HALO_W * 4), rem = g - row * (ROWS_HALO_W * 4);
        const int px = rem >> 2, q = rem & 3;
        const int yy = y0 - 1 + row, xx = x0 - 1 + px;
        if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          rx[k] = load8(a.x + ((int64_t)(b * a.H + yy) * a.W + xx) * a.ldx + c0 + 8 * q);
      }
    }
  };
  auto store_x = [&]() {
#pragma unroll
    for (int k = 0; k < NXG; ++k) {
      const int g = threadIdx.x + 256 * k;
      if (g < XG) {
        const int row = g / (ROWS_HALO_W * 4), rem = g - row * (ROWS_HALO_W * 4);
        *reinterpret_cast<u16x8*>(&sX[row][rem >> 2][8 * (rem & 3)]) = rx[k];
      }
    }
  };
  auto load_w = [&](int c0, int ty3) {        // weights of taps 3 ty3 .. 3 ty3 + 2, this chunk
#pragma unroll
    for (int k = 0; k < NWG; ++k) {
      const int g = threadIdx.x + 256 * k;
      rw[k] = zero8;
      if (g < WG) {
        const int t3 = g / (CT * 4), rem = g - t3 * (CT * 4);
        const int co = cb0 + (rem >> 2), q = rem & 3;
        if (co < a.cout) rw[k] = load8(a.w + (size_t)co * ktot + (3 * ty3 + t3) * a.cin + c0 + 8 * q);
      }
    }
  };
  auto store_w = [&]() {
#pragma unroll
    for (int k = 0; k < NWG; ++k) {
      const int g = threadIdx.x + 256 * k;
      if (g < WG) {
        const int t3 = g / (CT * 4), rem = g - t3 * (CT * 4);
        *reinterpret_cast<u16x8*>(&sW[t3][rem >> 2][8 * (rem & 3)]) = rw[k];
      }
    }
  };

  load_x(0);
  load_w(0, 0);
  for (int c0 = 0; c0 < a.cin; c0 += 32) {
    store_x();
    for (int ty3 = 0; ty3 < 3; ++ty3) {
      store_w();
      __syncthreads();
      if (ty3 < 2) {
        load_w(c0, ty3 + 1);
      } else if (c0 + 32 < a.cin) {
        load_w(c0 + 32, 0);
        load_x(c0 + 32);
      }
#pragma unroll
      for (int tx3 = 0; tx3 < 3; ++tx3) {          // offsets (dy + 1, dx + 1) into the halo tile
        bf16x8 A[4], Bv[WN];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          A[i] = as_bf16x8(*reinterpret_cast<const u16x8*>(&sX[wm + ty3][16 * i + r + tx3][8 * kg]));
#pragma unroll
        for (int j = 0; j < WN; ++j)
          Bv[j] = as_bf16x8(*reinterpret_cast<const u16x8*>(&sW[tx3][nl + 16 * j + r][8 * kg]));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[i][j] = mfma(A[i], Bv[j], acc[i][j]);
      }
      __syncthreads();
    }
  }

  const int64_t prow = ((int64_t)b * a.H + y0 + wm) * a.W + x0;
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int co = cb0 + nl + 16 * j + r;
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t p = prow + 16 * i + 4 * kg + q;
        float v = acc[i][j][q] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        uint16_t* dst = a.y + p * a.ldy + co;
        if (a.accum) v += bf2f(*dst);
        if (a.mask && !(bf2f(a.mask[p * a.ldm + co]) > 0.f)) v = 0.f;
        *dst = f2bf(v);
      }
  }
}

// Weights of the transposed convolution: wt[ci][t][co] = w[co][8 - t][ci]
// (tap 8 - t is the opposite offset).
__global__ void k_flip(int cout, int cin, const uint16_t* __restrict__ w, uint16_t* __restrict__ wt) {
  const int64_t n = (int64_t)cout * 9 * cin;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(e % cout);
    const int t = (int)((e / cout) % 9);
    const int ci = (int)(e / ((int64_t)cout * 9));
    wt[e] = w[((int64_t)co * 9 + (8 - t)) * cin + ci];
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: block = CT output channels x NT (tap, ci) columns, pixel
// chunks of 64 staged (transposed, 8 x 8 tiles in registers) through LDS;
// grid.z splits the pixels.
// Tiles (CT x NT): 32 x 128 for layers of at most 32 channels (waves 1 x 4,
// 2 x 2 MFMA tiles each), 64 x 128 for 64 channels (waves 2 x 2, 2 x 4 tiles),
// 128 x 128 otherwise (waves 2 x 2, 4 x 4 tiles).
// ---------------------------------------------------------------------------
struct WgradArgs {
  const uint16_t* x;    // [P][ldx] layer input slice (cin)
  const uint16_t* dy;   // [P][ldy] gradient wrt the pre-activation (cout)
  float* part;          // [nsplit][cout][9 cin]
  float* partb;         // [nsplit][cout]
  int B, H, W, cin, cout, ldx, ldy;
  int64_t chunks_per_split;
};

constexpr int WG_CHUNK = 64;
constexpr int WG_PAD = WG_CHUNK + 8;   // LDS row length (elements): 144 B rows stay 16-B aligned

// Block tile CT output channels x NT columns, waves WCO x (4 / WCO); a wave owns
// (CT / WCO) x (NT / (4 / WCO)) of the output as MI x NJ MFMA tiles.
template <int CT, int NT>
struct WgradTile {
  static constexpr int WCO = CT >= 64 ? 2 : 1;   // waves along the output channels
  static constexpr int WNN = 4 / WCO;            // waves along the (tap, ci) columns
  static constexpr int TM = CT / WCO, TN = NT / WNN;
  static constexpr int MI = TM / 16, NJ = TN / 16;
  static_assert(CT + NT <= 256, "one staging tile per thread");
};

template <int CT, int NT>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  using Tl = WgradTile<CT, NT>;
  constexpr int WCO = Tl::WCO, TM = Tl::TM, TN = Tl::TN, MI = Tl::MI, NJ = Tl::NJ;
  __shared__ __attribute__((aligned(16))) uint16_t sA[CT][WG_PAD];   // [co][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t sB[NT][WG_PAD];   // [(tap, ci)][pixel]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WCO, wn = wave / WCO;
  const int r = lane & 15, kg = lane >> 4;
  const int ktot = 9 * a.cin;
  const int n0 = blockIdx.x * NT, co0 = blockIdx.y * CT;
  const int64_t P = (int64_t)a.B * a.H * a.W;
  const int64_t nchunks = (P + WG_CHUNK - 1) / WG_CHUNK;
  const int64_t c_begin = blockIdx.z * a.chunks_per_split;
  const int64_t c_end = c_begin + a.chunks_per_split < nchunks ? c_begin + a.chunks_per_split : nchunks;
  const bool bias_block = blockIdx.x == 0;
  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};

  f32x4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;

  for (int64_t c = c_begin; c < c_end; ++c) {
    const int64_t pbase = c * WG_CHUNK;
    // Staging in 8 x 8 tiles: a thread loads 8 consecutive pixels x 8 channels
    // (eight 16-byte loads), transposes them in registers and writes each
    // channel's 8 pixels as one 16-byte LDS segment.  dY tiles: tid < CT;
    // shifted-input tiles: CT <= tid < CT + NT.  Tile t: channel group t / 8,
    // pixel block t % 8 of the chunk.
    if (tid < CT + NT) {
      const bool is_dy = tid < CT;
      const int t = is_dy ? tid : tid - CT;
      const int grp = t >> 3, pb = t & 7;
      const int64_t p0 = pbase + 8 * pb;
      u16x8 v[8];
      if (is_dy) {
        const int co = co0 + 8 * grp;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[e] = (p0 + e < P && co < a.cout) ? load8(a.dy + (p0 + e) * a.ldy + co) : zero8;
      } else {
        const int n = n0 + 8 * grp;
        const bool nv = n < ktot && p0 < P;
        const int tap = nv ? n / a.cin : 0, ci = n - tap * a.cin;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        // decode the first pixel once, then step along the row with carries
        int xx = nv ? (int)(p0 % a.W) : 0;
        const int64_t t0 = nv ? p0 / a.W : 0;
        int yy = (int)(t0 % a.H), bb = (int)(t0 / a.H);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int ys = yy + dy, xs = xx + dx;
          const bool ok = nv && p0 + e < P && ys >= 0 && ys < a.H && xs >= 0 && xs < a.W;
          v[e] = ok ? load8(a.x + ((int64_t)(bb * a.H + ys) * a.W + xs) * a.ldx + ci) : zero8;
          if (++xx == a.W) {
            xx = 0;
            if (++yy == a.H) {
              yy = 0;
              ++bb;
            }
          }
        }
      }
      uint16_t(*dst)[WG_PAD] = is_dy ? sA : sB;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        u16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = v[e][ch];
        *reinterpret_cast<u16x8*>(&dst[8 * grp + ch][8 * pb]) = o;
      }
    }
    __syncthreads();
    if (bias_block && tid < CT)
#pragma unroll
      for (int q = 0; q < WG_CHUNK / 8; ++q) {
        const u16x8 v = *reinterpret_cast<const u16x8*>(&sA[tid][8 * q]);
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum += bf2f(v[e]);
      }
#pragma unroll
    for (int ks = 0; ks < WG_CHUNK / 32; ++ks) {
      bf16x8 A[MI], Bv[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        A[i] = as_bf16x8(*reinterpret_cast<const u16x8*>(&sA[TM * wm + 16 * i + r][32 * ks + 8 * kg]));
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        Bv[j] = as_bf16x8(*reinterpret_cast<const u16x8*>(&sB[TN * wn + 16 * j + r][32 * ks + 8 * kg]));
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = mfma(A[i], Bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* part = a.part + (int64_t)blockIdx.z * a.cout * ktot;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int n = n0 + TN * wn + 16 * j + r;
    if (n >= ktot) continue;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int co = co0 + TM * wm + 16 * i + 4 * kg + q;
        if (co < a.cout) part[(int64_t)co * ktot + n] = acc[i][j][q];
      }
  }
  if (bias_block && tid < CT && co0 + tid < a.cout) a.partb[(int64_t)blockIdx.z * a.cout + co0 + tid] = bsum;
}

// Weight gradient of layers with at most 32 output channels on rows of 64-pixel
// multiples (cin a multiple of CI = 16 or 32): block = 32 output channels x CI
// input channels x all 9 taps (9 CI columns).  A 64-pixel chunk lies in one image row;
// its three input rows with a one-pixel halo are staged once (3 x 66 x 16),
// and the 9 shifted copies are built from LDS as transposed 8 x 8 tiles, so the
// input is fetched once per chunk and row instead of once per tap.  The
// 2 x 9 CI / 16 MFMA tiles of the block are dealt round-robin to the 4 waves.
template <int CI>
__global__ __launch_bounds__(256) void k_wgrad_rows(WgradArgs a) {
  constexpr int WGR_CI = CI, WGR_COLS = 9 * CI, WGR_TILES = 2 * WGR_COLS / 16;
  constexpr int SLOTS = (WGR_TILES + 3) / 4, HG = CI / 8;
  __shared__ __attribute__((aligned(16))) uint16_t sA[32][WG_PAD];          // [co][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t sB[WGR_COLS][WG_PAD];    // [(tap, ci)][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t sXh[3][66][WGR_CI];      // input rows with halo
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int ktot = 9 * a.cin;
  const int ci0 = blockIdx.x * WGR_CI, co0 = blockIdx.y * 32;
  const int64_t nchunks = (int64_t)a.B * a.H * a.W / WG_CHUNK;
  const int64_t c_begin = blockIdx.z * a.chunks_per_split;
  const int64_t c_end = c_begin + a.chunks_per_split < nchunks ? c_begin + a.chunks_per_split : nchunks;
  const bool bias_block = blockIdx.x == 0;
  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};

  f32x4 acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;

  for (int64_t c = c_begin; c < c_end; ++c) {
    const int64_t p0 = c * WG_CHUNK;
    const int x0 = (int)(p0 % a.W);
    const int64_t t0 = p0 / a.W;
    const int y = (int)(t0 % a.H), b = (int)(t0 / a.H);
    // dY: 4 channel groups x 8 pixel blocks of 8 x 8, transposed in registers
    if (tid < 32) {
      const int grp = tid >> 3, pb = tid & 7;
      const int co = co0 + 8 * grp;
      u16x8 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = co < a.cout ? load8(a.dy + (p0 + 8 * pb + e) * a.ldy + co) : zero8;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        u16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = v[e][ch];
        *reinterpret_cast<u16x8*>(&sA[8 * grp + ch][8 * pb]) = o;
      }
    }
    // input rows y - 1 .. y + 1, pixels x0 - 1 .. x0 + 64, channels ci0 .. ci0 + CI - 1
    for (int g = tid; g < 3 * 66 * HG; g += 256) {
      const int row = g / (66 * HG), rem = g - row * (66 * HG);
      const int px = rem / HG, h = rem % HG;
      const int yy = y - 1 + row, xx = x0 - 1 + px;
      const bool ok = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
      *reinterpret_cast<u16x8*>(&sXh[row][px][8 * h]) =
          ok ? load8(a.x + ((int64_t)(b * a.H + yy) * a.W + xx) * a.ldx + ci0 + 8 * h) : zero8;
    }
    __syncthreads();
    // the 9 shifted copies, transposed: tile (tap, channel group h, pixel block pb)
    for (int g = tid; g < WGR_COLS; g += 256) {
      const int tap = g / CI, rem = g % CI;
      const int h = rem >> 3, pb = rem & 7;
      const int dy = tap / 3, dx = tap % 3;
      u16x8 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = *reinterpret_cast<const u16x8*>(&sXh[dy][8 * pb + e + dx][8 * h]);
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        u16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = v[e][ch];
        *reinterpret_cast<u16x8*>(&sB[CI * tap + 8 * h + ch][8 * pb]) = o;
      }
    }
    __syncthreads();
    if (bias_block && tid < 32)
#pragma unroll
      for (int q = 0; q < WG_CHUNK / 8; ++q) {
        const u16x8 v = *reinterpret_cast<const u16x8*>(&sA[tid][8 * q]);
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum += bf2f(v[e]);
      }
#pragma unroll
    for (int ks = 0; ks < WG_CHUNK / 32; ++ks) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int tt = wave + 4 * s;
        if (tt < WGR_TILES) {
          const int i = tt & 1, j = tt >> 1;
          const bf16x8 A = as_bf16x8(*reinterpret_cast<const u16x8*>(&sA[16 * i + r][32 * ks + 8 * kg]));
          const bf16x8 Bv = as_bf16x8(*reinterpret_cast<const u16x8*>(&sB[16 * j + r][32 * ks + 8 * kg]));
          acc[s] = mfma(A, Bv, acc[s]);
        }
      }
    }
    __syncthreads();
  }
  float* part = a.part + (int64_t)blockIdx.z * a.cout * ktot;
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int tt = wave + 4 * s;
    if (tt >= WGR_TILES) continue;
    const int i = tt & 1, j = tt >> 1;
    const int nl = 16 * j + r;                    // local column: tap nl / CI, channel nl % CI
    const int n = (nl / CI) * a.cin + ci0 + (nl % CI);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = co0 + 16 * i + 4 * kg + q;
      if (co < a.cout) part[(int64_t)co * ktot + n] = acc[s][q];
    }
  }
  if (bias_block && tid < 32 && co0 + tid < a.cout) a.partb[(int64_t)blockIdx.z * a.cout + co0 + tid] = bsum;
}

// Two-stage fixed-order reduction of the pixel-split partials.  Stage 1:
// group g of WG_GROUP consecutive splits, part2[g][e] = sum over the group of
// part[s][e] (e < nw) or partb[s][e - nw] (the bias columns).  Stage 2:
// dw[e] / db[e - nw] = sum over the groups.
constexpr int WG_GROUP = 32;

__global__ void k_wgrad_reduce1(int nsplit, int64_t nw, int cout, const float* __restrict__ part,
                                const float* __restrict__ partb, float* __restrict__ part2) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nw + cout) return;
  const int s0 = blockIdx.y * WG_GROUP;
  const int s1 = s0 + WG_GROUP < nsplit ? s0 + WG_GROUP : nsplit;
  float s = 0.f;
  if (e < nw) {
    for (int z = s0; z < s1; ++z) s += part[(int64_t)z * nw + e];
  } else {
    for (int z = s0; z < s1; ++z) s += partb[(int64_t)z * cout + (e - nw)];
  }
  part2[(int64_t)blockIdx.y * (nw + cout) + e] = s;
}

__global__ void k_wgrad_reduce2(int ngroups, int64_t nw, int cout, const float* __restrict__ part2,
                                float* __restrict__ dw, float* __restrict__ db) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nw + cout;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int g = 0; g < ngroups; ++g) s += part2[(int64_t)g * (nw + cout) + e];
    if (e < nw) dw[e] = s;
    else if (db) db[e - nw] = s;
  }
}

// ---------------------------------------------------------------------------
// 2x2 average pooling, nearest upsampling and their adjoints (8 channels per
// thread; C and the leading dimensions are multiples of 8)
// ---------------------------------------------------------------------------
// y[b][i][j] = mean of x[b][2i..2i+1][2j..2j+1]; x is [B][H][W], y [B][H/2][W/2]
__global__ void k_avgpool2(int B, int H, int W, int C, const uint16_t* __restrict__ x, int ldx,
                           uint16_t* __restrict__ y, int ldy) {
  const int Ho = H / 2, Wo = W / 2, G = C / 8;
  const int64_t n = (int64_t)B * Ho * Wo * G;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % G);
    const int64_t q = e / G;
    const int j = (int)(q % Wo);
    const int i = (int)((q / Wo) % Ho);
    const int b = (int)(q / ((int64_t)Wo * Ho));
    const int64_t p00 = ((int64_t)b * H + 2 * i) * W + 2 * j;
    const u16x8 v0 = load8(x + p00 * ldx + 8 * g), v1 = load8(x + (p00 + 1) * ldx + 8 * g);
    const u16x8 v2 = load8(x + (p00 + W) * ldx + 8 * g), v3 = load8(x + (p00 + W + 1) * ldx + 8 * g);
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = f2bf(0.25f * ((bf2f(v0[k]) + bf2f(v1[k])) + (bf2f(v2[k]) + bf2f(v3[k]))));
    *reinterpret_cast<u16x8*>(y + q * ldy + 8 * g) = o;
  }
}

// dx[b][i][j] (fine, [B][H][W]) = (acc ? dx : 0) + dy[b][i/2][j/2] / 4, zero where mask <= 0
__global__ void k_avgpool2_bwd(int B, int H, int W, int C, const uint16_t* __restrict__ dy, int ldy,
                               uint16_t* __restrict__ dx, int ldx, const uint16_t* __restrict__ mask, int ldm,
                               int accum) {
  const int G = C / 8;
  const int64_t n = (int64_t)B * H * W * G;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % G);
    const int64_t p = e / G;
    const int j = (int)(p % W);
    const int i = (int)((p / W) % H);
    const int b = (int)(p / ((int64_t)W * H));
    const int64_t pc = ((int64_t)b * (H / 2) + i / 2) * (W / 2) + j / 2;
    const u16x8 d = load8(dy + pc * ldy + 8 * g);
    uint16_t* dst = dx + p * ldx + 8 * g;
    const u16x8 old = accum ? load8(dst) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    const u16x8 m = mask ? load8(mask + p * ldm + 8 * g) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float v = 0.25f * bf2f(d[k]) + (accum ? bf2f(old[k]) : 0.f);
      if (mask && !(bf2f(m[k]) > 0.f)) v = 0.f;
      o[k] = f2bf(v);
    }
    *reinterpret_cast<u16x8*>(dst) = o;
  }
}

// y (fine [B][H][W]) = x[b][i/2][j/2]
__global__ void k_upsample2(int B, int H, int W, int C, const uint16_t* __restrict__ x, int ldx,
                            uint16_t* __restrict__ y, int ldy) {
  const int G = C / 8;
  const int64_t n = (int64_t)B * H * W * G;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % G);
    const int64_t p = e / G;
    const int j = (int)(p % W);
    const int i = (int)((p / W) % H);
    const int b = (int)(p / ((int64_t)W * H));
    const int64_t pc = ((int64_t)b * (H / 2) + i / 2) * (W / 2) + j / 2;
    *reinterpret_cast<u16x8*>(y + p * ldy + 8 * g) = load8(x + pc * ldx + 8 * g);
  }
}

// dx (coarse [B][H/2][W/2]) = sum of the four fine dy, zero where mask <= 0
__global__ void k_upsample2_bwd(int B, int H, int W, int C, const uint16_t* __restrict__ dy, int ldy,
                                uint16_t* __restrict__ dx, int ldx, const uint16_t* __restrict__ mask, int ldm) {
  const int Ho = H / 2, Wo = W / 2, G = C / 8;
  const int64_t n = (int64_t)B * Ho * Wo * G;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % G);
    const int64_t q = e / G;
    const int j = (int)(q % Wo);
    const int i = (int)((q / Wo) % Ho);
    const int b = (int)(q / ((int64_t)Wo * Ho));
    const int64_t p00 = ((int64_t)b * H + 2 * i) * W + 2 * j;
    const u16x8 v0 = load8(dy + p00 * ldy + 8 * g), v1 = load8(dy + (p00 + 1) * ldy + 8 * g);
    const u16x8 v2 = load8(dy + (p00 + W) * ldy + 8 * g), v3 = load8(dy + (p00 + W + 1) * ldy + 8 * g);
    const u16x8 m = mask ? load8(mask + q * ldm + 8 * g) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float v = (bf2f(v0[k]) + bf2f(v1[k])) + (bf2f(v2[k]) + bf2f(v3[k]));
      if (mask && !(bf2f(m[k]) > 0.f)) v = 0.f;
      o[k] = f2bf(v);
    }
    *reinterpret_cast<u16x8*>(dx + q * ldx + 8 * g) = o;
  }
}

// ---------------------------------------------------------------------------
// 1x1 output head, its gradients, the masked squared loss
// ---------------------------------------------------------------------------
// r[p] = b + sum_c w[c] x[p][c]
__global__ void k_head(int64_t P, int C, const uint16_t* __restrict__ x, int ldx, const uint16_t* __restrict__ w,
                       const float* __restrict__ b, float* __restrict__ r) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    float s = b[0];
    for (int g = 0; g < C / 8; ++g) {
      const u16x8 v = load8(x + p * ldx + 8 * g), wv = load8(w + 8 * g);
#pragma unroll
      for (int k = 0; k < 8; ++k) s = fmaf(bf2f(wv[k]), bf2f(v[k]), s);
    }
    r[p] = s;
  }
}

// dx[p][c] = [x > 0] w[c] dr[p]  (the gradient wrt the pre-activation of the layer below)
__global__ void k_head_bwd_dx(int64_t P, int C, const uint16_t* __restrict__ x, int ldx,
                              const uint16_t* __restrict__ w, const float* __restrict__ dr, uint16_t* __restrict__ dx,
                              int lddx) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const float d = dr[p];
    for (int g = 0; g < C / 8; ++g) {
      const u16x8 v = load8(x + p * ldx + 8 * g), wv = load8(w + 8 * g);
      u16x8 o;
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = f2bf(bf2f(v[k]) > 0.f ? bf2f(wv[k]) * d : 0.f);
      *reinterpret_cast<u16x8*>(dx + p * lddx + 8 * g) = o;
    }
  }
}

// part[blk][c] = sum over the block's pixels of dr[p] x[p][c]; part[blk][C] = sum dr.
// 256 threads, C divides 256: thread t owns channel t mod C and pixel lane t / C.
constexpr int HEAD_BLOCKS = 2048;
__global__ __launch_bounds__(256) void k_head_wgrad(int64_t P, int C, const uint16_t* __restrict__ x, int ldx,
                                                    const float* __restrict__ dr, float* __restrict__ part) {
  __shared__ float sh[256];
  __shared__ float shb[256];
  const int t = threadIdx.x, c = t % C, lanes = 256 / C, pl = t / C;
  const int64_t per = (P + gridDim.x - 1) / gridDim.x;
  const int64_t p0 = blockIdx.x * per, p1 = p0 + per < P ? p0 + per : P;
  float s = 0.f, sb = 0.f;
  for (int64_t p = p0 + pl; p < p1; p += lanes) {
    const float d = dr[p];
    s = fmaf(d, bf2f(x[p * ldx + c]), s);
    if (c == 0) sb += d;
  }
  sh[t] = s;
  shb[t] = sb;
  __syncthreads();
  if (t < C) {
    float tot = 0.f;
    for (int l = 0; l < lanes; ++l) tot += sh[l * C + t];
    part[(int64_t)blockIdx.x * (C + 1) + t] = tot;
  }
  if (t == 0) {
    float tb = 0.f;
    for (int l = 0; l < lanes; ++l) tb += shb[l * C];
    part[(int64_t)blockIdx.x * (C + 1) + C] = tb;
  }
}

// Block c (0..C) sums column c of the partials: thread t adds blocks t, t + 256, ...
// in order, then a fixed tree over the 256 threads.
__global__ __launch_bounds__(256) void k_head_wgrad_final(int nblk, int C, const float* __restrict__ part,
                                                          float* __restrict__ dw, float* __restrict__ db) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[(int64_t)b * (C + 1) + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (c < C) dw[c] = sh[0];
    else db[0] = sh[0];
  }
}

// Masked squared loss over B images sharing one mask [HW]:
// partials of sum m (r - t)^2 and of the mask count, then L and dr.
constexpr int MSE_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_mse_partial(int64_t n, int64_t hw, const float* __restrict__ r,
                                                     const float* __restrict__ t, const uint8_t* __restrict__ mask,
                                                     double* __restrict__ part) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (mask[i % hw]) {
      const double e = (double)r[i] - (double)t[i];
      a += e * e;
      c += 1.0;
    }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

// out[0] = L = sse / (2 count), out[1] = count
__global__ void k_mse_final(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double a = 0.0, c = 0.0;
  for (int b = 0; b < nblk; ++b) {
    a += part[2 * b];
    c += part[2 * b + 1];
  }
  out[0] = c > 0.0 ? 0.5 * a / c : 0.0;
  out[1] = c;
}

__global__ void k_mse_grad(int64_t n, int64_t hw, const float* __restrict__ r, const float* __restrict__ t,
                           const uint8_t* __restrict__ mask, const double* __restrict__ stats,
                           float* __restrict__ dr) {
  const float inv = stats[1] > 0.0 ? (float)(1.0 / stats[1]) : 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dr[i] = mask[i % hw] ? (r[i] - t[i]) * inv : 0.f;
}

// ---------------------------------------------------------------------------
// Adam (bias-corrected), FP32 master weights, bf16 copy for the kernels
// ---------------------------------------------------------------------------
__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ wb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
  }
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = f2bf(a[i]);
}

// ---------------------------------------------------------------------------
// Network input: channel 0 = (c - shift) / scale, channel 1 = (sum_k g_k) /
// max |sum_k g_k|, channels 2..7 = 0; optionally under one of the 8
// symmetries of the square (bit 2: transpose, bit 0: flip rows, bit 1: flip
// columns, applied to the output pixel to find its source pixel).
// ---------------------------------------------------------------------------
constexpr int PACK_BLOCKS = 256;

__device__ __forceinline__ int64_t sym_src(int sym, int H, int W, int i, int j) {
  if (sym & 1) i = H - 1 - i;
  if (sym & 2) j = W - 1 - j;
  if (sym & 4) {
    const int t = i;
    i = j;
    j = t;
  }
  return (int64_t)i * W + j;
}

__global__ __launch_bounds__(256) void k_gsum_absmax(int64_t hw, int K, const float* __restrict__ g,
                                                     float* __restrict__ part) {
  __shared__ float sh[256];
  float mx = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hw; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < K; ++k) s += g[(int64_t)k * hw + i];
    mx = fmaxf(mx, fabsf(s));
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_pack_input(int H, int W, int K, const float* __restrict__ c_up, const float* __restrict__ g_up,
                             const float* __restrict__ c_true, int sym, float shift, float inv_scale,
                             const float* __restrict__ gpart, int npart, uint16_t* __restrict__ x,
                             float* __restrict__ base, float* __restrict__ target) {
  __shared__ float gscale;
  if (threadIdx.x == 0) {
    float mx = 0.f;
    for (int b = 0; b < npart; ++b) mx = fmaxf(mx, gpart[b]);
    gscale = mx > 0.f ? 1.f / mx : 0.f;
  }
  __syncthreads();
  const int64_t hw = (int64_t)H * W;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < hw; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p / W), j = (int)(p % W);
    const int64_t s = sym_src(sym, H, W, i, j);
    float gs = 0.f;
    for (int k = 0; k < K; ++k) gs += g_up[(int64_t)k * hw + s];
    const float c = c_up[s];
    u16x8 o = {0, 0, 0, 0, 0, 0, 0, 0};
    o[0] = f2bf((c - shift) * inv_scale);
    o[1] = f2bf(gs * gscale);
    *reinterpret_cast<u16x8*>(x + p * 8) = o;
    base[p] = c;
    if (target) target[p] = (c_true[s] - c) * inv_scale;
  }
}

}  // namespace nn
}  // namespace pat
