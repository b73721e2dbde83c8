// fast_kernels.hpp — register-resident passes for power-of-two grids (32..512).
//
// Same arithmetic as wave_kernels.hpp (the k-space scheme of Sec. 2.1 and its
// exact discrete adjoint), organised for gfx950:
//  * every thread owns the elements q + T*m (m < 8) of one transform, so the
//    first Stockham stage reads straight from HBM, the last stage leaves the
//    result where the fused physics and the next transform's first stage want
//    it, and only the inner stages exchange through LDS;
//  * twiddles live in registers, loaded once per kernel from the float64-exact
//    table;
//  * half spectra are folded: the real Nyquist bin of a row is stored in the
//    imaginary part of its (real) DC bin, so a row spectrum has exactly nx/2
//    complex entries and the column pass has nx/2 columns.  The column holding
//    DC + i * Nyquist is two real sequences along y; it is split with the usual
//    two-for-one identity, each half multiplied by its own wavenumber, and
//    recombined before the inverse column transform.
//  * row passes run one 64-thread block per (T threads x 2 rows) group set;
//    column passes load 8..64 adjacent columns per block so that every load
//    instruction touches contiguous 64-256 byte row segments.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"
#include "wave_kernels.hpp"

namespace pat {
namespace fast {

template <int N> struct Cfg;
// T threads per transform (8 elements each); TC adjacent columns per column
// block (at least one wave, at least 4 columns = 32-byte row segments; narrow
// tiles give several blocks per CU).
template <> struct Cfg<512> { static constexpr int T = 64; using L = RList<8, 8, 8>; static constexpr int TC = 4; };
template <> struct Cfg<256> { static constexpr int T = 32; using L = RList<8, 8, 4>; static constexpr int TC = 4; };
template <> struct Cfg<128> { static constexpr int T = 16; using L = RList<8, 4, 4>; static constexpr int TC = 4; };
template <> struct Cfg<64>  { static constexpr int T = 8;  using L = RList<8, 8>;    static constexpr int TC = 8; };
template <> struct Cfg<32>  { static constexpr int T = 4;  using L = RList<8, 4>;    static constexpr int TC = 16; };

// Element at a 32-bit byte offset from a (block-uniform) base: lets the
// compiler address global memory as scalar base + 32-bit lane offset.
template <class T>
__device__ __forceinline__ T* at_byte(T* base, unsigned byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ const T* at_byte(const T* base, unsigned byte_off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// LDS position of element i: one pad slot per 8 keeps the radix-8 exchanges
// (stride-8 writes, stride-1 reads) free of bank conflicts within a transform.
__device__ __forceinline__ int phys(int i) { return i + (i >> 3); }
// Pitch of one transform.  Row passes: one transform per lane group.  Column
// passes interleave TC columns across the lanes of a wave; a 16-lane group then
// holds TC columns x 16/TC rows, spread over all 32 banks by a pitch of
// 4 (mod 16) complex for TC = 4, 2 (mod 16) for TC = 8, odd for TC = 16.
template <int N> struct Lds { static constexpr int P = N + N / 8 + 2; };
template <int N, int TC> struct LdsCol {
  static constexpr int base = N + N / 8;
  static constexpr int want = TC == 4 ? 4 : (TC == 8 ? 2 : 1);
  static constexpr int P = TC >= 16 ? (base | 1) : base + ((16 + want - base % 16) % 16);
};

// Row transforms of length 512 (one 64-lane wave per transform) place element
// i at i ^ swz_key(i / 16) instead of the padded i + i/8: a permutation inside
// each run of 16 elements under which the stage-1 writes (stride 8), the
// stage-2 writes (two runs of 8, 64 apart) and the stride-1 reads of a 16-lane
// group each touch 16 distinct bank pairs (the padding costs a two-way
// conflict in every 16-lane group of every read).
__device__ __forceinline__ int swz_key(int b) { return (b & 7) | ((b & 4) << 1); }

// Orders one wave's shared-memory writes before its own later reads (a wave
// executes its shared-memory operations in order; the fences keep the compiler
// from moving them across), for transforms whose exchanges stay inside a wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One register-resident Stockham stage on NV transforms at once (shared barriers;
// WAVE: the transform's lanes are one wave, which orders its own exchanges).
template <int N, int T, int R, int NS, int DIR, bool LAST, int NV, bool SWZ = false, bool WAVE = false>
__device__ __forceinline__ void rstage(float2 (*v)[8], const float2* w, float2* const* lds, int q) {
  constexpr int B = 8 / R;
  float2 y[NV][B][R];
#pragma unroll
  for (int t = 0; t < NV; ++t)
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) y[t][b][r] = v[t][b + r * B];
  if (NS > 1) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 tw = w[b * (R - 1) + r - 1];
        if (DIR > 0) tw.y = -tw.y;
#pragma unroll
        for (int t = 0; t < NV; ++t) y[t][b][r] = cmul(y[t][b][r], tw);
      }
  }
#pragma unroll
  for (int t = 0; t < NV; ++t)
#pragma unroll
    for (int b = 0; b < B; ++b) Dft<R, DIR>::run(y[t][b]);
  if (LAST) {
#pragma unroll
    for (int t = 0; t < NV; ++t)
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][b + r * B] = y[t][b][r];
    return;
  }
  // Padded positions as one lane-dependent base plus compile-time offsets
  // (immediate offsets of the shared-memory instructions, no address register
  // per element): phys(base + r NS) = phys(base) + r NS 9/8 when NS is a
  // multiple of 8, and phys(8 j + r) = phys(8 j) + r for r < 8; likewise
  // phys(q + T m) = phys(q) + T m 9/8 when T is a multiple of 8.
  static_assert(NS % 8 == 0 || (NS == 1 && R == 8), "padded stage offsets");
  static_assert(!SWZ || LAST || (T == 64 && R == 8 && (NS == 1 || NS == 8)), "swizzled stages: 512-point rows");
  constexpr int WSTEP = NS % 8 == 0 ? NS + NS / 8 : 1;
  if (WAVE) wave_sync(); else __syncthreads();
  if (SWZ) {
    // stage 1: 8 q + r -> ((8 q) ^ (key & 8)) + (r ^ (key & 7)), key of run q/2;
    // stage 2: base + 8 r (base = 64 (q/8) + q%8) -> (base + 8 r) ^ (12 h + r/2), h = bit 3 of q
    const int key1 = swz_key(q >> 1), wb1 = (8 * q) ^ (key1 & 8), k7 = key1 & 7;
    const int base2 = 64 * (q >> 3) + (q & 7), h12 = 12 * ((q >> 3) & 1);
#pragma unroll
    for (int t = 0; t < NV; ++t)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int pos = NS == 1 ? wb1 + (r ^ k7) : (base2 + 8 * r) ^ (h12 + (r >> 1));
        lds[t][pos] = y[t][0][r];
      }
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = q + T * b;
      const int pb = phys((j / NS) * NS * R + (j % NS));
#pragma unroll
      for (int t = 0; t < NV; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r) lds[t][pb + r * WSTEP] = y[t][b][r];
    }
  }
  if (WAVE) wave_sync(); else __syncthreads();
  if (SWZ) {
    // q + 64 m -> 64 m + (q ^ (q/16 + 12 (m & 1)))
    const int r0 = q ^ (q >> 4), r1 = q ^ ((q >> 4) + 12);
#pragma unroll
    for (int t = 0; t < NV; ++t)
#pragma unroll
      for (int m = 0; m < 8; ++m) v[t][m] = lds[t][((m & 1) ? r1 : r0) + 64 * m];
    return;
  }
  const int pq = phys(q);
#pragma unroll
  for (int t = 0; t < NV; ++t)
#pragma unroll
    for (int m = 0; m < 8; ++m) v[t][m] = lds[t][T % 8 == 0 ? pq + (T + T / 8) * m : phys(q + T * m)];
}

template <int N, typename L> struct RegFft;

template <int N, int R1, int R2, int R3> struct RegFft<N, RList<R1, R2, R3>> {
  static constexpr int T = Cfg<N>::T, NS2 = R1, NS3 = R1 * R2;
  float2 w2[(8 / R2) * (R2 - 1)];
  float2 w3[(8 / R3) * (R3 - 1)];
  __device__ __forceinline__ void init(const float2* __restrict__ tw, int q) {
#pragma unroll
    for (int b = 0; b < 8 / R2; ++b)
#pragma unroll
      for (int r = 1; r < R2; ++r) w2[b * (R2 - 1) + r - 1] =
            *at_byte(tw, (unsigned)((r * ((q + T * b) % NS2)) * (N / (NS2 * R2))) * 8u);
#pragma unroll
    for (int b = 0; b < 8 / R3; ++b)
#pragma unroll
      for (int r = 1; r < R3; ++r) w3[b * (R3 - 1) + r - 1] =
            *at_byte(tw, (unsigned)((r * ((q + T * b) % NS3)) * (N / (NS3 * R3))) * 8u);
  }
  // SWZ: swizzled shared-memory positions (512-point rows, see swz_key);
  // WAVE: wave-level ordering of the exchanges (every lane of a transform in one wave)
  template <int DIR, int NV, bool SWZ = false, bool WAVE = false>
  __device__ __forceinline__ void run(float2 (*v)[8], float2* const* lds, int q) const {
    rstage<N, T, R1, 1, DIR, false, NV, SWZ, WAVE>(v, nullptr, lds, q);
    rstage<N, T, R2, NS2, DIR, false, NV, SWZ, WAVE>(v, w2, lds, q);
    rstage<N, T, R3, NS3, DIR, true, NV, SWZ, WAVE>(v, w3, lds, q);
  }
};

template <int N, int R1, int R2> struct RegFft<N, RList<R1, R2>> {
  static constexpr int T = Cfg<N>::T, NS2 = R1;
  float2 w2[(8 / R2) * (R2 - 1)];
  __device__ __forceinline__ void init(const float2* __restrict__ tw, int q) {
#pragma unroll
    for (int b = 0; b < 8 / R2; ++b)
#pragma unroll
      for (int r = 1; r < R2; ++r) w2[b * (R2 - 1) + r - 1] =
            *at_byte(tw, (unsigned)((r * ((q + T * b) % NS2)) * (N / (NS2 * R2))) * 8u);
  }
  template <int DIR, int NV, bool SWZ = false, bool WAVE = false>
  __device__ __forceinline__ void run(float2 (*v)[8], float2* const* lds, int q) const {
    static_assert(!SWZ, "swizzled stages: 512-point rows only");
    rstage<N, T, R1, 1, DIR, false, NV, false, WAVE>(v, nullptr, lds, q);
    rstage<N, T, R2, NS2, DIR, true, NV, false, WAVE>(v, w2, lds, q);
  }
};

template <int N> using Fft = RegFft<N, typename Cfg<N>::L>;

// ---------------------------------------------------------------------------
// Folded half spectra along a row of length N (h = N/2 entries)
// ---------------------------------------------------------------------------
// z[k] = a[k] + i b[k] for the two real rows whose folded spectra are A, B, at
// the owned bin k = q + T*M (N = 8T).  Bins M < 4 are stored directly; bins
// M >= 4 are mirrored (k > N/2, conjugate of bin N - k); the only special bins
// (k = 0 and k = N/2, both in lane q = 0) are chosen by select, not by branch.
template <int N, int M>
__device__ __forceinline__ float2 pack_folded(const float2* __restrict__ A, const float2* __restrict__ B, int q) {
  constexpr int T = N / 8;
  const unsigned k = q + T * M;
  if constexpr (M < 4) {
    const float2 a = A[k], b = B[k];
    const float2 gen = make_float2(a.x - b.y, a.y + b.x);
    if constexpr (M == 0) return q == 0 ? make_float2(a.x, b.x) : gen;   // DC: real parts
    return gen;
  } else {
    const unsigned idx = (M == 4 && q == 0) ? 0u : N - k;
    const float2 a = A[idx], b = B[idx];
    const float2 gen = make_float2(a.x + b.y, b.x - a.y);                 // conj(a) + i conj(b)
    if constexpr (M == 4) return q == 0 ? make_float2(a.y, b.y) : gen;   // Nyquist, folded into bin 0
    return gen;
  }
}

template <int N, int M = 0>
__device__ __forceinline__ void pack_row(float2 (&v)[8], const float2* __restrict__ A, const float2* __restrict__ B,
                                         int q) {
  v[M] = pack_folded<N, M>(A, B, q);
  if constexpr (M + 1 < 8) pack_row<N, M + 1>(v, A, B, q);
}

// Split the transform of a + i b (held in owner layout, element q + T m in v[m])
// into the folded spectra of a and b and store them (rows rowA, rowB).
template <int N>
__device__ __forceinline__ void unpack_store(const float2 (&v)[8], int q, int lane_base, float2* __restrict__ rowA,
                                             float2* __restrict__ rowB) {
  constexpr int T = Cfg<N>::T;
  const int src = lane_base + ((T - q) & (T - 1));
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    // partner bin N - k: lane T - q, register 7 - m (lane 0: its own register 8 - m)
    const float px = __shfl(v[7 - m].x, src);
    const float py = __shfl(v[7 - m].y, src);
    const float2 part = q == 0 ? v[(8 - m) & 7] : make_float2(px, py);
    const unsigned k = q + T * m;
    const float2 P = v[m], Q = make_float2(part.x, -part.y);   // Z[k], conj Z[N-k]
    float2 A = make_float2(0.5f * (P.x + Q.x), 0.5f * (P.y + Q.y));
    float2 B = make_float2(0.5f * (P.y - Q.y), -0.5f * (P.x - Q.x));
    if (m == 0) {
      // k = 0 (lane 0): DC parts, with the Nyquist bin (q = 0, m = 4) folded in
      const float2 Zn = v[4];
      A = q == 0 ? make_float2(P.x, Zn.x) : A;
      B = q == 0 ? make_float2(P.y, Zn.y) : B;
    }
    rowA[k] = A;
    rowB[k] = B;
  }
}

// ===========================================================================
// Row passes: 64-thread blocks, G = 64/T groups of T threads, 2 rows per group
// ===========================================================================
template <int N> struct RowF {
  static constexpr int T = Cfg<N>::T;
  static constexpr int G = 64 / T;
  static constexpr int ROWS = 2 * G;
};

// Row passes run one wave per block (64 threads: RowF<N>::G transforms of
// two rows each), so their exchanges need wave-level ordering only.
#define PAT_ROW_PROLOGUE(N)                                                    \
  using RC = RowF<N>;                                                          \
  constexpr int T = RC::T;                                                     \
  const int K = tb.K, ny = tb.ny, nhf = N / 2;                                 \
  const int k = bid % K, ybase = (bid / K) * RC::ROWS;                         \
  const int tid = threadIdx.x, q = tid % T;                                    \
  const int grp = RC::G == 1 ? 0 : tid / T, lane_base = grp * T; /* uniform at G = 1 */ \
  const int y0 = ybase + 2 * grp, y1 = y0 + 1;                                 \
  (void)nhf;                                                                   \
  Fft<N> fft;                                                                  \
  fft.init(tb.tw_x, q);

// n = 0: rho = p0/(2c^2), history, sensors, spectra of p0 (rows y0, y1 share one FFT)
template <int N>
__device__ __forceinline__ void k_fwd_init_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                                const float* __restrict__ p0, float* __restrict__ rx,
                                                float* __restrict__ ry, float* __restrict__ hist0,
                                                float* __restrict__ dpart, float2* __restrict__ SA) {
  PAT_ROW_PROLOGUE(N)
  __shared__ float2 X[RC::G][Lds<N>::P];
  __shared__ float P[RC::ROWS][N];
  float2 v[1][8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const unsigned x = q + T * m;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int y = y0 + h;
      if (y < ny) {
        const size_t i = ((size_t)k * ny + y) * N + x;
        const float val = p0[i];
        const float cc = c[(size_t)y * N + x];
        const float rr = val * (0.5f / (cc * cc));
        rx[i] = rr;
        ry[i] = rr;
        if (hist0) hist0[i] = val;
        (h == 0 ? a : b) = val;
      }
    }
    P[2 * grp][x] = a;
    P[2 * grp + 1][x] = b;
    v[0][m] = make_float2(a, b);
  }
  __syncthreads();
  if (dpart) gather_rows<N, 64>(tb, &P[0][0], ybase, RC::ROWS, dpart + (size_t)k * tb.nt * 2 * tb.m, tid);
  float2* L[1] = {X[grp]};
  fft.template run<-1, 1, N == 512>(v, L, q);
  float2* ra = SA + ((size_t)k * ny + min(y0, ny - 1)) * nhf;
  float2* rb = SA + ((size_t)k * ny + min(y1, ny - 1)) * nhf;
  if (y1 < ny) unpack_store<N>(v[0], q, lane_base, ra, rb);
}

template <int N>
__global__ __launch_bounds__(64) void k_fwd_init(Tables tb, const float* __restrict__ c, const float* __restrict__ p0,
                                                 float* __restrict__ rx, float* __restrict__ ry,
                                                 float* __restrict__ hist0, float* __restrict__ dpart,
                                                 float2* __restrict__ SA) {
  fast::k_fwd_init_body<N>(blockIdx.x, tb, c, p0, rx, ry, hist0, dpart, SA);
}

// velocity update (step 0: u^{-1/2} = G/2), spectra of (u_x + i u_y)
template <int N>
__device__ __forceinline__ void k_fwd_u_body(const int bid, const Tables& tb, float* __restrict__ ux,
                                             float* __restrict__ uy, float2* __restrict__ SA, float2* __restrict__ SB,
                                             const StepCtl* __restrict__ ctl) {
  PAT_ROW_PROLOGUE(N)
  const int first = ctl->fwd_n == 0;
  __shared__ float2 X[RC::G][2][Lds<N>::P];
  float2 v[2][8];
  float ox[2][8], oy[2][8];
  const bool ok = y1 < ny;
  // row pointers (block-uniform at one group per block) + unsigned lane offsets
  float* uxr[2];
  float* uyr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const size_t f = ((size_t)k * ny + y) * N;
    uxr[h] = ux + f;
    uyr[h] = uy + f;
    pack_row<N>(v[h], SA + ((size_t)k * ny + y) * nhf, SB + ((size_t)k * ny + y) * nhf, q);
    // loaded at every step (step 0 ignores them): a load under the step test
    // would wait for the step counter before it could issue
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      ox[h][m] = uxr[h][(unsigned)(q + T * m)];
      oy[h][m] = uyr[h][(unsigned)(q + T * m)];
    }
  }
  // PML factors (prefetched before the transforms)
  float pax[8], pay[2];
#pragma unroll
  for (int m = 0; m < 8; ++m) pax[m] = tb.asx[(unsigned)(q + T * m)];
  pay[0] = tb.asy[ok ? y0 : 0];
  pay[1] = tb.asy[ok ? y1 : 0];
  float2* L[2] = {X[grp][0], X[grp][1]};
  fft.template run<+1, 2, N == 512, true>(v, L, q);
  // step 0 starts from u^{-1/2} = G/2 (a uniform branch, not a per-element select)
  auto update = [&](auto first_c) {
    constexpr bool F0 = decltype(first_c)::value;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float ays = pay[h];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const float2 g = v[h][m];
        const float axs = pax[m];
        const float uxo = F0 ? 0.5f * g.x : ox[h][m];
        const float uyo = F0 ? 0.5f * g.y : oy[h][m];
        v[h][m] = make_float2(axs * (axs * uxo - g.x), ays * (ays * uyo - g.y));
      }
    }
  };
  if (first)
    update(std::true_type{});
  else
    update(std::false_type{});
  if (ok) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        uxr[h][(unsigned)(q + T * m)] = v[h][m].x;
        uyr[h][(unsigned)(q + T * m)] = v[h][m].y;
      }
  }
  fft.template run<-1, 2, N == 512, true>(v, L, q);
  if (ok) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t r = ((size_t)k * ny + y0 + h) * nhf;
      unpack_store<N>(v[h], q, lane_base, SA + r, SB + r);
    }
  }
}

template <int N>
__global__ __launch_bounds__(64) void k_fwd_u(Tables tb, float* __restrict__ ux, float* __restrict__ uy,
                                              float2* __restrict__ SA, float2* __restrict__ SB,
                                              const StepCtl* __restrict__ ctl) {
  fast::k_fwd_u_body<N>(blockIdx.x, tb, ux, uy, SA, SB, ctl);
}

// density / pressure update, history, sensors at n+1, spectra of p (rows y0, y1 share one FFT)
template <int N>
__device__ __forceinline__ void k_fwd_rho_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                               float* __restrict__ rx, float* __restrict__ ry,
                                               float* __restrict__ hist_base, float* __restrict__ dpart,
                                               float2* __restrict__ SA, const float2* __restrict__ SB,
                                               const StepCtl* __restrict__ ctl) {
  PAT_ROW_PROLOGUE(N)
  const int n = ctl->fwd_n;
  float* hist = hist_base ? hist_base + (size_t)(n + 1 - ctl->hist_first) * tb.K * ny * N : nullptr;
  float* dpart_n = dpart ? dpart + (size_t)(n + 1) * 2 * tb.m : nullptr;
  __shared__ float2 X[RC::G][2][Lds<N>::P];
  __shared__ float P[RC::ROWS][N];
  float2 v[2][8];
  float orx[2][8], ory[2][8], cc[2][8];
  const bool ok = y1 < ny;
  // row pointers (block-uniform at one group per block) + unsigned lane offsets
  float* rxr[2];
  float* ryr[2];
  float* hr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const size_t f = ((size_t)k * ny + y) * N;
    rxr[h] = rx + f;
    ryr[h] = ry + f;
    hr[h] = hist ? hist + f : nullptr;
    const float* cr = c + (size_t)y * N;
    pack_row<N>(v[h], SA + ((size_t)k * ny + y) * nhf, SB + ((size_t)k * ny + y) * nhf, q);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const unsigned x = q + T * m;
      orx[h][m] = rxr[h][x];
      ory[h][m] = ryr[h][x];
      cc[h][m] = cr[x];
    }
  }
  float pax[8], pay[2];
#pragma unroll
  for (int m = 0; m < 8; ++m) pax[m] = tb.ax[(unsigned)(q + T * m)];
  pay[0] = tb.ay[ok ? y0 : 0];
  pay[1] = tb.ay[ok ? y1 : 0];
  // sensor taps of this block's rows (one entry per thread, prefetched)
  const int g0 = tb.g_row_start[ybase], g1 = tb.g_row_start[min(ybase + RC::ROWS, ny)];
  GatherEnt ge{};
  const bool has_g = dpart && (g0 + tid < g1);   // the argument, not the step-dependent row: no wait for the counter
  if (has_g) ge = tb.g_ent[g0 + tid];
  float2* L[2] = {X[grp][0], X[grp][1]};
  fft.template run<+1, 2, N == 512, true>(v, L, q);
  float2 z[1][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float ays = pay[h];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const float2 d = v[h][m];
      const float axs = pax[m];
      const float nrx = axs * (axs * orx[h][m] - d.x);
      const float nry = ays * (ays * ory[h][m] - d.y);
      orx[h][m] = nrx;
      ory[h][m] = nry;
      const float p = (cc[h][m] * cc[h][m]) * (nrx + nry);
      if (h == 0) z[0][m].x = p; else z[0][m].y = p;
    }
  }
  if (ok) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const unsigned x = q + T * m;
        const float p = h == 0 ? z[0][m].x : z[0][m].y;
        rxr[h][x] = orx[h][m];
        ryr[h][x] = ory[h][m];
        P[2 * grp + h][x] = p;
      }
    if (hist) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int m = 0; m < 8; ++m) hr[h][(unsigned)(q + T * m)] = h == 0 ? z[0][m].x : z[0][m].y;
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int m = 0; m < 8; ++m) P[2 * grp + h][q + T * m] = 0.f;
  }
  wave_sync();   // one-wave blocks
  if (dpart_n) {
    float* dk = dpart_n + (size_t)k * tb.nt * 2 * tb.m;
    if (has_g) {
      const float* pr = &P[ge.row - ybase][0];
      dk[ge.slot * tb.m + ge.sensor] = ge.w0 * pr[ge.ix0] + ge.w1 * pr[ge.ix0 + 1];
    }
    for (int e2 = g0 + 64 + tid; e2 < g1; e2 += 64) {
      const GatherEnt g = tb.g_ent[e2];
      const float* pr = &P[g.row - ybase][0];
      dk[g.slot * tb.m + g.sensor] = g.w0 * pr[g.ix0] + g.w1 * pr[g.ix0 + 1];
    }
  }
  float2* L1[1] = {X[grp][0]};
  fft.template run<-1, 1, N == 512, true>(z, L1, q);
  if (ok) {
    float2* ra = SA + ((size_t)k * ny + y0) * nhf;
    float2* rb = SA + ((size_t)k * ny + y1) * nhf;
    unpack_store<N>(z[0], q, lane_base, ra, rb);
  }
}

template <int N>
__global__ __launch_bounds__(64) void k_fwd_rho(Tables tb, const float* __restrict__ c, float* __restrict__ rx,
                                                float* __restrict__ ry, float* __restrict__ hist_base,
                                                float* __restrict__ dpart, float2* __restrict__ SA,
                                                const float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  fast::k_fwd_rho_body<N>(blockIdx.x, tb, c, rx, ry, hist_base, dpart, SA, SB, ctl);
}

// Adjoint row passes that touch g_c run KB datasets per block (one wave per
// dataset, same rows): each wave leaves its per-pixel g_c term in LDS and the
// block adds the KB terms in dataset order to one g_c slice per dataset group,
// so g_c is read and written once per pixel and group instead of once per
// dataset.  Waves past the last dataset of a partial group compute on a valid
// dataset (block-uniform barriers) and store nothing.
template <int N, int KB>
struct AdjBlk {
  using RC = RowF<N>;
  static constexpr int T = RC::T;
  static constexpr int NR = RC::ROWS * N / (64 * KB);   // reduced pixels per thread
  int G, kg, ybase, wave, lane, kw, k, grp, q, lane_base, y0, y1;
  bool act, ok;
  __device__ __forceinline__ AdjBlk(const Tables& tb, int bid) {
    G = (tb.K + KB - 1) / KB;
    kg = bid % G;
    ybase = (bid / G) * RC::ROWS;
    wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);   // wave-uniform: scalar row addresses
    lane = threadIdx.x % 64;
    kw = kg * KB + wave;
    act = kw < tb.K;
    k = act ? kw : tb.K - 1;
    grp = RC::G == 1 ? 0 : lane / T;   // a literal 0 keeps the row index uniform
    q = lane % T;
    lane_base = grp * T;
    y0 = ybase + 2 * grp;
    y1 = y0 + 1;
    ok = y1 < tb.ny;
  }
  // g_c slice values of this thread's reduced pixels (prefetch)
  __device__ __forceinline__ void load_slice(const Tables& tb, const float* __restrict__ gcg, float (&gp)[NR]) const {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int i = threadIdx.x + j * 64 * KB, r = i / N, x = i % N, y = ybase + r;
      gp[j] = y < tb.ny ? gcg[((size_t)kg * tb.ny + y) * N + x] : 0.f;
    }
  }
  // gcg[slice kg] = prefetched + sum over the group's datasets of their terms
  __device__ __forceinline__ void reduce_store(const Tables& tb, float (*D)[RC::ROWS][N], const float (&gp)[NR],
                                               float* __restrict__ gcg) const {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int i = threadIdx.x + j * 64 * KB, r = i / N, x = i % N, y = ybase + r;
      float s = gp[j];
#pragma unroll
      for (int w = 0; w < KB; ++w)
        if (kg * KB + w < tb.K) s += D[w][r][x];
      if (y < tb.ny) gcg[((size_t)kg * tb.ny + y) * N + x] = s;
    }
  }
};

// adjoint: ph = S^T r^n + (inverse rows of the SUMM spectrum); rh += c^2 ph;
// g_c += (2/c) p^n ph (summed over the block's datasets); spectra of
// (a_x rh_x + i a_y rh_y); rh <- a^2 rh.  Every global load (spectra, state,
// history, g_c slice, sensor injections) is issued before the first transform.
template <int N, int KB>
__device__ __forceinline__ void k_adj_rho_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                               const float* __restrict__ hist_base, const float* __restrict__ resid,
                                               float* __restrict__ rhx, float* __restrict__ rhy,
                                               float* __restrict__ gcg, float2* __restrict__ SA,
                                               float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  using RC = RowF<N>;
  constexpr int T = RC::T;
  const AdjBlk<N, KB> b(tb, bid);
  const int ny = tb.ny, nhf = N / 2, k = b.k, grp = b.grp, q = b.q, y0 = b.y0;
  const bool ok = b.ok, st = b.ok && b.act;
  Fft<N> fft;
  fft.init(tb.tw_x, q);
  const int n = ctl->adj_n;
  const float* p_n = hist_base + (size_t)(n - ctl->hist_first) * tb.K * ny * N;
  const float* resid_n = resid + (size_t)n * tb.m;
  __shared__ float2 X[KB][RC::G][2][Lds<N>::P];
  __shared__ float PH[KB][RC::ROWS][N];
  float2 v[1][8];
  float orx[2][8], ory[2][8], op[2][8], oc[2][8];
  float gp[AdjBlk<N, KB>::NR];
  {
    const float2* A = SA + ((size_t)k * ny + (ok ? y0 : 0)) * nhf;
    const float2* B = SA + ((size_t)k * ny + (ok ? y0 + 1 : 0)) * nhf;
    pack_row<N>(v[0], A, B, q);
  }
  // row pointers (block-uniform at one group per block) + unsigned lane offsets
  float* rxr[2];
  float* ryr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const size_t f = ((size_t)k * ny + y) * N;
    rxr[h] = rhx + f;
    ryr[h] = rhy + f;
    const float* cr = c + (size_t)y * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const unsigned x = q + T * m;
      orx[h][m] = rxr[h][x];
      ory[h][m] = ryr[h][x];
      oc[h][m] = cr[x];
    }
  }
  b.load_slice(tb, gcg, gp);
  float pax[8], pax2[8], pay[2], pay2[2];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    pax[m] = tb.ax[(unsigned)(q + T * m)];
    pax2[m] = tb.ax2[(unsigned)(q + T * m)];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    pay[h] = tb.ay[ok ? y0 + h : 0];
    pay2[h] = tb.ay2[ok ? y0 + h : 0];
  }
  // the history slice of step n last: its address waits for the step counter,
  // and every load above is in flight meanwhile
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const float* pr = p_n + ((size_t)k * ny + y) * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) op[h][m] = pr[(unsigned)(q + T * m)];
  }
  // sensor injections of this block's rows for this wave's dataset: one pixel per lane (prefetched)
  const float* rk = resid_n + (size_t)k * tb.nt * tb.m;
  const int ybase = b.ybase, lane = b.lane;
  const int e0 = tb.s_row_start[ybase], e1 = tb.s_row_start[min(ybase + RC::ROWS, ny)];
  const int e = e0 + lane;
  float inj = 0.f;
  int inj_at = -1;
  if (e < e1) {
    const ScatterPix px = tb.s_pix[e];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < px.count) inj += px.w[t] * rk[px.sensor[t]];
    for (int t = 4; t < px.count; ++t) {
      const ScatterTap tp = tb.s_tap[px.start + t];
      inj += tp.w * rk[tp.sensor];
    }
    inj_at = (px.row - ybase) * N + px.ix;
  }
  float(*P)[N] = PH[b.wave];
  float2* L1[1] = {X[b.wave][grp][0]};
  fft.template run<+1, 1, N == 512, true>(v, L1, q);   // each wave's own rows
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    P[2 * grp][q + T * m] = v[0][m].x;
    P[2 * grp + 1][q + T * m] = v[0][m].y;
  }
  // the wave's own rows (P = PH[wave]): wave-level ordering suffices until the group sum
  wave_sync();
  if (inj_at >= 0) (&P[0][0])[inj_at] += inj;
  if (e1 - e0 > 64) {   // rows crowded with sensors: the remaining pixels, one pass each
    for (int e2 = e0 + 64 + lane; e2 < e1; e2 += 64) {
      const ScatterPix px = tb.s_pix[e2];
      float acc = 0.f;
      for (int t = 0; t < px.count; ++t) {
        const ScatterTap tp = tb.s_tap[px.start + t];
        acc += tp.w * rk[tp.sensor];
      }
      (&P[0][0])[(px.row - ybase) * N + px.ix] += acc;
    }
  }
  wave_sync();
  float2 w[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float ays = pay[h], ay2s = pay2[h];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const unsigned x = q + T * m;
      const float ph = P[2 * grp + h][x];
      const float cv = oc[h][m];
      const float c2 = cv * cv;
      const float nrx = orx[h][m] + c2 * ph;
      const float nry = ory[h][m] + c2 * ph;
      // this dataset's sound-speed term, 2/c with the hardware reciprocal (1 ulp);
      // left in place of ph (each lane rereads only its own pixels)
      P[2 * grp + h][x] = (2.0f * __builtin_amdgcn_rcpf(cv)) * op[h][m] * ph;
      orx[h][m] = pax2[m] * nrx;
      ory[h][m] = ay2s * nry;
      w[h][m] = make_float2(pax[m] * nrx, ays * nry);
    }
  }
  if (st) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        rxr[h][(unsigned)(q + T * m)] = orx[h][m];
        ryr[h][(unsigned)(q + T * m)] = ory[h][m];
      }
  }
  __syncthreads();
  b.reduce_store(tb, PH, gp, gcg);
  float2* L[2] = {X[b.wave][grp][0], X[b.wave][grp][1]};
  fft.template run<-1, 2, N == 512, true>(w, L, q);
  if (st) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t r = ((size_t)k * ny + y0 + h) * nhf;
      unpack_store<N>(w[h], q, b.lane_base, SA + r, SB + r);
    }
  }
}

template <int N, int KB>
__global__ __launch_bounds__(64 * KB) void k_adj_rho(Tables tb, const float* __restrict__ c,
                                                     const float* __restrict__ hist_base,
                                                     const float* __restrict__ resid, float* __restrict__ rhx,
                                                     float* __restrict__ rhy, float* __restrict__ gcg,
                                                     float2* __restrict__ SA, float2* __restrict__ SB,
                                                     const StepCtl* __restrict__ ctl) {
  fast::k_adj_rho_body<N, KB>(blockIdx.x, tb, c, hist_base, resid, rhx, rhy, gcg, SA, SB, ctl);
}

// adjoint velocities: uh <- as^2 uh + (inverse rows of PAIRP spectra);
// spectra of (w_x uh_x + i w_y uh_y), w = as, or as - as^2/2 at adjoint step n = 1
template <int N>
__device__ __forceinline__ void k_adj_u_body(const int bid, const Tables& tb, float* __restrict__ uhx,
                                             float* __restrict__ uhy, float2* __restrict__ SA,
                                             float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  PAT_ROW_PROLOGUE(N)
  const int final_ = ctl->adj_n == 1;
  __shared__ float2 X[RC::G][2][Lds<N>::P];
  float2 v[2][8];
  float ox[2][8], oy[2][8];
  const bool ok = y1 < ny;
  // row pointers (block-uniform at one group per block) + unsigned lane offsets
  float* uxr[2];
  float* uyr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const size_t f = ((size_t)k * ny + y) * N;
    uxr[h] = uhx + f;
    uyr[h] = uhy + f;
    pack_row<N>(v[h], SA + ((size_t)k * ny + y) * nhf, SB + ((size_t)k * ny + y) * nhf, q);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      ox[h][m] = uxr[h][(unsigned)(q + T * m)];
      oy[h][m] = uyr[h][(unsigned)(q + T * m)];
    }
  }
  const float* wxt = final_ ? tb.wfx : tb.asx;
  const float* wyt = final_ ? tb.wfy : tb.asy;
  float pa2x[8], pwx[8], pa2y[2], pwy[2];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    pa2x[m] = tb.asx2[(unsigned)(q + T * m)];
    pwx[m] = wxt[(unsigned)(q + T * m)];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    pa2y[h] = tb.asy2[ok ? y0 + h : 0];
    pwy[h] = wyt[ok ? y0 + h : 0];
  }
  float2* L[2] = {X[grp][0], X[grp][1]};
  fft.template run<+1, 2, N == 512, true>(v, L, q);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float a2y = pa2y[h];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const float2 g = v[h][m];
      ox[h][m] = pa2x[m] * ox[h][m] + g.x;
      oy[h][m] = a2y * oy[h][m] + g.y;
      v[h][m] = make_float2(pwx[m] * ox[h][m], pwy[h] * oy[h][m]);
    }
  }
  if (ok) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        uxr[h][(unsigned)(q + T * m)] = ox[h][m];
        uyr[h][(unsigned)(q + T * m)] = oy[h][m];
      }
  }
  fft.template run<-1, 2, N == 512, true>(v, L, q);
  if (ok) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const size_t r = ((size_t)k * ny + y0 + h) * nhf;
      unpack_store<N>(v[h], q, lane_base, SA + r, SB + r);
    }
  }
}

template <int N>
__global__ __launch_bounds__(64) void k_adj_u(Tables tb, float* __restrict__ uhx, float* __restrict__ uhy,
                                              float2* __restrict__ SA, float2* __restrict__ SB,
                                              const StepCtl* __restrict__ ctl) {
  fast::k_adj_u_body<N>(blockIdx.x, tb, uhx, uhy, SA, SB, ctl);
}

// closing terms of the adjoint: g_p0 and the initial-state part of g_c
// (summed over the block's datasets into the group's g_c slice)
template <int N, int KB>
__device__ __forceinline__ void k_adj_final_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                                 const float* __restrict__ p0, const float* __restrict__ resid0,
                                                 const float* __restrict__ rhx, const float* __restrict__ rhy,
                                                 float* __restrict__ gcg, float* __restrict__ gp0,
                                                 const float2* __restrict__ SA) {
  using RC = RowF<N>;
  constexpr int T = RC::T;
  const AdjBlk<N, KB> b(tb, bid);
  const int ny = tb.ny, nhf = N / 2, k = b.k, grp = b.grp, q = b.q, y0 = b.y0;
  const bool ok = b.ok;
  Fft<N> fft;
  fft.init(tb.tw_x, q);
  __shared__ float2 X[KB][RC::G][Lds<N>::P];
  __shared__ float PH[KB][RC::ROWS][N];
  float gp[AdjBlk<N, KB>::NR];
  b.load_slice(tb, gcg, gp);
  float2 v[1][8];
  {
    const float2* A = SA + ((size_t)k * ny + (ok ? y0 : 0)) * nhf;
    const float2* B = SA + ((size_t)k * ny + (ok ? y0 + 1 : 0)) * nhf;
    pack_row<N>(v[0], A, B, q);
  }
  float(*P)[N] = PH[b.wave];
  float2* L1[1] = {X[b.wave][grp]};
  fft.template run<+1, 1, N == 512>(v, L1, q);
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    P[2 * grp][q + T * m] = v[0][m].x;
    P[2 * grp + 1][q + T * m] = v[0][m].y;
  }
  __syncthreads();
  scatter_rows<N, 64>(tb, &P[0][0], b.ybase, RC::ROWS, resid0 + (size_t)k * tb.nt * tb.m, b.lane);
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = ok ? y0 + h : 0;
    const size_t f = ((size_t)k * ny + y) * N;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const unsigned x = q + T * m;
      const float cv = c[(size_t)y * N + x];
      const float rs = rhx[f + x] + rhy[f + x];
      if (ok && b.act) gp0[f + x] = P[2 * grp + h][x] + rs * (0.5f / (cv * cv));
      P[2 * grp + h][x] = -(p0[f + x] / (cv * cv * cv)) * rs;
    }
  }
  __syncthreads();
  b.reduce_store(tb, PH, gp, gcg);
}

template <int N, int KB>
__global__ __launch_bounds__(64 * KB) void k_adj_final(Tables tb, const float* __restrict__ c,
                                                       const float* __restrict__ p0, const float* __restrict__ resid0,
                                                       const float* __restrict__ rhx, const float* __restrict__ rhy,
                                                       float* __restrict__ gcg, float* __restrict__ gp0,
                                                       const float2* __restrict__ SA) {
  fast::k_adj_final_body<N, KB>(blockIdx.x, tb, c, p0, resid0, rhx, rhy, gcg, gp0, SA);
}

// Spectral products of the column passes with contraction off: every product
// and sum rounds on its own, so the column-pass variants (which place these
// products differently over threads and registers) form the same bits.
__device__ __forceinline__ float2 sp_mul(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 sp_add(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x + b.x, a.y + b.y);
}
// o0 + i oN
__device__ __forceinline__ float2 sp_join(float2 o0, float2 oN) {
#pragma clang fp contract(off)
  return make_float2(o0.x - oN.y, o0.y + oN.x);
}

// ===========================================================================
// Column pass (transform length NY = N), nx/2 folded columns, TC per block
// ===========================================================================
// TC: columns per block (the default Cfg<N>::TC, or a width picked by the tuner).
// SEQ: the two transforms of a thread run one after the other (the second
// array's loads issued once the first array's data have arrived, so that its
// transform runs while the second array streams in, and the first output is
// stored while the second is transformed) instead of stage by stage together
// (shared barriers).  Same arithmetic.
template <int N, int MODE, int TC = Cfg<N>::TC, bool SEQ = false>
__device__ __forceinline__ void k_col_body(const int bid, const Tables& tb, float2* __restrict__ SA,
                                           float2* __restrict__ SB, float scale, int32_t* __restrict__ step,
                                           int32_t delta) {
  constexpr int T = Cfg<N>::T, P = LdsCol<N, TC>::P;
  static_assert((TC == 4 && P % 16 == 4) || (TC == 8 && P % 16 == 2) || (TC >= 16 && P % 2 == 1),
                "column pitch");
  constexpr bool TWO_IN = MODE != COL_GRAD1;
  constexpr bool TWO_OUT = MODE != COL_SUMM;
  __shared__ float2 LA[TC * P];
  __shared__ float2 LB[(TWO_IN || TWO_OUT) ? TC * P : 1];
  const int K = tb.K, nx = tb.nx, nhf = nx / 2;
  const int k = bid % K, c0 = (bid / K) * TC;
  const int tid = threadIdx.x, cl = tid % TC, q = tid / TC, cx = c0 + cl;
  const bool ok = cx < nhf;
  // dataset base pointers (block-uniform) + 32-bit byte offsets per lane and row
  float2* const colA = SA + (size_t)k * N * nhf;
  float2* const colB = SB + (size_t)k * N * nhf;
  const unsigned lane_b = ((unsigned)q * nhf + (ok ? cx : 0)) * 8u, row_b = (unsigned)T * nhf * 8u;
  Fft<N> fft;
  float2 a[2][8];
  if (SEQ) {
#pragma unroll
    for (int m = 0; m < 8; ++m) a[0][m] = *at_byte(colA, lane_b + m * row_b);
    if (TWO_IN) {
      // staged: the second array's loads issue once the first array's data
      // have arrived, so that they stream in while the first is transformed
      // (loads issued together arrive interleaved, and neither transform
      // could start before the end of both)
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
      for (int m = 0; m < 8; ++m) a[1][m] = *at_byte(colB, lane_b + m * row_b);
    }
  } else {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const unsigned o = lane_b + m * row_b;
      a[0][m] = *at_byte(colA, o);
      if (TWO_IN) a[1][m] = *at_byte(colB, o);
    }
  }
  // spectral multiplier factors (prefetched before the transforms)
  constexpr bool PLUS = MODE == COL_GRAD1 || MODE == COL_PAIRP;
  const float2* eyt = PLUS ? tb.ey_p : tb.ey_m;
  const float2* ext = PLUS ? tb.ex_p : tb.ex_m;
  const bool col0 = c0 == 0 && cl == 0;   // DC + i Nyquist column
  // the tables every column of the block shares (transform twiddles, y shift
  // factors) pass through shared memory: a few loads per thread instead of
  // one per twiddle and factor
  constexpr int NTH = TC * T, NST = (N + NTH - 1) / NTH;
  __shared__ float2 TWs[N], EYs[N];
  float2 stw[NST], sey[NST];
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int i = tid + j * NTH;
    if (NTH * NST == N || i < N) { stw[j] = tb.tw_y[i]; sey[j] = eyt[i]; }
  }
  float kap[8], kapN[8];
  float2 eyv[8];
  const float2 exv = ext[col0 ? 0 : (ok ? cx : 0)];
  const float2 exN = ext[nx / 2];
  // kappa is column-major, so a wave reads 64-byte runs of it; the Nyquist
  // column's kappa only in the block that holds column 0 (a block-uniform
  // branch: no lane waits inside a divergent branch)
  const float* const kcol = tb.kappa + (size_t)(ok ? cx : 0) * N;
  const float* const kcolN = tb.kappa + (size_t)(nx / 2) * N;
#pragma unroll
  for (int m = 0; m < 8; ++m) kap[m] = kcol[q + T * m] * scale;
  if (c0 == 0) {
#pragma unroll
    for (int m = 0; m < 8; ++m) kapN[m] = kcolN[q + T * m] * scale;
  }
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int i = tid + j * NTH;
    if (NTH * NST == N || i < N) { TWs[i] = stw[j]; EYs[i] = sey[j]; }
  }
  __syncthreads();
  fft.init(TWs, q);
#pragma unroll
  for (int m = 0; m < 8; ++m) eyv[m] = EYs[q + T * m];
  float2* LL[2] = {LA + cl * P, LB + cl * P};
  if (TWO_IN && SEQ) {
    fft.template run<-1, 1>(&a[0], &LL[0], q);
    fft.template run<-1, 1>(&a[1], &LL[1], q);
  } else if (TWO_IN) {
    fft.template run<-1, 2>(a, LL, q);
  } else {
    fft.template run<-1, 1>(a, LL, q);
  }
  if (c0 == 0) {
    // column 0 holds DC + i Nyquist: split by conjugate symmetry along y
    __syncthreads();
    if (cl == 0) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        LA[phys(q + T * m)] = a[0][m];
        if (TWO_IN) LB[phys(q + T * m)] = a[1][m];
      }
    }
    __syncthreads();
    if (cl == 0) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = q + T * m, ep = (N - e) & (N - 1);
        const float k0 = kap[m], kN = kapN[m];
        const float2 ey = eyv[m];
        float2 ZA = a[0][m], ZAp = LA[phys(ep)];
        // A0 = (Z + conj Zp)/2 (DC column), AN = (Z - conj Zp)/(2i) (Nyquist column)
        float2 A0 = make_float2(0.5f * (ZA.x + ZAp.x), 0.5f * (ZA.y - ZAp.y));
        float2 AN = make_float2(0.5f * (ZA.y + ZAp.y), -0.5f * (ZA.x - ZAp.x));
        float2 B0 = A0, BN = AN;
        if (TWO_IN) {
          const float2 ZB = a[1][m], ZBp = LB[phys(ep)];
          B0 = make_float2(0.5f * (ZB.x + ZBp.x), 0.5f * (ZB.y - ZBp.y));
          BN = make_float2(0.5f * (ZB.y + ZBp.y), -0.5f * (ZB.x - ZBp.x));
        }
        float2 o0, oN, p0_, pN;
        if (MODE == COL_GRAD1) {
          o0 = cscale(sp_mul(A0, exv), k0); oN = cscale(sp_mul(AN, exN), kN);
          p0_ = cscale(sp_mul(A0, ey), k0); pN = cscale(sp_mul(AN, ey), kN);
        } else if (MODE == COL_PAIRP || MODE == COL_PAIRM) {
          o0 = cscale(sp_mul(A0, exv), k0); oN = cscale(sp_mul(AN, exN), kN);
          p0_ = cscale(sp_mul(B0, ey), k0); pN = cscale(sp_mul(BN, ey), kN);
        } else {
          o0 = cscale(sp_add(sp_mul(A0, exv), sp_mul(B0, ey)), k0);
          oN = cscale(sp_add(sp_mul(AN, exN), sp_mul(BN, ey)), kN);
          p0_ = o0; pN = oN;
        }
        // recombine: out = o0 + i oN
        a[0][m] = sp_join(o0, oN);
        if (TWO_OUT) a[1][m] = sp_join(p0_, pN);
      }
    }
  }
  if (!col0) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const float2 x0 = a[0][m];
      if (MODE == COL_GRAD1) {
        a[0][m] = cscale(sp_mul(x0, exv), kap[m]);
        a[1][m] = cscale(sp_mul(x0, eyv[m]), kap[m]);
      } else if (MODE == COL_PAIRP || MODE == COL_PAIRM) {
        a[0][m] = cscale(sp_mul(x0, exv), kap[m]);
        a[1][m] = cscale(sp_mul(a[1][m], eyv[m]), kap[m]);
      } else {
        a[0][m] = cscale(sp_add(sp_mul(x0, exv), sp_mul(a[1][m], eyv[m])), kap[m]);
      }
    }
  }
  if (TWO_OUT && SEQ) {
    fft.template run<+1, 1>(&a[0], &LL[0], q);
    if (ok) {
#pragma unroll
      for (int m = 0; m < 8; ++m) *at_byte(colA, lane_b + m * row_b) = a[0][m];
    }
    fft.template run<+1, 1>(&a[1], &LL[1], q);
    if (ok) {
#pragma unroll
      for (int m = 0; m < 8; ++m) *at_byte(colB, lane_b + m * row_b) = a[1][m];
    }
  } else {
    if (TWO_OUT)
      fft.template run<+1, 2>(a, LL, q);
    else
      fft.template run<+1, 1>(a, LL, q);
    if (ok) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const unsigned o = lane_b + m * row_b;
        *at_byte(colA, o) = a[0][m];
        if (TWO_OUT) *at_byte(colB, o) = a[1][m];
      }
    }
  }
  // first pass of a step: advance the step counter (read by the row passes
  // that follow, not by this one), after the stores so that no block waits
  // for it before its own loads
  if (step && bid == 0 && threadIdx.x == 0) *step += delta;
}

// Split column pass: the two arrays of a pass on the two halves of a block
// (twice the threads of k_col, one transform per thread), so that a launch
// holds twice the waves.  Array A on threads [0, TC*T), array B on
// [TC*T, 2*TC*T).  Single-input pass (COL_GRAD1): both halves transform A and
// each applies its own direction's factor.  Single-output pass (COL_SUMM): the
// B half hands its weighted spectrum to the A half through shared memory and
// then runs the same inverse transform on its registers (result discarded), so
// that both halves pass the same barriers.  Same arithmetic as k_col.
template <int N, int MODE, int TC = Cfg<N>::TC>
__device__ __forceinline__ void k_cols_body(const int bid, const Tables& tb, float2* __restrict__ SA,
                                            float2* __restrict__ SB, float scale, int32_t* __restrict__ step,
                                            int32_t delta) {
  constexpr int T = Cfg<N>::T, P = LdsCol<N, TC>::P, HALF = TC * T;
  static_assert(HALF % 64 == 0, "each half is whole waves");
  static_assert((TC == 4 && P % 16 == 4) || (TC == 8 && P % 16 == 2) || (TC >= 16 && P % 2 == 1),
                "column pitch");
  constexpr bool TWO_IN = MODE != COL_GRAD1;
  constexpr bool SUMM = MODE == COL_SUMM;
  __shared__ float2 LS[2][TC * P];
  __shared__ float2 Q0[SUMM ? N : 1];   // COL_SUMM: B's products of column 0, DC part
  __shared__ float2 QN[SUMM ? N : 1];   // and Nyquist part
  __shared__ float2 QA[SUMM ? N : 1];   // A's Nyquist part of column 0
  const int K = tb.K, nx = tb.nx, nhf = nx / 2;
  const int k = bid % K, c0 = (bid / K) * TC;
  const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.x / HALF);   // 0: array A, 1: array B
  const int tid = (int)threadIdx.x - s * HALF, cl = tid % TC, q = tid / TC, cx = c0 + cl;
  const bool ok = cx < nhf;
  const size_t koff = (size_t)k * N * nhf;
  float2* const src = ((TWO_IN && s) ? SB : SA) + koff;
  float2* const dst = (s ? SB : SA) + koff;
  const unsigned lane_b = ((unsigned)q * nhf + (ok ? cx : 0)) * 8u, row_b = (unsigned)T * nhf * 8u;
  Fft<N> fft;
  fft.init(tb.tw_y, q);
  float2 a[1][8];
#pragma unroll
  for (int m = 0; m < 8; ++m) a[0][m] = *at_byte(src, lane_b + m * row_b);
  float2* const L = LS[s] + cl * P;
  float2* LL[1] = {L};
  fft.template run<-1, 1>(a, LL, q);
  // spectral factors, loaded after the forward transform (fewer live
  // registers; other waves hide the latency): this half's direction factor
  // (x: per column, y: per row) and kappa
  constexpr bool PLUS = MODE == COL_GRAD1 || MODE == COL_PAIRP;
  const float2* eyt = PLUS ? tb.ey_p : tb.ey_m;
  const float2* ext = PLUS ? tb.ex_p : tb.ex_m;
  const bool col0 = c0 == 0 && cl == 0;   // DC + i Nyquist column
  float kap[8];
  float2 fac[8];
  float kap_n[SUMM ? 8 : 1];   // COL_SUMM, half A, column 0: kappa of the Nyquist part
  // branch-free per half: half A reads its column's x factor (the same
  // address for every m), half B the y factor of each of its rows
  const float2* const ft = s ? eyt : ext;
  const unsigned f_b = (s ? (unsigned)q : (unsigned)(ok ? cx : 0)) * 8u, f_step = s ? (unsigned)T * 8u : 0u;
  // kappa is column-major: a wave reads 64-byte runs of it
  const unsigned k_b = ((unsigned)(ok ? cx : 0) * N + q) * 4u, k_step = (unsigned)T * 4u;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    kap[m] = *at_byte(tb.kappa, k_b + m * k_step) * scale;
    fac[m] = *at_byte(ft, f_b + m * f_step);
  }
  // own-direction products, in place: x direction (half A), y direction
  // (half B), times kappa; column 0 splits into its DC and Nyquist parts by
  // conjugate symmetry along y.  COL_SUMM: the B half stores its products
  // unscaled (column 0's two parts in Q0 and QN, the other columns over its
  // own transform positions, which no other thread reads any more) and the A
  // half adds them before scaling.
  if (c0 == 0) {   // block-uniform
    const float2 exN = ext[nx / 2];
    const unsigned n_b = ((unsigned)(nx / 2) * N + q) * 4u;
    float kapN[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) kapN[m] = *at_byte(tb.kappa, n_b + m * k_step) * scale;
    __syncthreads();
    if (cl == 0) {
#pragma unroll
      for (int m = 0; m < 8; ++m) L[phys(q + T * m)] = a[0][m];
    }
    __syncthreads();
    if (cl == 0) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = q + T * m, ep = (N - e) & (N - 1);
        const float2 Z = a[0][m], Zp = L[phys(ep)];
        const float2 X0 = make_float2(0.5f * (Z.x + Zp.x), 0.5f * (Z.y - Zp.y));
        const float2 XN = make_float2(0.5f * (Z.y + Zp.y), -0.5f * (Z.x - Zp.x));
        const float2 u0 = sp_mul(X0, fac[m]), uN = sp_mul(XN, s ? fac[m] : exN);
        if (SUMM && s) {
          Q0[e] = u0;
          QN[e] = uN;
        } else if (!SUMM) {
          const float2 o0 = cscale(u0, kap[m]), oN = cscale(uN, kapN[m]);
          a[0][m] = sp_join(o0, oN);
        } else {
          a[0][m] = u0;                 // A's parts, combined below
          QA[e] = uN;
          kap_n[m] = kapN[m];
        }
      }
    }
  }
  if (!col0) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const float2 u = sp_mul(a[0][m], fac[m]);
      if (SUMM && s)
        L[phys(q + T * m)] = u;
      else if (!SUMM)
        a[0][m] = cscale(u, kap[m]);
      else
        a[0][m] = u;
    }
  }
  if (SUMM) {
    __syncthreads();
    if (!s) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = q + T * m;
        if (col0) {
          const float2 o0 = cscale(sp_add(a[0][m], Q0[e]), kap[m]);
          const float2 oN = cscale(sp_add(QA[e], QN[e]), kap_n[m]);
          a[0][m] = sp_join(o0, oN);
        } else {
          a[0][m] = cscale(sp_add(a[0][m], LS[1][cl * P + phys(e)]), kap[m]);
        }
      }
    }
  }
  fft.template run<+1, 1>(a, LL, q);
  if (ok && (!SUMM || !s)) {
#pragma unroll
    for (int m = 0; m < 8; ++m) *at_byte(dst, lane_b + m * row_b) = a[0][m];
  }
  if (step && bid == 0 && threadIdx.x == 0) *step += delta;
}

template <int N, int MODE, int TC = Cfg<N>::TC>
__global__ __launch_bounds__(2 * TC * Cfg<N>::T, 4) void k_cols(Tables tb, float2* __restrict__ SA,
                                                                 float2* __restrict__ SB, float scale,
                                                                 int32_t* __restrict__ step, int32_t delta) {
  fast::k_cols_body<N, MODE, TC>(blockIdx.x, tb, SA, SB, scale, step, delta);
}

template <int N, int MODE, int TC = Cfg<N>::TC, bool SEQ = false>
__global__ __launch_bounds__(TC * Cfg<N>::T) void k_col(Tables tb, float2* __restrict__ SA,
                                                                float2* __restrict__ SB, float scale,
                                                                int32_t* __restrict__ step, int32_t delta) {
  fast::k_col_body<N, MODE, TC, SEQ>(blockIdx.x, tb, SA, SB, scale, step, delta);
}

}  // namespace fast
}  // namespace pat
