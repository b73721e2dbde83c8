// wave_kernels.hpp — fused row / column passes of the k-space forward solver
// and of its exact discrete adjoint (gfx950).
//
// Scheme (Sec. 2.1, eq. (1), solved by a k-space pseudospectral method; the
// first-order staggered split-field form with constant ambient density):
//   u_x  <- as_x (as_x u_x  - dt/rho0 Dx+ p)          (same for y)
//   rho_x<- a_x  (a_x  rho_x - dt rho0 Dx- u_x)        (same for y)
//   p     = c^2 (rho_x + rho_y)
// with D+- f = IFFT2[ i k kappa exp(+-i k dx/2) FFT2 f ], kappa = sinc(c_ref |k| dt/2).
//
// A 2-D transform is a row pass (along x, contiguous) and a column pass
// (along y).  Each time step is four passes over HBM:
//   col GRAD  : spectrum of p -> spectra of dt/rho0 Dx+ p, Dy+ p
//   row U     : inverse rows, velocity update + PML, forward rows of (u_x + i u_y)
//   col DIV   : spectra of u_x, u_y -> spectra of dt rho0 Dx- u_x, Dy- u_y
//   row RHO   : inverse rows, density update + PML, p = c^2 (rho_x + rho_y),
//               sensor sampling, pressure history, forward rows of p
// Spectra are half spectra along x ([K][ny][nx/2+1] complex): two real rows
// share one complex FFT (z = a + i b), so every row transform is a full
// complex transform of length nx.  The adjoint runs the transposed passes
// backwards in time (eqs. (5)-(9) for the discrete scheme).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace pat {

struct GatherEnt {   // one (sensor, tap row) pair: partial = w0 p[ix0] + w1 p[ix0+1]
  int32_t row, ix0, sensor, slot;
  float w0, w1;
};
struct ScatterPix {  // one pixel receiving sensor injections: sum over its taps
  int32_t row, ix, start, count;   // taps s_tap[start .. start + count)
  int32_t sensor[4];               // the first four taps inline (one load for the usual case)
  float w[4];
};
struct ScatterTap {
  int32_t sensor;
  float w;
};

// Device control block (in the workspace): the step indices that the time-step
// kernels read, so that a chunk of steps has identical launch arguments (and can
// be replayed as one captured graph).  The first pass of each step advances the
// counter; nothing else writes it.
struct StepCtl {
  int32_t fwd_n;       // forward update n -> n+1 in progress
  int32_t adj_n;       // adjoint step n in progress
  int32_t hist_first;  // time level stored in slot 0 of the pressure-history buffer
  int32_t pad;
};

// Device tables owned by a plan.
struct Tables {
  const float2* tw_x;   // [nx] exp(-2 pi i j / nx)
  const float2* tw_y;   // [ny]
  const float2* ex_p;   // [nh] kx * (i exp(+i kx dx/2)), real at the Nyquist column
  const float2* ex_m;   // [nh] kx * (i exp(-i kx dx/2))
  const float2* ey_p;   // [ny]
  const float2* ey_m;   // [ny]
  const float* kappa;   // [nh][ny] sinc(c_ref |k| dt / 2), column-major: the column passes read it along y
  const float* ax;      // [nx] exp(-alpha dt/2) at grid points
  const float* asx;     // [nx] at staggered points (i + 1/2)
  const float* ax2;     // [nx] ax^2
  const float* asx2;    // [nx] asx^2
  const float* wfx;     // [nx] asx - asx^2/2 (closing term of the adjoint)
  const float* ay;
  const float* asy;
  const float* ay2;
  const float* asy2;
  const float* wfy;
  const int32_t* g_row_start;  // [ny+1] into g_ent (sorted by row)
  const GatherEnt* g_ent;
  const int32_t* s_row_start;  // [ny+1] into s_pix (sorted by row)
  const ScatterPix* s_pix;
  const ScatterTap* s_tap;
  int32_t nx, ny, nh, K, m, nt;
};

template <int N> struct RowCfg {
  static constexpr int T = Threads<N>::v;   // threads per row transform
  static constexpr int BLOCK = 256;
  static constexpr int ROWS = BLOCK / T;    // rows per block (even)
  static constexpr int PITCH = N + 1;       // LDS pitch (complex) of one transform
};

template <int N> struct ColCfg {
  static constexpr int T = Threads<N>::v;
  static constexpr int TC = (256 / T) > 8 ? (256 / T) : 8;   // columns per block
  static constexpr int BLOCK = TC * T;
  static constexpr int PITCH = N + 1;
};

// z = a + i b from two half spectra A, B of real rows (Hermitian extension);
// the DC and Nyquist bins of a real row are real, so their imaginary parts
// are dropped (what an inverse real transform does).
__device__ __forceinline__ float2 pack_two(const float2* __restrict__ A, const float2* __restrict__ B,
                                           int kk, int N, int nh) {
  if (kk < nh) {
    float2 a = A[kk], b = B[kk];
    if (kk == 0 || 2 * kk == N) { a.y = 0.f; b.y = 0.f; }
    return make_float2(a.x - b.y, a.y + b.x);
  }
  float2 a = A[N - kk], b = B[N - kk];
  return make_float2(a.x + b.y, b.x - a.y);   // conj(a) + i conj(b)
}

// Split Z = FFT(a + i b) into the half spectra of a and b at bin kk.
__device__ __forceinline__ void unpack_two(const float2* __restrict__ Z, int kk, int N, float2& A, float2& B) {
  float2 P = Z[kk];
  float2 Qc = Z[kk == 0 ? 0 : N - kk];
  float2 Q = make_float2(Qc.x, -Qc.y);
  A = make_float2(0.5f * (P.x + Q.x), 0.5f * (P.y + Q.y));
  B = make_float2(0.5f * (P.y - Q.y), -0.5f * (P.x - Q.x));
}

// ---------------------------------------------------------------------------
// Sensor sampling of the rows [y0, y0 + rows) held in LDS (P: [ROWS][NX]).
// ---------------------------------------------------------------------------
template <int NX, int BLOCK>
__device__ __forceinline__ void gather_rows(const Tables& tb, const float* P, int y0, int rows,
                                            float* __restrict__ dpart_kn, int tid) {
  const int ylast = min(y0 + rows, tb.ny);
  const int e0 = tb.g_row_start[y0], e1 = tb.g_row_start[ylast];
  for (int e = e0 + tid; e < e1; e += BLOCK) {
    const GatherEnt g = tb.g_ent[e];
    const float* pr = P + (g.row - y0) * NX;
    dpart_kn[g.slot * tb.m + g.sensor] = g.w0 * pr[g.ix0] + g.w1 * pr[g.ix0 + 1];
  }
}

// Adjoint source injection S^T r^n into the rows held in LDS (PH: [ROWS][NX]).
template <int NX, int BLOCK>
__device__ __forceinline__ void scatter_rows(const Tables& tb, float* PH, int y0, int rows,
                                             const float* __restrict__ r_kn, int tid) {
  const int ylast = min(y0 + rows, tb.ny);
  const int e0 = tb.s_row_start[y0], e1 = tb.s_row_start[ylast];
  for (int e = e0 + tid; e < e1; e += BLOCK) {
    const ScatterPix px = tb.s_pix[e];
    float acc = 0.f;
    for (int t = 0; t < px.count; ++t) {
      const ScatterTap tp = tb.s_tap[px.start + t];
      acc += tp.w * r_kn[tp.sensor];
    }
    PH[(px.row - y0) * NX + px.ix] += acc;
  }
}

// ===========================================================================
// Forward passes
// ===========================================================================

// n = 0: p = p0, rho_x = rho_y = p0 / (2 c^2), sensors, history, row spectra of p0.
template <int NX>
__device__ __forceinline__ void k_fwd_init_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                                const float* __restrict__ p0, float* __restrict__ rx,
                                                float* __restrict__ ry, float* __restrict__ hist0,
                                                float* __restrict__ dpart, float2* __restrict__ SA) {
  using C = RowCfg<NX>;
  __shared__ float2 Z[C::ROWS / 2][C::PITCH];
  __shared__ float P[C::ROWS][NX];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x, r = tid / C::T, q = tid % C::T, y = y0 + r;
  const size_t fk = (size_t)k * ny * NX;
  if (y < ny) {
    for (int x = q; x < NX; x += C::T) {
      const size_t i = fk + (size_t)y * NX + x;
      const float v = p0[i];
      const float cc = c[(size_t)y * NX + x];
      const float rr = v * (0.5f / (cc * cc));
      rx[i] = rr;
      ry[i] = rr;
      if (hist0) hist0[i] = v;
      P[r][x] = v;
    }
  } else {
    for (int x = q; x < NX; x += C::T) P[r][x] = 0.f;
  }
  __syncthreads();
  if (dpart) gather_rows<NX, C::BLOCK>(tb, &P[0][0], y0, C::ROWS, dpart + (size_t)k * tb.nt * 2 * tb.m, tid);
  constexpr int T2 = 2 * C::T;
  const int pr = tid / T2, q2 = tid % T2;
  for (int x = q2; x < NX; x += T2) Z[pr][x] = make_float2(P[2 * pr][x], P[2 * pr + 1][x]);
  __syncthreads();
  fft<NX, T2, -1>(Z[pr], tb.tw_x, q2, true);
  for (int kk = q2; kk < nh; kk += T2) {
    float2 A, B;
    unpack_two(Z[pr], kk, NX, A, B);
    const int ya = y0 + 2 * pr;
    if (ya < ny) SA[((size_t)k * ny + ya) * nh + kk] = A;
    if (ya + 1 < ny) SA[((size_t)k * ny + ya + 1) * nh + kk] = B;
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_fwd_init(Tables tb, const float* __restrict__ c,
                                                  const float* __restrict__ p0, float* __restrict__ rx,
                                                  float* __restrict__ ry, float* __restrict__ hist0,
                                                  float* __restrict__ dpart, float2* __restrict__ SA) {
  pat::k_fwd_init_body<NX>(blockIdx.x, tb, c, p0, rx, ry, hist0, dpart, SA);
}

// Velocity update.  first != 0: u^{-1/2} = dt/(2 rho0) D+ p0 = G/2 (eq. (1): p_t(0) = 0).
template <int NX>
__device__ __forceinline__ void k_fwd_u_body(const int bid, const Tables& tb, float* __restrict__ ux,
                                             float* __restrict__ uy, float2* __restrict__ SA, float2* __restrict__ SB,
                                             const StepCtl* __restrict__ ctl) {
  using C = RowCfg<NX>;
  const int first = ctl->fwd_n == 0;
  __shared__ float2 Z[C::ROWS][C::PITCH];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x, r = tid / C::T, q = tid % C::T, y = y0 + r;
  const bool ok = y < ny;
  const size_t srow = ((size_t)k * ny + (ok ? y : 0)) * nh;
  if (ok)
    for (int kk = q; kk < NX; kk += C::T) Z[r][kk] = pack_two(SA + srow, SB + srow, kk, NX, nh);
  __syncthreads();
  fft<NX, C::T, +1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    const float ay_s = tb.asy[y];
    const size_t f = ((size_t)k * ny + y) * NX;
    for (int x = q; x < NX; x += C::T) {
      const float2 g = Z[r][x];
      const float ax_s = tb.asx[x];
      const float uxo = first ? 0.5f * g.x : ux[f + x];
      const float uyo = first ? 0.5f * g.y : uy[f + x];
      const float nux = ax_s * (ax_s * uxo - g.x);
      const float nuy = ay_s * (ay_s * uyo - g.y);
      ux[f + x] = nux;
      uy[f + x] = nuy;
      Z[r][x] = make_float2(nux, nuy);
    }
  }
  __syncthreads();
  fft<NX, C::T, -1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    for (int kk = q; kk < nh; kk += C::T) {
      float2 A, B;
      unpack_two(Z[r], kk, NX, A, B);
      SA[srow + kk] = A;
      SB[srow + kk] = B;
    }
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_fwd_u(Tables tb, float* __restrict__ ux, float* __restrict__ uy,
                                               float2* __restrict__ SA, float2* __restrict__ SB,
                                               const StepCtl* __restrict__ ctl) {
  pat::k_fwd_u_body<NX>(blockIdx.x, tb, ux, uy, SA, SB, ctl);
}

// Density / pressure update, sensors at time level n+1, history, row spectra of p.
template <int NX>
__device__ __forceinline__ void k_fwd_rho_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                               float* __restrict__ rx, float* __restrict__ ry,
                                               float* __restrict__ hist_base, float* __restrict__ dpart,
                                               float2* __restrict__ SA, const float2* __restrict__ SB,
                                               const StepCtl* __restrict__ ctl) {
  using C = RowCfg<NX>;
  const int n = ctl->fwd_n;
  float* hist = hist_base ? hist_base + (size_t)(n + 1 - ctl->hist_first) * tb.K * tb.ny * NX : nullptr;
  float* dpart_n = dpart ? dpart + (size_t)(n + 1) * 2 * tb.m : nullptr;
  __shared__ float2 Z[C::ROWS][C::PITCH];
  __shared__ float P[C::ROWS][NX];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x, r = tid / C::T, q = tid % C::T, y = y0 + r;
  const bool ok = y < ny;
  const size_t srow = ((size_t)k * ny + (ok ? y : 0)) * nh;
  if (ok)
    for (int kk = q; kk < NX; kk += C::T) Z[r][kk] = pack_two(SA + srow, SB + srow, kk, NX, nh);
  __syncthreads();
  fft<NX, C::T, +1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    const float ay_s = tb.ay[y];
    const size_t f = ((size_t)k * ny + y) * NX;
    const size_t fc = (size_t)y * NX;
    for (int x = q; x < NX; x += C::T) {
      const float2 d = Z[r][x];
      const float ax_s = tb.ax[x];
      const float nrx = ax_s * (ax_s * rx[f + x] - d.x);
      const float nry = ay_s * (ay_s * ry[f + x] - d.y);
      const float cc = c[fc + x];
      const float p = (cc * cc) * (nrx + nry);
      rx[f + x] = nrx;
      ry[f + x] = nry;
      if (hist) hist[f + x] = p;
      P[r][x] = p;
    }
  } else {
    for (int x = q; x < NX; x += C::T) P[r][x] = 0.f;
  }
  __syncthreads();
  if (dpart_n) gather_rows<NX, C::BLOCK>(tb, &P[0][0], y0, C::ROWS, dpart_n + (size_t)k * tb.nt * 2 * tb.m, tid);
  constexpr int T2 = 2 * C::T;
  const int pr = tid / T2, q2 = tid % T2;
  for (int x = q2; x < NX; x += T2) Z[pr][x] = make_float2(P[2 * pr][x], P[2 * pr + 1][x]);
  __syncthreads();
  fft<NX, T2, -1>(Z[pr], tb.tw_x, q2, true);
  for (int kk = q2; kk < nh; kk += T2) {
    float2 A, B;
    unpack_two(Z[pr], kk, NX, A, B);
    const int ya = y0 + 2 * pr;
    if (ya < ny) SA[((size_t)k * ny + ya) * nh + kk] = A;
    if (ya + 1 < ny) SA[((size_t)k * ny + ya + 1) * nh + kk] = B;
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_fwd_rho(Tables tb, const float* __restrict__ c, float* __restrict__ rx,
                                                 float* __restrict__ ry, float* __restrict__ hist_base,
                                                 float* __restrict__ dpart, float2* __restrict__ SA,
                                                 const float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  pat::k_fwd_rho_body<NX>(blockIdx.x, tb, c, rx, ry, hist_base, dpart, SA, SB, ctl);
}

// ===========================================================================
// Column pass: forward column transforms, spectral multiplier, inverse.
// ===========================================================================
enum ColMode : int {
  COL_GRAD1 = 0,  // A -> (A*Mx+, A*My+)       forward: spectra of D+ p
  COL_PAIRP = 1,  // (A, B) -> (A*Mx+, B*My+)  adjoint: D+ (a rho^)
  COL_PAIRM = 2,  // (A, B) -> (A*Mx-, B*My-)  forward: D- u
  COL_SUMM = 3,   // (A, B) -> A*Mx- + B*My-   adjoint: sum_j Dj- (as_j u^_j)
};

template <int NY, int MODE>
__device__ __forceinline__ void k_col_body(const int bid, const Tables& tb, float2* __restrict__ SA,
                                           float2* __restrict__ SB, float scale, int32_t* __restrict__ step,
                                           int32_t delta) {
  using C = ColCfg<NY>;
  if (step && bid == 0 && threadIdx.x == 0) *step += delta;   // first pass of a step
  __shared__ float2 A[C::TC][C::PITCH];
  __shared__ float2 B[C::TC][C::PITCH];
  const int K = tb.K, nh = tb.nh;
  const int k = bid % K, c0 = (bid / K) * C::TC;
  const int tid = threadIdx.x;
  const size_t base = (size_t)k * NY * nh;
  constexpr bool TWO_IN = MODE != COL_GRAD1;
  constexpr bool TWO_OUT = MODE != COL_SUMM;
  // coalesced tile load: consecutive lanes -> consecutive columns
  for (int i = tid; i < C::TC * NY; i += C::BLOCK) {
    const int col = i % C::TC, e = i / C::TC, cx = c0 + col;
    float2 a = make_float2(0.f, 0.f), b = a;
    if (cx < nh) {
      a = SA[base + (size_t)e * nh + cx];
      if (TWO_IN) b = SB[base + (size_t)e * nh + cx];
    }
    A[col][e] = a;
    if (TWO_IN) B[col][e] = b;
  }
  __syncthreads();
  const int tr = tid / C::T, q = tid % C::T;
  fft<NY, C::T, -1>(A[tr], tb.tw_y, q, true);
  if (TWO_IN) fft<NY, C::T, -1>(B[tr], tb.tw_y, q, true);
  // multiplier: column tr of this tile, rows e = q, q + T, ...
  {
    const int cx = c0 + tr;
    if (cx < nh) {
      const float2 exp_ = tb.ex_p[cx], exm = tb.ex_m[cx];
      for (int e = q; e < NY; e += C::T) {
        const float kap = tb.kappa[(size_t)cx * NY + e] * scale;
        const float2 a = A[tr][e];
        if (MODE == COL_GRAD1) {
          A[tr][e] = cscale(cmul(a, exp_), kap);
          B[tr][e] = cscale(cmul(a, tb.ey_p[e]), kap);
        } else if (MODE == COL_PAIRP) {
          A[tr][e] = cscale(cmul(a, exp_), kap);
          B[tr][e] = cscale(cmul(B[tr][e], tb.ey_p[e]), kap);
        } else if (MODE == COL_PAIRM) {
          A[tr][e] = cscale(cmul(a, exm), kap);
          B[tr][e] = cscale(cmul(B[tr][e], tb.ey_m[e]), kap);
        } else {
          A[tr][e] = cscale(cadd(cmul(a, exm), cmul(B[tr][e], tb.ey_m[e])), kap);
        }
      }
    }
  }
  __syncthreads();
  fft<NY, C::T, +1>(A[tr], tb.tw_y, q, true);
  if (TWO_OUT) fft<NY, C::T, +1>(B[tr], tb.tw_y, q, true);
  for (int i = tid; i < C::TC * NY; i += C::BLOCK) {
    const int col = i % C::TC, e = i / C::TC, cx = c0 + col;
    if (cx < nh) {
      SA[base + (size_t)e * nh + cx] = A[col][e];
      if (TWO_OUT) SB[base + (size_t)e * nh + cx] = B[col][e];
    }
  }
}

template <int NY, int MODE>
__global__ __launch_bounds__(ColCfg<NY>::BLOCK) void k_col(Tables tb, float2* __restrict__ SA,
                                                           float2* __restrict__ SB, float scale,
                                                           int32_t* __restrict__ step, int32_t delta) {
  pat::k_col_body<NY, MODE>(blockIdx.x, tb, SA, SB, scale, step, delta);
}

// ===========================================================================
// Adjoint passes (exact transpose of the forward recurrence, run backwards)
// ===========================================================================

// ph = S^T r^n + (inverse rows of the SUMM spectrum); rh += c^2 ph;
// gc += (2/c) p^n ph; spectra of (a_x rh_x, a_y rh_y); then rh <- a^2 rh.
template <int NX>
__device__ __forceinline__ void k_adj_rho_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                               const float* __restrict__ hist_base, const float* __restrict__ resid,
                                               float* __restrict__ rhx, float* __restrict__ rhy,
                                               float* __restrict__ gck, float2* __restrict__ SA,
                                               float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  using C = RowCfg<NX>;
  const int n = ctl->adj_n;
  const float* p_n = hist_base + (size_t)(n - ctl->hist_first) * tb.K * tb.ny * NX;
  const float* resid_n = resid + (size_t)n * tb.m;
  __shared__ float2 Z[C::ROWS][C::PITCH];
  __shared__ float PH[C::ROWS][NX];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x;
  constexpr int T2 = 2 * C::T;
  {
    const int pr = tid / T2, q2 = tid % T2;
    const int ya = y0 + 2 * pr, yb = ya + 1;
    if (ya < ny) {
      const float2* Ar = SA + ((size_t)k * ny + ya) * nh;
      if (yb < ny) {
        const float2* Br = SA + ((size_t)k * ny + yb) * nh;
        for (int kk = q2; kk < NX; kk += T2) Z[pr][kk] = pack_two(Ar, Br, kk, NX, nh);
      } else {
        for (int kk = q2; kk < NX; kk += T2) {
          float2 a = kk < nh ? Ar[kk] : cconj(Ar[NX - kk]);
          if (kk == 0 || 2 * kk == NX) a.y = 0.f;
          Z[pr][kk] = a;
        }
      }
    }
    __syncthreads();
    fft<NX, T2, +1>(Z[pr], tb.tw_x, q2, ya < ny);
    for (int x = q2; x < NX; x += T2) {
      const float2 t = Z[pr][x];
      PH[2 * pr][x] = ya < ny ? t.x : 0.f;
      PH[2 * pr + 1][x] = yb < ny ? t.y : 0.f;
    }
  }
  __syncthreads();
  scatter_rows<NX, C::BLOCK>(tb, &PH[0][0], y0, C::ROWS, resid_n + (size_t)k * tb.nt * tb.m, tid);
  __syncthreads();
  const int r = tid / C::T, q = tid % C::T, y = y0 + r;
  const bool ok = y < ny;
  if (ok) {
    const float ay_s = tb.ay[y], ay2_s = tb.ay2[y];
    const size_t f = ((size_t)k * ny + y) * NX;
    const size_t fc = (size_t)y * NX;
    for (int x = q; x < NX; x += C::T) {
      const float ph = PH[r][x];
      const float cc = c[fc + x];
      const float c2 = cc * cc;
      const float nrx = rhx[f + x] + c2 * ph;
      const float nry = rhy[f + x] + c2 * ph;
      gck[f + x] += (2.0f / cc) * p_n[f + x] * ph;
      Z[r][x] = make_float2(tb.ax[x] * nrx, ay_s * nry);
      rhx[f + x] = tb.ax2[x] * nrx;
      rhy[f + x] = ay2_s * nry;
    }
  }
  __syncthreads();
  fft<NX, C::T, -1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    const size_t srow = ((size_t)k * ny + y) * nh;
    for (int kk = q; kk < nh; kk += C::T) {
      float2 A, B;
      unpack_two(Z[r], kk, NX, A, B);
      SA[srow + kk] = A;
      SB[srow + kk] = B;
    }
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_adj_rho(Tables tb, const float* __restrict__ c,
                                                 const float* __restrict__ hist_base, const float* __restrict__ resid,
                                                 float* __restrict__ rhx, float* __restrict__ rhy,
                                                 float* __restrict__ gck, float2* __restrict__ SA,
                                                 float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  pat::k_adj_rho_body<NX>(blockIdx.x, tb, c, hist_base, resid, rhx, rhy, gck, SA, SB, ctl);
}

// uh <- as^2 uh + (inverse rows of the PAIRP spectra); spectra of (w_x uh_x, w_y uh_y)
// with w = as (next step) or as - as^2/2 (closing term, at adjoint step n = 1).
template <int NX>
__device__ __forceinline__ void k_adj_u_body(const int bid, const Tables& tb, float* __restrict__ uhx,
                                             float* __restrict__ uhy, float2* __restrict__ SA,
                                             float2* __restrict__ SB, const StepCtl* __restrict__ ctl) {
  using C = RowCfg<NX>;
  const int final_ = ctl->adj_n == 1;
  __shared__ float2 Z[C::ROWS][C::PITCH];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x, r = tid / C::T, q = tid % C::T, y = y0 + r;
  const bool ok = y < ny;
  const size_t srow = ((size_t)k * ny + (ok ? y : 0)) * nh;
  if (ok)
    for (int kk = q; kk < NX; kk += C::T) Z[r][kk] = pack_two(SA + srow, SB + srow, kk, NX, nh);
  __syncthreads();
  fft<NX, C::T, +1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    const float a2y = tb.asy2[y];
    const float wy = final_ ? tb.wfy[y] : tb.asy[y];
    const float* wxt = final_ ? tb.wfx : tb.asx;
    const size_t f = ((size_t)k * ny + y) * NX;
    for (int x = q; x < NX; x += C::T) {
      const float2 g = Z[r][x];
      const float nux = tb.asx2[x] * uhx[f + x] + g.x;
      const float nuy = a2y * uhy[f + x] + g.y;
      uhx[f + x] = nux;
      uhy[f + x] = nuy;
      Z[r][x] = make_float2(wxt[x] * nux, wy * nuy);
    }
  }
  __syncthreads();
  fft<NX, C::T, -1>(Z[r], tb.tw_x, q, ok);
  if (ok) {
    for (int kk = q; kk < nh; kk += C::T) {
      float2 A, B;
      unpack_two(Z[r], kk, NX, A, B);
      SA[srow + kk] = A;
      SB[srow + kk] = B;
    }
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_adj_u(Tables tb, float* __restrict__ uhx, float* __restrict__ uhy,
                                               float2* __restrict__ SA, float2* __restrict__ SB,
                                               const StepCtl* __restrict__ ctl) {
  pat::k_adj_u_body<NX>(blockIdx.x, tb, uhx, uhy, SA, SB, ctl);
}

// Closing terms: g_p0 = S^T r^0 + (inverse rows of SUMM spectrum of
// (as - as^2/2) uh) + (rh_x + rh_y) / (2 c^2);  gc += -(p0 / c^3)(rh_x + rh_y).
template <int NX>
__device__ __forceinline__ void k_adj_final_body(const int bid, const Tables& tb, const float* __restrict__ c,
                                                 const float* __restrict__ p0, const float* __restrict__ resid0,
                                                 const float* __restrict__ rhx, const float* __restrict__ rhy,
                                                 float* __restrict__ gck, float* __restrict__ gp0,
                                                 const float2* __restrict__ SA) {
  using C = RowCfg<NX>;
  __shared__ float2 Z[C::ROWS / 2][C::PITCH];
  __shared__ float PH[C::ROWS][NX];
  const int K = tb.K, ny = tb.ny, nh = tb.nh;
  const int k = bid % K, y0 = (bid / K) * C::ROWS;
  const int tid = threadIdx.x;
  constexpr int T2 = 2 * C::T;
  {
    const int pr = tid / T2, q2 = tid % T2;
    const int ya = y0 + 2 * pr, yb = ya + 1;
    if (ya < ny) {
      const float2* Ar = SA + ((size_t)k * ny + ya) * nh;
      if (yb < ny) {
        const float2* Br = SA + ((size_t)k * ny + yb) * nh;
        for (int kk = q2; kk < NX; kk += T2) Z[pr][kk] = pack_two(Ar, Br, kk, NX, nh);
      } else {
        for (int kk = q2; kk < NX; kk += T2) {
          float2 a = kk < nh ? Ar[kk] : cconj(Ar[NX - kk]);
          if (kk == 0 || 2 * kk == NX) a.y = 0.f;
          Z[pr][kk] = a;
        }
      }
    }
    __syncthreads();
    fft<NX, T2, +1>(Z[pr], tb.tw_x, q2, ya < ny);
    for (int x = q2; x < NX; x += T2) {
      const float2 t = Z[pr][x];
      PH[2 * pr][x] = ya < ny ? t.x : 0.f;
      PH[2 * pr + 1][x] = yb < ny ? t.y : 0.f;
    }
  }
  __syncthreads();
  scatter_rows<NX, C::BLOCK>(tb, &PH[0][0], y0, C::ROWS, resid0 + (size_t)k * tb.nt * tb.m, tid);
  __syncthreads();
  const int r = tid / C::T, q = tid % C::T, y = y0 + r;
  if (y < ny) {
    const size_t f = ((size_t)k * ny + y) * NX;
    const size_t fc = (size_t)y * NX;
    for (int x = q; x < NX; x += C::T) {
      const float cc = c[fc + x];
      const float rs = rhx[f + x] + rhy[f + x];
      gp0[f + x] = PH[r][x] + rs * (0.5f / (cc * cc));
      gck[f + x] += -(p0[f + x] / (cc * cc * cc)) * rs;
    }
  }
}

template <int NX>
__global__ __launch_bounds__(256) void k_adj_final(Tables tb, const float* __restrict__ c,
                                                   const float* __restrict__ p0, const float* __restrict__ resid0,
                                                   const float* __restrict__ rhx, const float* __restrict__ rhy,
                                                   float* __restrict__ gck, float* __restrict__ gp0,
                                                   const float2* __restrict__ SA) {
  pat::k_adj_final_body<NX>(blockIdx.x, tb, c, p0, resid0, rhx, rhy, gck, gp0, SA);
}

}  // namespace pat
