// prior_kernels.hpp — Ornstein-Uhlenbeck prior of eq. (4) (Sec. 4.1.2) on gfx950.
//
// The prior precision Xi^{-1}, Xi_ij = exp(-|r_i - r_j| / tau) over the masked
// pixels of a box of nby x nbx pixels, is applied by conjugate gradients on
// Xi.  Products Xi v are exact: v is zero-padded into an L x L periodic grid
// (L >= 2 nb - 1), convolved with the kernel laid out on the wrapped offsets by
// FFTs (row pass, column pass with the spectral multiply, inverse row pass),
// and cropped.  The preconditioner is the same circulant with the reciprocal
// spectrum (floored), which is symmetric positive definite.
//
// Work arrays of nvec right-hand sides: box vectors [nvec][nby][nbx] (zero
// outside the mask) and complex row spectra [nvec][nby][L].  Reductions run in
// float64 with a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace pat {
namespace ou {

constexpr int DOT_BLOCKS = 64;   // partial sums per right-hand side
constexpr int DOT_THREADS = 256;

// Row pass: rows y < nby of every vector, zero-padded to L, forward FFT along x.
template <int L>
__global__ __launch_bounds__(256) void k_rows_fwd(const float* __restrict__ v, int nvec, int nby, int nbx,
                                                  const float2* __restrict__ tw, float2* __restrict__ W) {
  constexpr int T = Threads<L>::v, ROWS = 256 / T;
  __shared__ float2 X[ROWS][L + 1];
  const int tid = threadIdx.x, r = tid / T, q = tid % T;
  const int grow = blockIdx.x * ROWS + r;   // over nvec * nby rows
  const bool active = grow < nvec * nby;
  const int vec = active ? grow / nby : 0, y = active ? grow % nby : 0;
  const float* src = v + ((size_t)vec * nby + y) * nbx;
  for (int x = q; x < L; x += T) X[r][x] = make_float2(active && x < nbx ? src[x] : 0.f, 0.f);
  __syncthreads();
  fft<L, T, -1>(X[r], tw, q, active);
  if (active) {
    float2* dst = W + ((size_t)vec * nby + y) * L;
    for (int x = q; x < L; x += T) dst[x] = X[r][x];
  }
}

// Column pass: column x of every vector (rows >= nby are zero), forward FFT
// along y, multiply by the real spectrum S[ky][kx], inverse FFT, keep rows < nby.
template <int L>
__global__ __launch_bounds__(256) void k_cols(float2* __restrict__ W, int nvec, int nby,
                                              const float* __restrict__ S, const float2* __restrict__ tw) {
  constexpr int T = Threads<L>::v, TC = 256 / T;
  __shared__ float2 X[TC][L + 1];
  const int tid = threadIdx.x, c = tid % TC, q = tid / TC;   // adjacent lanes: adjacent columns
  const int gcol = blockIdx.x * TC + c;                      // over nvec * L columns
  const bool active = gcol < nvec * L;
  const int vec = active ? gcol / L : 0, x = active ? gcol % L : 0;
  float2* col = W + (size_t)vec * nby * L + x;
  for (int y = q; y < L; y += T) X[c][y] = active && y < nby ? col[(size_t)y * L] : make_float2(0.f, 0.f);
  __syncthreads();
  fft<L, T, -1>(X[c], tw, q, active);
  if (active)
    for (int y = q; y < L; y += T) X[c][y] = cscale(X[c][y], S[(size_t)y * L + x]);
  __syncthreads();
  fft<L, T, +1>(X[c], tw, q, active);
  if (active)
    for (int y = q; y < nby; y += T) col[(size_t)y * L] = X[c][y];
}

// Inverse row pass: rows y < nby, inverse FFT along x, crop to the box, scale,
// zero outside the mask.
template <int L>
__global__ __launch_bounds__(256) void k_rows_inv(const float2* __restrict__ W, int nvec, int nby, int nbx,
                                                  const uint8_t* __restrict__ mask, const float2* __restrict__ tw,
                                                  float scale, float* __restrict__ out) {
  constexpr int T = Threads<L>::v, ROWS = 256 / T;
  __shared__ float2 X[ROWS][L + 1];
  const int tid = threadIdx.x, r = tid / T, q = tid % T;
  const int grow = blockIdx.x * ROWS + r;
  const bool active = grow < nvec * nby;
  const int vec = active ? grow / nby : 0, y = active ? grow % nby : 0;
  const float2* src = W + ((size_t)vec * nby + y) * L;
  for (int x = q; x < L; x += T) X[r][x] = active ? src[x] : make_float2(0.f, 0.f);
  __syncthreads();
  fft<L, T, +1>(X[r], tw, q, active);
  if (active) {
    float* dst = out + ((size_t)vec * nby + y) * nbx;
    const uint8_t* mr = mask + (size_t)y * nbx;
    for (int x = q; x < nbx; x += T) dst[x] = mr[x] ? X[r][x].x * scale : 0.f;
  }
}

// Box <-> grid: gather the box [nby][nbx] at (oy, ox) of every grid vector
// [nvec][ny][nx] (masked), and scatter back (zero outside the mask).
__global__ void k_gather(const float* __restrict__ g, int nvec, int ny, int nx, int oy, int ox, int nby, int nbx,
                         const uint8_t* __restrict__ mask, float eta_scale, const float* __restrict__ eta,
                         float* __restrict__ b) {
  const int64_t n = (int64_t)nvec * nby * nbx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nbx);
    const int y = (int)((i / nbx) % nby);
    const int vec = (int)(i / ((int64_t)nbx * nby));
    const float val = g[((int64_t)vec * ny + oy + y) * nx + ox + x] - (eta ? eta_scale * eta[vec] : 0.f);
    b[i] = mask[(int64_t)y * nbx + x] ? val : 0.f;
  }
}

__global__ void k_scatter(const float* __restrict__ b, int nvec, int ny, int nx, int oy, int ox, int nby, int nbx,
                          const float* __restrict__ wvec, float* __restrict__ g) {
  const int64_t n = (int64_t)nvec * ny * nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx) - ox;
    const int y = (int)((i / nx) % ny) - oy;
    const int vec = (int)(i / ((int64_t)nx * ny));
    const bool in = x >= 0 && x < nbx && y >= 0 && y < nby;
    g[i] = in ? b[((int64_t)vec * nby + y) * nbx + x] * (wvec ? wvec[vec] : 1.f) : 0.f;
  }
}

// Per-vector dot products: partial[vec][blk] over the n elements of vector vec.
__global__ __launch_bounds__(DOT_THREADS) void k_dots(const float* __restrict__ a, const float* __restrict__ b,
                                                      int64_t n, double* __restrict__ partial) {
  __shared__ double sh[DOT_THREADS];
  const int vec = blockIdx.y;
  const float* av = a + (int64_t)vec * n;
  const float* bv = b + (int64_t)vec * n;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)DOT_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * DOT_THREADS)
    acc += (double)av[i] * (double)bv[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = DOT_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)vec * DOT_BLOCKS + blockIdx.x] = sh[0];
}

// Sum the partials of each vector (fixed order) into out[vec].
__global__ void k_dot_final(const double* __restrict__ partial, int nvec, double* __restrict__ out) {
  const int vec = blockIdx.x * blockDim.x + threadIdx.x;
  if (vec >= nvec) return;
  double s = 0.0;
  for (int b = 0; b < DOT_BLOCKS; ++b) s += partial[(int64_t)vec * DOT_BLOCKS + b];
  out[vec] = s;
}

// CG scalars per vector, sc = [rz, pAp, alpha, beta, rz_new] x nvec (struct of arrays).
// alpha = rz / pAp (0 when pAp = 0: the vector has converged exactly)
__global__ void k_cg_alpha(double* __restrict__ sc, int nvec) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  const double pAp = sc[nvec + v];
  sc[2 * nvec + v] = pAp > 0.0 ? sc[v] / pAp : 0.0;
}
// beta = rz_new / rz; rz <- rz_new
__global__ void k_cg_beta(double* __restrict__ sc, int nvec) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  const double rz = sc[v], rzn = sc[4 * nvec + v];
  sc[3 * nvec + v] = rz > 0.0 ? rzn / rz : 0.0;
  sc[v] = rzn;
}
// x += alpha p; r -= alpha Ap (per vector alpha)
__global__ void k_cg_update(int nvec, int64_t n, const double* __restrict__ sc, const float* __restrict__ p,
                            const float* __restrict__ Ap, float* __restrict__ x, float* __restrict__ r) {
  const int64_t tot = (int64_t)nvec * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const float a = (float)sc[2 * nvec + i / n];
    x[i] += a * p[i];
    r[i] -= a * Ap[i];
  }
}
// p = z + beta p
__global__ void k_cg_dir(int nvec, int64_t n, const double* __restrict__ sc, const float* __restrict__ z,
                         float* __restrict__ p) {
  const int64_t tot = (int64_t)nvec * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + (float)sc[3 * nvec + i / n] * p[i];
}

}  // namespace ou
}  // namespace pat
