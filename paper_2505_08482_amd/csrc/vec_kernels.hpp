// vec_kernels.hpp — streaming vector kernels of the reconstruction (gfx950):
// misfit and deterministic float64 reductions, bound projection, multigrid
// prolongation, data time resampling, L-BFGS two-loop updates.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pat {

constexpr int RED_BLOCKS = 512;   // first-level partial sums (fixed: deterministic)
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// Sensor traces from the two per-row partials: data = part[.., 0, :] + part[.., 1, :]
__global__ void k_sensor_finalize(const float* __restrict__ part, float* __restrict__ data, int64_t rows, int m) {
  const int64_t n = rows * m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / m, s = i % m;
    data[i] = part[(r * 2) * m + s] + part[(r * 2 + 1) * m + s];
  }
}

// g_c = sum of the K partial slices gck[0..K)  (fixed order)
__global__ void k_reduce_k(const float* __restrict__ gck, float* __restrict__ gc, int K, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < K; ++k) s += gck[(int64_t)k * n + i];
    gc[i] = s;
  }
}

// Set fields of the step control block (mask bit 1: forward step, 2: adjoint
// step, 4: first history slot).  One thread.
__global__ void k_set_ctl(int32_t* __restrict__ ctl, int mask, int fwd_n, int adj_n, int hist_first) {
  if (mask & 1) ctl[0] = fwd_n;
  if (mask & 2) ctl[1] = adj_n;
  if (mask & 4) ctl[2] = hist_first;
}

__global__ void k_set_flag(int32_t* __restrict__ flag, int32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = v;
}

// flag = 1 if any x[i] is NaN or infinite (every writer writes the same value)
__global__ void k_flag_nonfinite(const float* __restrict__ x, int64_t n, int32_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(x[i]);
  if (bad) flag[0] = 1;
}

__global__ void k_fill_zero(float* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.f;
}

// resid = w_k^2 (data - y); partial sums of w_k^2 (data - y)^2 in float64
__global__ __launch_bounds__(RED_THREADS) void k_misfit(const float* __restrict__ data, const float* __restrict__ y,
                                                        const float* __restrict__ w, float* __restrict__ resid,
                                                        double* __restrict__ partial, int64_t per_k, int K) {
  __shared__ double sh[RED_THREADS];
  const int64_t n = per_k * K;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS) {
    const float wk = w[i / per_k];
    const float w2 = wk * wk;
    const float d = data[i] - y[i];
    resid[i] = w2 * d;
    acc += (double)w2 * (double)d * (double)d;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = factor * sum(partial[0..nb))
__global__ __launch_bounds__(RED_THREADS) void k_sum_partials(const double* __restrict__ partial, int nb,
                                                              double* __restrict__ out, double factor) {
  __shared__ double sh[RED_THREADS];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += RED_THREADS) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = factor * s;
}

__global__ __launch_bounds__(RED_THREADS) void k_dot_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                             int64_t n, double* __restrict__ partial) {
  __shared__ double sh[RED_THREADS];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS)
    acc += (double)a[i] * (double)b[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// eq. (10)-(11): x <- clamp(x - alpha d, lo, hi)
__global__ void k_project_update(int64_t n, float* __restrict__ x, const float* __restrict__ d, float alpha,
                                 const float* __restrict__ lo, const float* __restrict__ hi, float lo_s, float hi_s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float z = x[i] - alpha * d[i];
    const float L = lo ? lo[i] : lo_s;
    const float U = hi ? hi[i] : hi_s;
    x[i] = z <= L ? L : (z >= U ? U : z);
  }
}

// eq. (10)-(11): out = 0 on the active set (x on a bound with the gradient
// pointing out of the box), else v
__global__ void k_free_part(int64_t n, const float* __restrict__ x, const float* __restrict__ g,
                            const float* __restrict__ lo, const float* __restrict__ hi, const float* v,
                            float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float xi = x[i], gi = g[i];
    const bool active = (xi <= lo[i] && gi > 0.f) || (xi >= hi[i] && gi < 0.f);
    out[i] = active ? 0.f : v[i];
  }
}

// out = a x + b y (y may be null)
__global__ void k_axpby(int64_t n, float a, const float* x, float b, const float* y, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// out = x * s (element-wise)
__global__ void k_mul(int64_t n, const float* x, const float* __restrict__ s, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = x[i] * s[i];
}

// partial maxima of |x| (float64 slots of the dot-product scratch)
__global__ __launch_bounds__(RED_THREADS) void k_absmax_partial(const float* __restrict__ x, int64_t n,
                                                                double* __restrict__ partial) {
  __shared__ double sh[RED_THREADS];
  float m = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS)
    m = fmaxf(m, fabsf(x[i]));
  const int t = threadIdx.x;
  sh[t] = m;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(RED_THREADS) void k_max_partials(const double* __restrict__ partial, int nb,
                                                              double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += RED_THREADS) m = fmax(m, partial[i]);
  const int t = threadIdx.x;
  sh[t] = m;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  if (t == 0) *out = sh[0];
}

// Bilinear, cell-centred, same physical extent, clamped at the border.
__device__ __forceinline__ void axis_tap(int i, int nf, int nc, int& i0, int& i1, float& t) {
  double f = (i + 0.5) * ((double)nc / (double)nf) - 0.5;
  f = f < 0.0 ? 0.0 : (f > nc - 1.0 ? nc - 1.0 : f);
  int a = (int)floor(f);
  const int amax = nc >= 2 ? nc - 2 : 0;
  a = a > amax ? amax : a;
  i0 = a;
  i1 = a + 1 < nc ? a + 1 : nc - 1;
  t = (float)(f - a);
}

__global__ void k_prolong(int nchan, const float* __restrict__ coarse, int nyc, int nxc, float* __restrict__ fine,
                          int nyf, int nxf) {
  const int64_t n = (int64_t)nchan * nyf * nxf;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nxf);
    const int y = (int)((i / nxf) % nyf);
    const int64_t ch = i / ((int64_t)nxf * nyf);
    int x0, x1, y0, y1;
    float tx, ty;
    axis_tap(x, nxf, nxc, x0, x1, tx);
    axis_tap(y, nyf, nyc, y0, y1, ty);
    const float* cc = coarse + ch * (int64_t)nyc * nxc;
    const float r0 = cc[(int64_t)y0 * nxc + x0] * (1.f - tx) + cc[(int64_t)y0 * nxc + x1] * tx;
    const float r1 = cc[(int64_t)y1 * nxc + x0] * (1.f - tx) + cc[(int64_t)y1 * nxc + x1] * tx;
    fine[i] = r0 * (1.f - ty) + r1 * ty;
  }
}

// Bilinear at the same physical point: fine pixel i sits at (i + 1/2 - nf/2) dxf,
// i.e. at the fractional coarse index x / dxc + nc/2 - 1/2 (both grids centred
// on the origin); clamped to the coarse grid.
__device__ __forceinline__ void axis_tap_phys(int i, int nf, double dxf, int nc, double dxc, int& i0, int& i1,
                                              float& t) {
  double f = ((i + 0.5 - 0.5 * nf) * dxf) / dxc + 0.5 * nc - 0.5;
  f = f < 0.0 ? 0.0 : (f > nc - 1.0 ? nc - 1.0 : f);
  int a = (int)floor(f);
  const int amax = nc >= 2 ? nc - 2 : 0;
  a = a > amax ? amax : a;
  i0 = a;
  i1 = a + 1 < nc ? a + 1 : nc - 1;
  t = (float)(f - a);
}

__global__ void k_prolong_phys(int nchan, const float* __restrict__ coarse, int nyc, int nxc, double dxc,
                               float* __restrict__ fine, int nyf, int nxf, double dxf) {
  const int64_t n = (int64_t)nchan * nyf * nxf;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nxf);
    const int y = (int)((i / nxf) % nyf);
    const int64_t ch = i / ((int64_t)nxf * nyf);
    int x0, x1, y0, y1;
    float tx, ty;
    axis_tap_phys(x, nxf, dxf, nxc, dxc, x0, x1, tx);
    axis_tap_phys(y, nyf, dxf, nyc, dxc, y0, y1, ty);
    const float* cc = coarse + ch * (int64_t)nyc * nxc;
    const float r0 = cc[(int64_t)y0 * nxc + x0] * (1.f - tx) + cc[(int64_t)y0 * nxc + x1] * tx;
    const float r1 = cc[(int64_t)y1 * nxc + x0] * (1.f - tx) + cc[(int64_t)y1 * nxc + x1] * tx;
    fine[i] = r0 * (1.f - ty) + r1 * ty;
  }
}

__global__ void k_time_interp(int nlead, int nt_src, int m, const float* __restrict__ y, double dt_src,
                              float* __restrict__ out, int nt_dst, double dt_dst) {
  const int64_t n = (int64_t)nlead * nt_dst * m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i % m);
    const int t = (int)((i / m) % nt_dst);
    const int64_t l = i / ((int64_t)m * nt_dst);
    const double f = (t * dt_dst) / dt_src;
    const float* yl = y + l * (int64_t)nt_src * m;
    float v;
    if (f >= nt_src - 1) {
      v = yl[(int64_t)(nt_src - 1) * m + s];
    } else {
      const int a = (int)floor(f);
      const float w = (float)(f - a);
      v = yl[(int64_t)a * m + s] * (1.f - w) + yl[(int64_t)(a + 1) * m + s] * w;
    }
    out[i] = v;
  }
}

__global__ void k_copy(int64_t n, const float* __restrict__ src, float* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Two-loop helpers; sc = device scalars: ys[j] at j, lambda[j] at np + j,
// the latest dot at 2 np, y^T y at 2 np + 1.
// first loop:  lambda_j = (s_j^T q) / (y_j^T s_j);  q -= lambda_j y_j
__global__ void k_lbfgs_loop1(int64_t n, float* __restrict__ q, const float* __restrict__ yj, double* __restrict__ sc,
                              int np, int j) {
  const double lam = sc[2 * np] / sc[j];
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[np + j] = lam;
  const float fl = (float)lam;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    q[i] -= fl * yj[i];
}

// H^0 scaling: psi = (s^T y / y^T y) q  for the newest pair
__global__ void k_lbfgs_h0(int64_t n, float* __restrict__ q, const double* __restrict__ sc, int np) {
  const float g = (float)(sc[np - 1] / sc[2 * np + 1]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    q[i] *= g;
}

// second loop: beta = (y_j^T psi) / (y_j^T s_j);  psi += s_j (lambda_j - beta)
__global__ void k_lbfgs_loop2(int64_t n, float* __restrict__ psi, const float* __restrict__ sj,
                              const double* __restrict__ sc, int np, int j) {
  const double beta = sc[2 * np] / sc[j];
  const float coef = (float)(sc[np + j] - beta);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    psi[i] += coef * sj[i];
}

}  // namespace pat
