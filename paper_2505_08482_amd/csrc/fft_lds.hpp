// fft_lds.hpp — mixed-radix (2, 3, 4, 5, 7, 8) Stockham FFTs on LDS-resident
// data for gfx950.
//
// The k-space derivative of the forward and adjoint passes (D+- f =
// IFFT2[M+- FFT2 f]) needs one row pass and one column pass per 2-D
// transform; both passes call the 1-D transforms below on a block-wide set of
// transforms held in LDS.  A block of threads is split into groups of T
// threads, one group per transform; every stage reads R values per butterfly
// (stride N/R), applies twiddles w^(r*k), a radix-R DFT in registers, and
// writes them back in autosorted order, so the output is in natural order
// without a bit-reversal pass.  Twiddles come from a table exp(-2 pi i j / N),
// j < N, computed in float64 on the host and rounded once.
#pragma once
#include <hip/hip_runtime.h>

namespace pat {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by DIR * i  (DIR = -1: forward transform sign, +1: inverse)
template <int DIR>
__device__ __forceinline__ float2 mul_diri(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Radix-R DFTs in registers: y_s = sum_q a_q exp(DIR 2 pi i q s / R)
// ---------------------------------------------------------------------------
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <int DIR> struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    float2 t2 = cadd(a[1], a[3]), t3 = mul_diri<DIR>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <int DIR> struct Dft<8, DIR> {
  __device__ __forceinline__ static void run(float2* a) {
    constexpr float h = 0.70710678118654752440f;  // cos(pi/4)
    float2 e[4] = {a[0], a[2], a[4], a[6]};
    float2 o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, DIR>::run(e);
    Dft<4, DIR>::run(o);
    // w8^1 = h (1 + DIR i), w8^2 = DIR i, w8^3 = h (-1 + DIR i)
    float2 o1 = cscale(cadd(o[1], mul_diri<DIR>(o[1])), h);
    float2 o2 = mul_diri<DIR>(o[2]);
    float2 o3 = cscale(csub(mul_diri<DIR>(o[3]), o[3]), h);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
};

// cos / sin of 2 pi m / R for the odd radices
template <int R> struct Trig;
template <> struct Trig<3> {
  __device__ __forceinline__ static float c(int m) { return m == 0 ? 1.0f : -0.5f; }
  __device__ __forceinline__ static float s(int m) {
    return m == 0 ? 0.0f : (m == 1 ? 0.86602540378443864676f : -0.86602540378443864676f);
  }
};
template <> struct Trig<5> {
  __device__ __forceinline__ static float c(int m) {
    switch (m) {
      case 0: return 1.0f;
      case 1: case 4: return 0.30901699437494742410f;
      default: return -0.80901699437494742410f;
    }
  }
  __device__ __forceinline__ static float s(int m) {
    switch (m) {
      case 0: return 0.0f;
      case 1: return 0.95105651629515357212f;
      case 2: return 0.58778525229247312917f;
      case 3: return -0.58778525229247312917f;
      default: return -0.95105651629515357212f;
    }
  }
};
template <> struct Trig<7> {
  __device__ __forceinline__ static float c(int m) {
    switch (m) {
      case 0: return 1.0f;
      case 1: case 6: return 0.62348980185873353053f;
      case 2: case 5: return -0.22252093395631440429f;
      default: return -0.90096886790241912624f;
    }
  }
  __device__ __forceinline__ static float s(int m) {
    switch (m) {
      case 0: return 0.0f;
      case 1: return 0.78183148246802980871f;
      case 2: return 0.97492791218182360702f;
      case 3: return 0.43388373911755812048f;
      case 4: return -0.43388373911755812048f;
      case 5: return -0.97492791218182360702f;
      default: return -0.78183148246802980871f;
    }
  }
};

// odd radix: pair a_q with a_{R-q}; a_q w^{qs} + a_{R-q} w^{-qs}
//   = (a_q + a_{R-q}) cos(theta) + DIR i (a_q - a_{R-q}) sin(theta)
template <int R, int DIR> struct DftOdd {
  __device__ __forceinline__ static void run(float2* a) {
    float2 y[R];
#pragma unroll
    for (int s = 0; s < R; ++s) y[s] = a[0];
#pragma unroll
    for (int q = 1; q <= (R - 1) / 2; ++q) {
      float2 sm = cadd(a[q], a[R - q]);
      float2 df = mul_diri<DIR>(csub(a[q], a[R - q]));
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int m = (q * s) % R;
        const float cc = Trig<R>::c(m), ss = Trig<R>::s(m);
        y[s].x += sm.x * cc + df.x * ss;
        y[s].y += sm.y * cc + df.y * ss;
      }
    }
#pragma unroll
    for (int s = 0; s < R; ++s) a[s] = y[s];
  }
};
template <int DIR> struct Dft<3, DIR> : DftOdd<3, DIR> {};
template <int DIR> struct Dft<5, DIR> : DftOdd<5, DIR> {};
template <int DIR> struct Dft<7, DIR> : DftOdd<7, DIR> {};

// ---------------------------------------------------------------------------
// Radix plans (product of the radices = N)
// ---------------------------------------------------------------------------
template <int... Rs> struct RList {};

template <int N> struct Plan;
template <> struct Plan<32>  { using L = RList<8, 4>; };
template <> struct Plan<36>  { using L = RList<4, 3, 3>; };
template <> struct Plan<40>  { using L = RList<8, 5>; };
template <> struct Plan<48>  { using L = RList<4, 4, 3>; };
template <> struct Plan<64>  { using L = RList<8, 8>; };
template <> struct Plan<81>  { using L = RList<3, 3, 3, 3>; };
template <> struct Plan<84>  { using L = RList<4, 3, 7>; };
template <> struct Plan<96>  { using L = RList<8, 4, 3>; };
template <> struct Plan<125> { using L = RList<5, 5, 5>; };
template <> struct Plan<128> { using L = RList<8, 4, 4>; };
template <> struct Plan<160> { using L = RList<8, 4, 5>; };
template <> struct Plan<175> { using L = RList<7, 5, 5>; };
template <> struct Plan<192> { using L = RList<8, 8, 3>; };
template <> struct Plan<243> { using L = RList<3, 3, 3, 3, 3>; };
template <> struct Plan<256> { using L = RList<8, 8, 4>; };
template <> struct Plan<375> { using L = RList<5, 5, 5, 3>; };
template <> struct Plan<384> { using L = RList<8, 8, 3, 2>; };
template <> struct Plan<512> { using L = RList<8, 8, 8>; };
template <> struct Plan<768> { using L = RList<8, 8, 4, 3>; };

// Threads per transform: a power of two near N/8, between 8 and 64.
template <int N> struct Threads {
  static constexpr int v = N >= 512 ? 64 : (N >= 256 ? 32 : (N >= 96 ? 16 : 8));
};

// One Stockham stage on transform `x` (contiguous N complex in LDS).
// All threads of the block must call it (it contains two barriers).
template <int N, int R, int NS, int T, int DIR>
__device__ __forceinline__ void stage(float2* x, const float2* __restrict__ tw, int q, bool active) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + T - 1) / T;
  float2 v[PER][R];
  if (active) {
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int j = q + b * T;
      if ((NB % T) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = x[j + r * NB];
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int j = q + b * T;
      if ((NB % T) == 0 || j < NB) {
        const int k = j % NS;
        if (NS > 1) {
          constexpr int TS = N / (NS * R);
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * TS];
            if (DIR > 0) w.y = -w.y;
            v[b][r] = cmul(v[b][r], w);
          }
        }
        Dft<R, DIR>::run(v[b]);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) x[base + r * NS] = v[b][r];
      }
    }
  }
  __syncthreads();
}

template <int N, int T, int DIR, int NS, typename L> struct Stages;
template <int N, int T, int DIR, int NS> struct Stages<N, T, DIR, NS, RList<>> {
  __device__ __forceinline__ static void run(float2*, const float2*, int, bool) {}
};
template <int N, int T, int DIR, int NS, int R, int... Rest>
struct Stages<N, T, DIR, NS, RList<R, Rest...>> {
  __device__ __forceinline__ static void run(float2* x, const float2* tw, int q, bool active) {
    stage<N, R, NS, T, DIR>(x, tw, q, active);
    Stages<N, T, DIR, NS * R, RList<Rest...>>::run(x, tw, q, active);
  }
};

// In-place N-point transform of the LDS array x[0..N) by the T threads of a
// group (q = thread index within the group).  DIR = -1 forward (no scaling),
// +1 inverse (no 1/N scaling).  Every thread of the block must call it.
template <int N, int T, int DIR>
__device__ __forceinline__ void fft(float2* x, const float2* __restrict__ tw, int q, bool active) {
  Stages<N, T, DIR, 1, typename Plan<N>::L>::run(x, tw, q, active);
}

}  // namespace pat
