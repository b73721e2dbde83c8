// pat_api.hip — C ABI (include/pat.h): plans, workspace layout and the time
// loops of the forward solve and of its adjoint, on top of the fused passes.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <utility>
#include <new>
#include <vector>

#include "../../include/pat.h"
#include "vec_kernels.hpp"
#include "wave_kernels.hpp"
#include "fast_kernels.hpp"
#include "prior_kernels.hpp"
#include "batch_slot.hpp"

using namespace pat;

namespace {

constexpr int kSupported[] = {32, 36, 40, 48, 64, 81, 84, 96, 125, 128, 160, 175, 192, 243, 256, 375, 384, 512, 768};

bool supported(int n) {
  for (int s : kSupported)
    if (s == n) return true;
  return false;
}

#define PAT_SIZE_CASES(X)                                                                                  \
  X(32) X(36) X(40) X(48) X(64) X(81) X(84) X(96) X(125) X(128) X(160) X(175) X(192) X(243) X(256) X(375) \
  X(384) X(512) X(768)

#define PAT_FAST_CASES(X) X(32) X(64) X(128) X(256) X(512)

bool fast_size(int n) { return n == 32 || n == 64 || n == 128 || n == 256 || n == 512; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int grid_blocks(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 8192) b = 8192;
  return (int)std::max<int64_t>(b, 1);
}

// ---------------------------------------------------------------------------
// Launch timing (pat_trace_*): sampled event pairs per pass kind
// ---------------------------------------------------------------------------
constexpr int kTraceCap = 1024;
struct Trace {
  bool on = false;
  int every = 1;
  bool created = false;
  int64_t seen[PAT_PASS_KINDS] = {};
  int used[PAT_PASS_KINDS] = {};
  std::vector<hipEvent_t> ev;   // [kind][cap][2]
};
Trace g_trace;

// A sampled launch gets the event pair of its slot as the start / stop events
// of its own dispatch (hipExtLaunchKernelGGL), so the elapsed time between them
// is the kernel's execution alone, without the queue's dispatch latency.
thread_local hipEvent_t g_launch_ev[2] = {nullptr, nullptr};

struct TraceScope {
  TraceScope(int kind, hipStream_t) {
    g_launch_ev[0] = g_launch_ev[1] = nullptr;
    if (!g_trace.on) return;
    const int64_t s = g_trace.seen[kind]++;
    if (s % g_trace.every != 0 || g_trace.used[kind] >= kTraceCap) return;
    const int slot = g_trace.used[kind]++;
    g_launch_ev[0] = g_trace.ev[((size_t)kind * kTraceCap + slot) * 2];
    g_launch_ev[1] = g_trace.ev[((size_t)kind * kTraceCap + slot) * 2 + 1];
  }
  ~TraceScope() { g_launch_ev[0] = g_launch_ev[1] = nullptr; }
};

// Launch a pass kernel; the launch under a sampled TraceScope carries its events.
#define PAT_LAUNCH(KERN, GRID, BLOCK, SHM, ST, ...)                                                   \
  do {                                                                                                \
    if (g_launch_ev[0]) {                                                                             \
      hipExtLaunchKernelGGL(KERN, GRID, BLOCK, SHM, ST, g_launch_ev[0], g_launch_ev[1], 0, __VA_ARGS__); \
      g_launch_ev[0] = g_launch_ev[1] = nullptr;                                                      \
    } else {                                                                                          \
      hipLaunchKernelGGL(KERN, GRID, BLOCK, SHM, ST, __VA_ARGS__);                                    \
    }                                                                                                 \
  } while (0)

}  // namespace

struct pat_plan {
  pat_grid g;
  int K = 0, m = 0, nh = 0;
  bool fast = false;         // register-resident power-of-two passes (folded spectra)
  int col_tile = 0;          // column-pass tile width: 0 = default for the length, or 8
  int col_order = 0;         // column pass: 0 two transforms per thread together, 1 one after the other,
                             // 2 the two arrays on two halves of the block
  bool check_finite = false; // check mode: scan outputs, return PAT_ENONFINITE on NaN / Inf
  int32_t* flag = nullptr;   // device flag of the check mode
  int kb = 1;                // datasets per block of the fast adjoint density / closing passes
  int gsl = 0;               // g_c partial slices: ceil(K / kb) (fast), K (generic)
  int nhs = 0;               // spectrum row pitch: nx/2 (fast, folded) or nx/2 + 1
  void* dev = nullptr;       // one allocation for every table
  Tables tb{};
  double* red = nullptr;     // RED_BLOCKS partial sums (misfit)
  // bookkeeping of the last recording forward (for pat_adjoint_gradient)
  bool recorded = false;
  const void* rec_ws = nullptr;
  const float* rec_c = nullptr;
  const float* rec_p0 = nullptr;
  int rec_ckpt = 0;
  // captured step-chunk graphs (replayed while their launch arguments repeat)
  struct GraphEntry {
    uint64_t key[14];
    hipGraphExec_t exec;
    uint64_t last_use;
    hipEvent_t done;      // recorded after each launch: waited for before the graph is destroyed
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t cap = nullptr;   // private stream for capture (the caller's may be the null stream)
};

namespace {

struct Layout {
  size_t F = 0, Sp = 0;           // bytes of one [K][ny][nx] field / one [K][ny][nh] spectrum
  size_t ctl;                     // StepCtl
  size_t ux, uy, rx, ry;          // forward state
  size_t uhx, uhy, rhx, rhy, gck; // adjoint state
  size_t SA, SB, SC, SD;          // spectra (forward pair, adjoint pair)
  size_t dpart;                   // [K][nt][2][m]
  size_t hist;                    // store-all history [nt] fields, or the segment buffer [s] fields
  size_t ckpt;                    // checkpoints: ncks * (4 fields + 1 spectrum)
  int ncks = 0, s = 0;
  size_t total = 0;
};

Layout make_layout(const pat_plan* p, int ckpt_every) {
  Layout L;
  const pat_grid& g = p->g;
  L.F = (size_t)p->K * g.ny * g.nx * sizeof(float);
  L.Sp = (size_t)p->K * g.ny * p->nhs * sizeof(float2);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += align256(b);
    return o;
  };
  L.ctl = take(sizeof(StepCtl));
  L.ux = take(L.F); L.uy = take(L.F); L.rx = take(L.F); L.ry = take(L.F);
  L.uhx = take(L.F); L.uhy = take(L.F); L.rhx = take(L.F); L.rhy = take(L.F); L.gck = take(L.F);
  L.SA = take(L.Sp); L.SB = take(L.Sp); L.SC = take(L.Sp); L.SD = take(L.Sp);
  L.dpart = take((size_t)p->K * g.nt * 2 * p->m * sizeof(float));
  L.s = ckpt_every;
  if (ckpt_every <= 0) {
    L.hist = take(L.F * (size_t)g.nt);
    L.ckpt = off;
    L.ncks = 0;
  } else {
    L.hist = take(L.F * (size_t)ckpt_every);
    // checkpoints at n = s, 2s, ... < nt - 1
    L.ncks = g.nt >= 2 ? (g.nt - 2) / ckpt_every : 0;
    L.ckpt = take((4 * align256(L.F) + align256(L.Sp)) * (size_t)L.ncks);
  }
  L.total = off;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int last_error() { return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP; }

// ----------------------------------------------------------------------------
// Launchers (template dispatch on the transform length)
// ----------------------------------------------------------------------------
template <int NX>
int rows_blocks(const pat_plan* p) {
  return p->K * ((p->g.ny + RowCfg<NX>::ROWS - 1) / RowCfg<NX>::ROWS);
}
template <int NY>
int cols_blocks(const pat_plan* p) {
  return p->K * ((p->nh + ColCfg<NY>::TC - 1) / ColCfg<NY>::TC);
}
template <int NX>
int frows_blocks(const pat_plan* p) {
  return p->K * ((p->g.ny + fast::RowF<NX>::ROWS - 1) / fast::RowF<NX>::ROWS);
}
// adjoint density / closing passes: one block per (dataset group, ROWS rows)
template <int NX>
int fadj_blocks(const pat_plan* p) {
  return p->gsl * ((p->g.ny + fast::RowF<NX>::ROWS - 1) / fast::RowF<NX>::ROWS);
}
int fcols_blocks(const pat_plan* p, int TC) {
  return p->K * ((p->g.nx / 2 + TC - 1) / TC);
}

int launch_fwd_init(const pat_plan* p, hipStream_t st, const float* c, const float* p0, float* rx, float* ry,
                    float* hist0, float* dpart, float2* SA) {
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                              \
  case N:                                                                                                 \
    hipLaunchKernelGGL(fast::k_fwd_init<N>, dim3(frows_blocks<N>(p)), dim3(64), 0, st, p->tb, c, p0, rx, ry, \
                       hist0, dpart, SA);                                                                 \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                           \
  case N:                                                                                              \
    hipLaunchKernelGGL(k_fwd_init<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, c, p0, rx, ry, \
                       hist0, dpart, SA);                                                              \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int launch_fwd_u(const pat_plan* p, hipStream_t st, float* ux, float* uy, float2* SA, float2* SB,
                 const StepCtl* ctl) {
  TraceScope ts(PAT_PASS_FWD_ROW_U, st);
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                                \
  case N:                                                                                                   \
    PAT_LAUNCH(fast::k_fwd_u<N>, dim3(frows_blocks<N>(p)), dim3(64), 0, st, p->tb, ux, uy, SA, SB, ctl); \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                                \
  case N:                                                                                                   \
    PAT_LAUNCH(k_fwd_u<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, ux, uy, SA, SB, ctl); \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int launch_fwd_rho(const pat_plan* p, hipStream_t st, const float* c, float* rx, float* ry, float* hist_base,
                   float* dpart, float2* SA, float2* SB, const StepCtl* ctl) {
  TraceScope ts(PAT_PASS_FWD_ROW_RHO, st);
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    PAT_LAUNCH(fast::k_fwd_rho<N>, dim3(frows_blocks<N>(p)), dim3(64), 0, st, p->tb, c, rx, ry,       \
                       hist_base, dpart, SA, SB, ctl);                                                        \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    PAT_LAUNCH(k_fwd_rho<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, c, rx, ry, hist_base, \
                       dpart, SA, SB, ctl);                                                                   \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

// step != nullptr: this launch is the first pass of a step and advances *step by delta
template <int MODE>
int launch_col(const pat_plan* p, hipStream_t st, float2* SA, float2* SB, float scale, int32_t* step,
               int32_t delta) {
  constexpr int kind = MODE == COL_GRAD1 ? PAT_PASS_FWD_COL_GRAD
                       : MODE == COL_PAIRM ? PAT_PASS_FWD_COL_DIV
                       : MODE == COL_SUMM  ? PAT_PASS_ADJ_COL_SUMM
                                           : PAT_PASS_ADJ_COL_GRAD;
  TraceScope ts(kind, st);
  if (p->fast) {
    switch (p->g.ny) {
#define X(N)                                                                                                   \
  case N:                                                                                                      \
    if (p->col_order == 2)                                                                                      \
      PAT_LAUNCH((fast::k_cols<N, MODE>), dim3(fcols_blocks(p, fast::Cfg<N>::TC)),                              \
                 dim3(2 * fast::Cfg<N>::TC * fast::Cfg<N>::T), 0, st, p->tb, SA, SB, scale, step, delta);      \
    else if (p->col_tile == 8 && p->col_order == 1)                                                             \
      PAT_LAUNCH((fast::k_col<N, MODE, 8, true>), dim3(fcols_blocks(p, 8)), dim3(8 * fast::Cfg<N>::T), 0, st, \
                 p->tb, SA, SB, scale, step, delta);                                                             \
    else if (p->col_tile == 8)                                                                                  \
      PAT_LAUNCH((fast::k_col<N, MODE, 8>), dim3(fcols_blocks(p, 8)), dim3(8 * fast::Cfg<N>::T), 0, st,        \
                 p->tb, SA, SB, scale, step, delta);                                                             \
    else if (p->col_order == 1)                                                                                 \
      PAT_LAUNCH((fast::k_col<N, MODE, fast::Cfg<N>::TC, true>), dim3(fcols_blocks(p, fast::Cfg<N>::TC)),     \
                 dim3(fast::Cfg<N>::TC * fast::Cfg<N>::T), 0, st, p->tb, SA, SB, scale, step, delta);          \
    else                                                                                                        \
      PAT_LAUNCH((fast::k_col<N, MODE>), dim3(fcols_blocks(p, fast::Cfg<N>::TC)),                               \
                 dim3(fast::Cfg<N>::TC * fast::Cfg<N>::T), 0, st, p->tb, SA, SB, scale, step, delta);          \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.ny) {
#define X(N)                                                                                                 \
  case N:                                                                                                    \
    PAT_LAUNCH((k_col<N, MODE>), dim3(cols_blocks<N>(p)), dim3(ColCfg<N>::BLOCK), 0, st, p->tb, SA, \
                       SB, scale, step, delta);                                                              \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int launch_adj_rho(const pat_plan* p, hipStream_t st, const float* c, const float* hist_base, const float* resid,
                   float* rhx, float* rhy, float* gck, float2* SA, float2* SB, const StepCtl* ctl) {
  TraceScope ts(PAT_PASS_ADJ_ROW_RHO, st);
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                                   \
  case N:                                                                                                      \
    switch (p->kb) {                                                                                           \
      case 8: PAT_LAUNCH((fast::k_adj_rho<N, 8>), dim3(fadj_blocks<N>(p)), dim3(512), 0, st, p->tb, c,  \
                                 hist_base, resid, rhx, rhy, gck, SA, SB, ctl); break;                          \
      case 4: PAT_LAUNCH((fast::k_adj_rho<N, 4>), dim3(fadj_blocks<N>(p)), dim3(256), 0, st, p->tb, c,  \
                                 hist_base, resid, rhx, rhy, gck, SA, SB, ctl); break;                          \
      case 2: PAT_LAUNCH((fast::k_adj_rho<N, 2>), dim3(fadj_blocks<N>(p)), dim3(128), 0, st, p->tb, c,  \
                                 hist_base, resid, rhx, rhy, gck, SA, SB, ctl); break;                          \
      default: PAT_LAUNCH((fast::k_adj_rho<N, 1>), dim3(fadj_blocks<N>(p)), dim3(64), 0, st, p->tb, c,  \
                                  hist_base, resid, rhx, rhy, gck, SA, SB, ctl); break;                         \
    }                                                                                                          \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                                    \
  case N:                                                                                                       \
    PAT_LAUNCH(k_adj_rho<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, c, hist_base, resid, rhx, \
                       rhy, gck, SA, SB, ctl);                                                                  \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int launch_adj_u(const pat_plan* p, hipStream_t st, float* uhx, float* uhy, float2* SA, float2* SB,
                 const StepCtl* ctl) {
  TraceScope ts(PAT_PASS_ADJ_ROW_U, st);
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                                    \
  case N:                                                                                                       \
    PAT_LAUNCH(fast::k_adj_u<N>, dim3(frows_blocks<N>(p)), dim3(64), 0, st, p->tb, uhx, uhy, SA, SB, ctl); \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    PAT_LAUNCH(k_adj_u<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, uhx, uhy, SA, SB, ctl); \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int launch_adj_final(const pat_plan* p, hipStream_t st, const float* c, const float* p0, const float* resid0,
                     const float* rhx, const float* rhy, float* gck, float* gp0, const float2* SA) {
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    switch (p->kb) {                                                                                          \
      case 8: hipLaunchKernelGGL((fast::k_adj_final<N, 8>), dim3(fadj_blocks<N>(p)), dim3(512), 0, st, p->tb,  \
                                 c, p0, resid0, rhx, rhy, gck, gp0, SA); break;                                \
      case 4: hipLaunchKernelGGL((fast::k_adj_final<N, 4>), dim3(fadj_blocks<N>(p)), dim3(256), 0, st, p->tb,  \
                                 c, p0, resid0, rhx, rhy, gck, gp0, SA); break;                                \
      case 2: hipLaunchKernelGGL((fast::k_adj_final<N, 2>), dim3(fadj_blocks<N>(p)), dim3(128), 0, st, p->tb,  \
                                 c, p0, resid0, rhx, rhy, gck, gp0, SA); break;                                \
      default: hipLaunchKernelGGL((fast::k_adj_final<N, 1>), dim3(fadj_blocks<N>(p)), dim3(64), 0, st, p->tb,  \
                                  c, p0, resid0, rhx, rhy, gck, gp0, SA); break;                               \
    }                                                                                                         \
    return last_error();
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
  }
  switch (p->g.nx) {
#define X(N)                                                                                               \
  case N:                                                                                                  \
    hipLaunchKernelGGL(k_adj_final<N>, dim3(rows_blocks<N>(p)), dim3(256), 0, st, p->tb, c, p0, resid0, \
                       rhx, rhy, gck, gp0, SA);                                                            \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return last_error();
}

int fill_zero(hipStream_t st, void* ptr, size_t bytes) {
  const int64_t n = (int64_t)(bytes / sizeof(float));
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_blocks(n)), dim3(256), 0, st, static_cast<float*>(ptr), n);
  return last_error();
}

int copy_dev(hipStream_t st, const void* src, void* dst, size_t bytes) {
  const int64_t n = (int64_t)(bytes / sizeof(float));
  hipLaunchKernelGGL(k_copy, dim3(grid_blocks(n)), dim3(256), 0, st, n, static_cast<const float*>(src),
                     static_cast<float*>(dst));
  return last_error();
}

int set_ctl(hipStream_t st, StepCtl* ctl, int mask, int fwd_n, int adj_n, int hist_first) {
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(1), 0, st, reinterpret_cast<int32_t*>(ctl), mask, fwd_n, adj_n,
                     hist_first);
  return last_error();
}

#define PAT_TRY(expr)            \
  do {                           \
    int _s = (expr);             \
    if (_s != PAT_OK) return _s; \
  } while (0)

// Check mode: PAT_ENONFINITE if any of the arrays holds a NaN or an infinity
// (clears the plan's flag with a kernel, scans, copies the flag back and
// synchronizes the stream).
int check_outputs(const pat_plan* p, hipStream_t st, std::initializer_list<std::pair<const float*, int64_t>> arrays) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, st, p->flag, 0);
  PAT_TRY(last_error());
  for (const auto& a : arrays) {
    hipLaunchKernelGGL(k_flag_nonfinite, dim3(grid_blocks(a.second)), dim3(256), 0, st, a.first, a.second, p->flag);
    PAT_TRY(last_error());
  }
  int32_t h = 0;
  if (hipMemcpyAsync(&h, p->flag, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PAT_EHIP;
  return h ? PAT_ENONFINITE : PAT_OK;
}

// Arguments of a run of time steps (identical for every step of the run).
struct FwdArgs {
  const float* c;
  float *ux, *uy, *rx, *ry;
  float2 *SA, *SB;
  float* hist_base;   // nullptr: no history
  float* dpart;       // nullptr: no sensor samples
  StepCtl* ctl;
};
struct AdjArgs {
  const float* c;
  const float* hist_base;
  const float* resid;
  float *uhx, *uhy, *rhx, *rhy, *gck;
  float2 *SC, *SD;
  StepCtl* ctl;
};

int fwd_steps(const pat_plan* p, hipStream_t st, const FwdArgs& a, int count) {
  const pat_grid& g = p->g;
  const double nrm = 1.0 / ((double)g.nx * (double)g.ny);
  for (int i = 0; i < count; ++i) {
    PAT_TRY(launch_col<COL_GRAD1>(p, st, a.SA, a.SB, (float)(g.dt / g.rho0 * nrm), &a.ctl->fwd_n, +1));
    PAT_TRY(launch_fwd_u(p, st, a.ux, a.uy, a.SA, a.SB, a.ctl));
    PAT_TRY(launch_col<COL_PAIRM>(p, st, a.SA, a.SB, (float)(g.dt * g.rho0 * nrm), nullptr, 0));
    PAT_TRY(launch_fwd_rho(p, st, a.c, a.rx, a.ry, a.hist_base, a.dpart, a.SA, a.SB, a.ctl));
  }
  return PAT_OK;
}

int adj_steps(const pat_plan* p, hipStream_t st, const AdjArgs& a, int count) {
  const pat_grid& g = p->g;
  const double nrm = 1.0 / ((double)g.nx * (double)g.ny);
  for (int i = 0; i < count; ++i) {
    PAT_TRY(launch_col<COL_SUMM>(p, st, a.SC, a.SD, (float)(g.dt / g.rho0 * nrm), &a.ctl->adj_n, -1));
    PAT_TRY(launch_adj_rho(p, st, a.c, a.hist_base, a.resid, a.rhx, a.rhy, a.gck, a.SC, a.SD, a.ctl));
    PAT_TRY(launch_col<COL_PAIRP>(p, st, a.SC, a.SD, (float)(g.dt * g.rho0 * nrm), nullptr, 0));
    PAT_TRY(launch_adj_u(p, st, a.uhx, a.uhy, a.SC, a.SD, a.ctl));
  }
  return PAT_OK;
}

bool graphs_enabled() { return !g_trace.on && !std::getenv("PAT_NO_GRAPHS"); }

// Enqueue `count` steps on `st`: replay a captured graph when the same run
// (kind, arguments, count) was captured before, else capture it on the plan's
// private stream first.  Runs of one step are launched directly.
template <typename Args, typename Body>
int run_steps(pat_plan* p, hipStream_t st, const Args& a, int count, uint64_t kind, Body body) {
  if (count <= 0) return PAT_OK;
  if (count == 1 || !graphs_enabled()) return body(p, st, a, count);
  uint64_t key[14] = {kind, (uint64_t)count};
  static_assert(sizeof(Args) <= 12 * sizeof(uint64_t), "graph key");
  std::memcpy(&key[2], &a, sizeof(Args));
  for (auto& e : p->graphs) {
    if (std::memcmp(e.key, key, sizeof(key)) == 0) {
      e.last_use = ++p->graph_clock;
      if (hipGraphLaunch(e.exec, st) != hipSuccess) return PAT_EHIP;
      return hipEventRecord(e.done, st) == hipSuccess ? PAT_OK : PAT_EHIP;
    }
  }
  if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) return PAT_EHIP;
  // the capture stream must not run ahead of work already queued on st
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PAT_EHIP;
  const int st_body = body(p, p->cap, a, count);
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(p->cap, &graph);
  if (st_body != PAT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st_body;
  }
  if (e_end != hipSuccess || !graph) return PAT_EHIP;
  hipGraphExec_t exec = nullptr;
  const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e_inst != hipSuccess) return PAT_EHIP;
  if (p->graphs.size() >= 8) {   // evict the least recently used
    auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                [](const pat_plan::GraphEntry& x, const pat_plan::GraphEntry& y) {
                                  return x.last_use < y.last_use;
                                });
    (void)hipEventSynchronize(lru->done);   // it may still be running
    (void)hipEventDestroy(lru->done);
    (void)hipGraphExecDestroy(lru->exec);
    p->graphs.erase(lru);
  }
  pat_plan::GraphEntry ent;
  std::memcpy(ent.key, key, sizeof(key));
  ent.exec = exec;
  ent.last_use = ++p->graph_clock;
  if (hipEventCreateWithFlags(&ent.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return PAT_EHIP;
  }
  p->graphs.push_back(ent);
  if (hipGraphLaunch(exec, st) != hipSuccess) return PAT_EHIP;
  return hipEventRecord(ent.done, st) == hipSuccess ? PAT_OK : PAT_EHIP;
}

// Destroy a plan's captured graphs once their last launches have finished.
void drop_graphs(pat_plan* p) {
  for (auto& e : p->graphs) {
    (void)hipEventSynchronize(e.done);
    (void)hipEventDestroy(e.done);
    (void)hipGraphExecDestroy(e.exec);
  }
  p->graphs.clear();
}

constexpr int kChunk = 32;   // time steps per captured graph in store-all runs

// ----------------------------------------------------------------------------
// Host-side tables
// ----------------------------------------------------------------------------
double wavenumber(int i, int n, double d) {
  const int mm = i < (n + 1) / 2 ? i : i - n;   // FFT order, Nyquist negative
  return 2.0 * M_PI * mm / (n * d);
}

// k * (i exp(sgn i k d/2)); at the Nyquist bin of an even axis only the real part.
float2 shift_factor(int i, int n, double d, int sgn) {
  const double k = wavenumber(i, n, d);
  const double th = k * d / 2.0;
  double re = -sgn * k * std::sin(th);
  double im = k * std::cos(th);
  if (n % 2 == 0 && i == n / 2) im = 0.0;
  return make_float2((float)re, (float)im);
}

double pml_depth(int n, int P, double x) {
  double d = std::max(P - x, x - (n - 1 - P));
  return d > 0.0 ? d : 0.0;
}

void pml_axis(const pat_grid& g, int n, std::vector<float>& a, std::vector<float>& as, std::vector<float>& a2,
              std::vector<float>& as2, std::vector<float>& wf) {
  a.resize(n); as.resize(n); a2.resize(n); as2.resize(n); wf.resize(n);
  for (int i = 0; i < n; ++i) {
    double fa = 1.0, fs = 1.0;
    if (g.pml > 0) {
      const double d0 = pml_depth(n, g.pml, (double)i) / g.pml;
      const double d1 = pml_depth(n, g.pml, i + 0.5) / g.pml;
      const double amax = g.pml_alpha * g.c_ref / g.dx;
      fa = std::exp(-amax * d0 * d0 * d0 * d0 * g.dt / 2.0);
      fs = std::exp(-amax * d1 * d1 * d1 * d1 * g.dt / 2.0);
    }
    a[i] = (float)fa;
    as[i] = (float)fs;
    a2[i] = (float)(fa * fa);
    as2[i] = (float)(fs * fs);
    wf[i] = (float)(fs - 0.5 * fs * fs);
  }
}

}  // namespace

namespace {

// ----------------------------------------------------------------------------
// Batch executor.  Problems of one transform family and grid size form a
// class; the time steps of a class's problems advance in shared launches
// (batch_kernels.hpp), one stream per class.  The forward solves are aligned
// at their ends (a problem with fewer steps starts later) and the adjoint
// solves at their starts, so that between two start (or end) points the set
// of active problems is fixed: an epoch.  Each epoch has its slot tables in
// device memory, and its runs of up to kChunk steps are captured as graphs
// once and replayed.  Per-problem work (initial state, misfit, closing terms)
// is launched per problem.  A context (slot tables, graphs) is kept for the
// last batch and reused while the same problems come back.
// ----------------------------------------------------------------------------
std::vector<hipStream_t> g_pool;   // created on first use, destroyed by pat_batch_release

int pool_streams(int n) {
  while ((int)g_pool.size() < n) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return PAT_EHIP;
    g_pool.push_back(s);
  }
  return PAT_OK;
}

struct BatchProb {
  pat_problem pr;
  Layout L;
  FwdArgs f;
  AdjArgs a;
  int steps = 0;      // nt - 1 updates in each direction
  int col = 0, row = 0, adj = 0;   // blocks of one launch of each kind
};

struct SlotRange {     // a slot table in the context's device blob
  size_t off = 0;      // in slots
  int n = 0;
  int blocks = 0;      // total blocks of the launch over these slots
  int kb = 1;          // datasets per block (adjoint density, power-of-two family)
};

struct BatchEpoch {
  int begin = 0, end = 0;        // global steps [begin, end)
  SlotRange col, row;
  std::vector<SlotRange> adj;    // per group of equal datasets per block
  std::vector<int> starting;     // forward: members whose solve starts at `begin`
  std::vector<int> ending;       // adjoint: members whose solve ends at `end`
};

struct BatchClass {
  int nx = 0, ny = 0;
  bool fast = false;
  std::vector<int> members;
  int T = 0;
  std::vector<BatchEpoch> fwd, adj;
  std::vector<int> no_steps;     // members with nt = 1
  int stream = 0;
};

struct BatchGraph {
  uint64_t key;
  hipGraphExec_t exec;
  hipEvent_t done;
};

struct BatchContext {
  uint64_t sig = 0;
  std::vector<BatchProb> probs;
  std::vector<BatchClass> classes;
  std::vector<BatchSlot> host;   // every slot table
  BatchSlot* dev = nullptr;
  std::vector<BatchGraph> graphs;
  hipStream_t cap = nullptr;
};

BatchContext* g_batch = nullptr;

void batch_free(BatchContext* c) {
  if (!c) return;
  for (auto& g : c->graphs) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
    (void)hipGraphExecDestroy(g.exec);
  }
  if (c->dev) {
    (void)hipDeviceSynchronize();
    (void)hipFree(c->dev);
  }
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// Blocks of one launch of each kind for a problem (the single-problem launch shapes).
int launch_blocks(const pat_plan* p, int* col, int* row, int* adj) {
  if (p->fast) {
    switch (p->g.nx) {
#define X(N)                                                  \
  case N:                                                     \
    *row = frows_blocks<N>(p);                                \
    *adj = fadj_blocks<N>(p);                                 \
    break;
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
    switch (p->g.ny) {
#define X(N)                                                  \
  case N:                                                     \
    *col = fcols_blocks(p, fast::Cfg<N>::TC);                 \
    break;
      PAT_FAST_CASES(X)
#undef X
      default: return PAT_EUNSUPPORTED;
    }
    return PAT_OK;
  }
  switch (p->g.nx) {
#define X(N)                                                  \
  case N:                                                     \
    *row = rows_blocks<N>(p);                                 \
    *adj = *row;                                              \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  switch (p->g.ny) {
#define X(N)                                                  \
  case N:                                                     \
    *col = cols_blocks<N>(p);                                 \
    break;
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
  return PAT_OK;
}

BatchSlot make_slot(const BatchProb& b) {
  const pat_plan* p = b.pr.plan;
  const pat_grid& g = p->g;
  const double nrm = 1.0 / ((double)g.nx * (double)g.ny);
  BatchSlot s{};
  s.tb = p->tb;
  s.c = b.pr.c;
  s.ux = b.f.ux; s.uy = b.f.uy; s.rx = b.f.rx; s.ry = b.f.ry;
  s.SA = b.f.SA; s.SB = b.f.SB;
  s.hist_base = b.f.hist_base;
  s.dpart = b.f.dpart;
  s.resid = b.a.resid;
  s.uhx = b.a.uhx; s.uhy = b.a.uhy; s.rhx = b.a.rhx; s.rhy = b.a.rhy; s.gck = b.a.gck;
  s.SC = b.a.SC; s.SD = b.a.SD;
  s.ctl = b.f.ctl;
  s.sc_grad = (float)(g.dt / g.rho0 * nrm);
  s.sc_div = (float)(g.dt * g.rho0 * nrm);
  return s;
}

// Slot tables of an active set (members in class order) appended to ctx->host.
void add_tables(BatchContext* ctx, const BatchClass& cl, const std::vector<int>& active, BatchEpoch& e) {
  e.col.off = e.row.off = ctx->host.size();
  e.col.n = e.row.n = (int)active.size();
  int bc = 0, br = 0;
  for (int i : active) {
    BatchSlot s = make_slot(ctx->probs[i]);
    s.b_col = bc;
    s.b_row = br;
    s.b_adj = br;
    bc += ctx->probs[i].col;
    br += ctx->probs[i].row;
    ctx->host.push_back(s);
  }
  e.col.blocks = bc;
  e.row.blocks = br;
  e.adj.clear();
  if (!cl.fast) {                   // one adjoint-density launch over the row slots
    SlotRange r = e.row;
    e.adj.push_back(r);
    return;
  }
  for (int kb : {1, 2, 4, 8}) {     // one launch per block shape
    SlotRange r;
    r.off = ctx->host.size();
    r.kb = kb;
    int ba = 0;
    for (int i : active) {
      if (ctx->probs[i].pr.plan->kb != kb) continue;
      BatchSlot s = make_slot(ctx->probs[i]);
      s.b_adj = ba;
      ba += ctx->probs[i].adj;
      ctx->host.push_back(s);
      ++r.n;
    }
    r.blocks = ba;
    if (r.n) e.adj.push_back(r);
  }
}

int batch_build(BatchContext* ctx, int32_t nprob, const pat_problem* probs, int nstreams) {
  ctx->probs.resize((size_t)nprob);
  for (int i = 0; i < nprob; ++i) {
    const pat_problem& pr = probs[i];
    BatchProb& b = ctx->probs[i];
    b.pr = pr;
    pat_plan* p = pr.plan;
    b.L = make_layout(p, 0);
    if (pr.ws_bytes < b.L.total) return PAT_EWORKSPACE;
    void* ws = pr.ws;
    b.f.c = pr.c;
    b.f.ux = at<float>(ws, b.L.ux); b.f.uy = at<float>(ws, b.L.uy);
    b.f.rx = at<float>(ws, b.L.rx); b.f.ry = at<float>(ws, b.L.ry);
    b.f.SA = at<float2>(ws, b.L.SA); b.f.SB = at<float2>(ws, b.L.SB);
    b.f.hist_base = at<float>(ws, b.L.hist);
    b.f.dpart = at<float>(ws, b.L.dpart);
    b.f.ctl = at<StepCtl>(ws, b.L.ctl);
    b.a.c = pr.c;
    b.a.hist_base = b.f.hist_base;
    b.a.resid = pr.resid;
    b.a.uhx = at<float>(ws, b.L.uhx); b.a.uhy = at<float>(ws, b.L.uhy);
    b.a.rhx = at<float>(ws, b.L.rhx); b.a.rhy = at<float>(ws, b.L.rhy); b.a.gck = at<float>(ws, b.L.gck);
    b.a.SC = at<float2>(ws, b.L.SC); b.a.SD = at<float2>(ws, b.L.SD);
    b.a.ctl = b.f.ctl;
    b.steps = p->g.nt - 1;
    PAT_TRY(launch_blocks(p, &b.col, &b.row, &b.adj));
  }
  // classes: same family and grid size, in order of first appearance
  for (int i = 0; i < nprob; ++i) {
    const pat_plan* p = ctx->probs[i].pr.plan;
    BatchClass* cl = nullptr;
    for (auto& c : ctx->classes)
      if (c.nx == p->g.nx && c.ny == p->g.ny && c.fast == p->fast) cl = &c;
    if (!cl) {
      ctx->classes.emplace_back();
      cl = &ctx->classes.back();
      cl->nx = p->g.nx;
      cl->ny = p->g.ny;
      cl->fast = p->fast;
    }
    cl->members.push_back(i);
    cl->T = std::max(cl->T, ctx->probs[i].steps);
  }
  // the classes with the most work get their own streams first
  std::vector<double> work(ctx->classes.size(), 0.0);
  for (size_t c = 0; c < ctx->classes.size(); ++c)
    for (int i : ctx->classes[c].members) {
      const pat_plan* p = ctx->probs[i].pr.plan;
      work[c] += (double)p->K * p->g.nx * p->g.ny * p->g.nt;
    }
  std::vector<int> order(ctx->classes.size());
  for (size_t c = 0; c < order.size(); ++c) order[c] = (int)c;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<double> load((size_t)nstreams, 0.0);
  for (int c : order) {
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    ctx->classes[c].stream = s;
    load[s] += work[c];
  }
  // epochs and their slot tables
  for (auto& cl : ctx->classes) {
    std::vector<int> bounds;
    for (int i : cl.members) {
      if (ctx->probs[i].steps == 0) cl.no_steps.push_back(i);
      else bounds.push_back(cl.T - ctx->probs[i].steps);
    }
    bounds.push_back(cl.T);
    std::sort(bounds.begin(), bounds.end());
    bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
    for (size_t k = 0; k + 1 < bounds.size(); ++k) {
      BatchEpoch e;
      e.begin = bounds[k];
      e.end = bounds[k + 1];
      std::vector<int> active;
      for (int i : cl.members) {
        const int st = ctx->probs[i].steps;
        if (st == 0) continue;
        if (cl.T - st <= e.begin) active.push_back(i);
        if (cl.T - st == e.begin) e.starting.push_back(i);
      }
      add_tables(ctx, cl, active, e);
      cl.fwd.push_back(std::move(e));
    }
    bounds.assign(1, 0);
    for (int i : cl.members)
      if (ctx->probs[i].steps > 0) bounds.push_back(ctx->probs[i].steps);
    std::sort(bounds.begin(), bounds.end());
    bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
    for (size_t k = 0; k + 1 < bounds.size(); ++k) {
      BatchEpoch e;
      e.begin = bounds[k];
      e.end = bounds[k + 1];
      std::vector<int> active;
      for (int i : cl.members) {
        const int st = ctx->probs[i].steps;
        if (st >= e.end) active.push_back(i);
        if (st == e.end) e.ending.push_back(i);
      }
      add_tables(ctx, cl, active, e);
      cl.adj.push_back(std::move(e));
    }
  }
  if (!ctx->host.empty()) {
    const size_t bytes = ctx->host.size() * sizeof(BatchSlot);
    if (hipMalloc(&ctx->dev, bytes) != hipSuccess) return PAT_EHIP;
    if (hipMemcpy(ctx->dev, ctx->host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return PAT_EHIP;
  }
  return PAT_OK;
}

// `count` steps of an epoch, launched directly.
int batch_steps(const BatchContext* ctx, const BatchClass& cl, const BatchEpoch& e, bool fwd, int count,
                hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    const BatchSlot* sc = ctx->dev + e.col.off;
    const BatchSlot* sr = ctx->dev + e.row.off;
    if (fwd) {
      PAT_TRY(batch_launch_col(COL_GRAD1, cl.fast, cl.ny, sc, e.col.n, e.col.blocks, st));
      PAT_TRY(batch_launch_row(BK_FWD_U, cl.fast, cl.nx, sr, e.row.n, e.row.blocks, st));
      PAT_TRY(batch_launch_col(COL_PAIRM, cl.fast, cl.ny, sc, e.col.n, e.col.blocks, st));
      PAT_TRY(batch_launch_row(BK_FWD_RHO, cl.fast, cl.nx, sr, e.row.n, e.row.blocks, st));
    } else {
      PAT_TRY(batch_launch_col(COL_SUMM, cl.fast, cl.ny, sc, e.col.n, e.col.blocks, st));
      for (const auto& r : e.adj)
        PAT_TRY(batch_launch_adj_rho(cl.fast, cl.nx, r.kb, ctx->dev + r.off, r.n, r.blocks, st));
      PAT_TRY(batch_launch_col(COL_PAIRP, cl.fast, cl.ny, sc, e.col.n, e.col.blocks, st));
      PAT_TRY(batch_launch_row(BK_ADJ_U, cl.fast, cl.nx, sr, e.row.n, e.row.blocks, st));
    }
  }
  return PAT_OK;
}

// Enqueue `count` steps of an epoch: replay its captured graph (captured on
// first use), or launch directly for a single step or without graphs.
int batch_run(BatchContext* ctx, const BatchClass& cl, const BatchEpoch& e, bool fwd, int count, hipStream_t st) {
  if (count <= 0) return PAT_OK;
  if (count == 1 || !graphs_enabled()) return batch_steps(ctx, cl, e, fwd, count, st);
  uint64_t key = 1469598103934665603ull;
  const void* idents[3] = {&cl, &e, nullptr};
  key = fnv(key, idents, sizeof(idents));
  key = fnv(key, &fwd, sizeof(fwd));
  key = fnv(key, &count, sizeof(count));
  for (auto& g : ctx->graphs)
    if (g.key == key) {
      if (hipGraphLaunch(g.exec, st) != hipSuccess) return PAT_EHIP;
      return hipEventRecord(g.done, st) == hipSuccess ? PAT_OK : PAT_EHIP;
    }
  if (!ctx->cap && hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) return PAT_EHIP;
  if (hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PAT_EHIP;
  const int sb = batch_steps(ctx, cl, e, fwd, count, ctx->cap);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(ctx->cap, &graph);
  if (sb != PAT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return sb;
  }
  if (ee != hipSuccess || !graph) return PAT_EHIP;
  BatchGraph g{key, nullptr, nullptr};
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return PAT_EHIP;
  if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGraphExecDestroy(g.exec);
    return PAT_EHIP;
  }
  ctx->graphs.push_back(g);
  if (hipGraphLaunch(g.exec, st) != hipSuccess) return PAT_EHIP;
  return hipEventRecord(g.done, st) == hipSuccess ? PAT_OK : PAT_EHIP;
}

int batch_fwd_init(const BatchProb& b, hipStream_t st) {
  PAT_TRY(set_ctl(st, b.f.ctl, 1 | 4, -1, 0, 0));
  return launch_fwd_init(b.pr.plan, st, b.pr.c, b.pr.p0, b.f.rx, b.f.ry, b.f.hist_base, b.f.dpart, b.f.SA);
}

// Between the two solves: traces, misfit and J, adjoint state at zero.
int batch_middle(const BatchProb& b, hipStream_t st) {
  const pat_plan* p = b.pr.plan;
  const pat_grid& g = p->g;
  const int64_t rows = (int64_t)p->K * g.nt;
  hipLaunchKernelGGL(k_sensor_finalize, dim3(grid_blocks(rows * p->m)), dim3(256), 0, st, b.f.dpart, b.pr.data,
                     rows, p->m);
  PAT_TRY(last_error());
  const int64_t per_k = (int64_t)g.nt * p->m;
  hipLaunchKernelGGL(k_misfit, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, b.pr.data, b.pr.y, b.pr.w, b.pr.resid,
                     p->red, per_k, p->K);
  PAT_TRY(last_error());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RED_THREADS), 0, st, p->red, RED_BLOCKS, b.pr.J, 0.5);
  PAT_TRY(last_error());
  PAT_TRY(fill_zero(st, b.a.uhx, b.L.F));
  PAT_TRY(fill_zero(st, b.a.uhy, b.L.F));
  PAT_TRY(fill_zero(st, b.a.rhx, b.L.F));
  PAT_TRY(fill_zero(st, b.a.rhy, b.L.F));
  PAT_TRY(fill_zero(st, b.a.gck, b.L.F));
  PAT_TRY(fill_zero(st, b.a.SC, b.L.Sp));
  PAT_TRY(fill_zero(st, b.a.SD, b.L.Sp));
  return set_ctl(st, b.a.ctl, 2 | 4, 0, g.nt, 0);
}

// Closing terms of the adjoint: g_p0 and the initial-state part of g_c.
int batch_closing(const BatchProb& b, hipStream_t st) {
  const pat_plan* p = b.pr.plan;
  const pat_grid& g = p->g;
  const double nrm = 1.0 / ((double)g.nx * (double)g.ny);
  PAT_TRY(launch_col<COL_SUMM>(p, st, b.a.SC, b.a.SD, (float)(g.dt / g.rho0 * nrm), nullptr, 0));
  PAT_TRY(launch_adj_final(p, st, b.pr.c, b.pr.p0, b.pr.resid, b.a.rhx, b.a.rhy, b.a.gck, b.pr.g_p0, b.a.SC));
  const int64_t npix = (int64_t)g.ny * g.nx;
  hipLaunchKernelGGL(k_reduce_k, dim3(grid_blocks(npix)), dim3(256), 0, st, b.a.gck, b.pr.g_c, p->gsl, npix);
  return last_error();
}

// One class's whole evaluation on stream st.
int batch_class(BatchContext* ctx, const BatchClass& cl, hipStream_t st) {
  for (const auto& e : cl.fwd) {
    for (int i : e.starting) PAT_TRY(batch_fwd_init(ctx->probs[i], st));
    for (int n = e.begin; n < e.end;) {
      const int cnt = std::min(kChunk, e.end - n);
      PAT_TRY(batch_run(ctx, cl, e, true, cnt, st));
      n += cnt;
    }
  }
  for (int i : cl.no_steps) PAT_TRY(batch_fwd_init(ctx->probs[i], st));
  for (int i : cl.members) PAT_TRY(batch_middle(ctx->probs[i], st));
  for (int i : cl.no_steps) PAT_TRY(batch_closing(ctx->probs[i], st));
  for (const auto& e : cl.adj) {
    for (int n = e.begin; n < e.end;) {
      const int cnt = std::min(kChunk, e.end - n);
      PAT_TRY(batch_run(ctx, cl, e, false, cnt, st));
      n += cnt;
    }
    for (int i : e.ending) PAT_TRY(batch_closing(ctx->probs[i], st));
  }
  return PAT_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
struct pat_ou {
  int ny = 0, nx = 0;                 // grid of the vectors
  int oy = 0, ox = 0, nby = 0, nbx = 0;   // bounding box of the mask
  int L = 0;                          // periodic embedding (L x L, L >= 2 max(nby, nbx) - 1)
  void* dev = nullptr;                // twiddles, spectra, box mask
  float2* tw = nullptr;
  float* s_op = nullptr;              // spectrum of the embedded kernel (exact products)
  float* s_pre = nullptr;             // reciprocal spectrum, floored (preconditioner)
  uint8_t* mask = nullptr;            // [nby][nbx]
};

namespace {

// Scratch of an OU solve with nvec right-hand sides.
struct OuLayout {
  size_t b, x, r, z, p, Ap, W, partial, sc, dots, total;
};
OuLayout ou_layout(const pat_ou* o, int nvec) {
  OuLayout L{};
  const size_t nb = (size_t)nvec * o->nby * o->nbx * sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  L.b = take(nb); L.x = take(nb); L.r = take(nb); L.z = take(nb); L.p = take(nb); L.Ap = take(nb);
  L.W = take((size_t)nvec * o->nby * o->L * sizeof(float2));
  L.partial = take((size_t)nvec * ou::DOT_BLOCKS * sizeof(double));
  L.sc = take((size_t)5 * nvec * sizeof(double));
  L.dots = take((size_t)nvec * sizeof(double));
  L.total = off;
  return L;
}

// out = P_M C P_M v for the circulant C with spectrum S (box vectors).
int ou_circ(const pat_ou* o, hipStream_t st, int nvec, const float* v, const float* S, float2* W, float* out) {
  const float scale = 1.0f / ((float)o->L * (float)o->L);
  switch (o->L) {
#define X(N)                                                                                                  \
  case N: {                                                                                                   \
    constexpr int T = Threads<N>::v;                                                                          \
    const int rows = nvec * o->nby, cols = nvec * N;                                                          \
    hipLaunchKernelGGL(ou::k_rows_fwd<N>, dim3((rows + 256 / T - 1) / (256 / T)), dim3(256), 0, st, v, nvec,  \
                       o->nby, o->nbx, o->tw, W);                                                             \
    hipLaunchKernelGGL(ou::k_cols<N>, dim3((cols + 256 / T - 1) / (256 / T)), dim3(256), 0, st, W, nvec,      \
                       o->nby, S, o->tw);                                                                     \
    hipLaunchKernelGGL(ou::k_rows_inv<N>, dim3((rows + 256 / T - 1) / (256 / T)), dim3(256), 0, st, W, nvec,  \
                       o->nby, o->nbx, o->mask, o->tw, scale, out);                                           \
    return last_error();                                                                                      \
  }
    PAT_SIZE_CASES(X)
#undef X
    default: return PAT_EUNSUPPORTED;
  }
}

// dots[vec] = a_vec . b_vec (box vectors, fixed order)
int ou_dots(const pat_ou* o, hipStream_t st, int nvec, const float* a, const float* b, double* partial,
            double* out) {
  const int64_t n = (int64_t)o->nby * o->nbx;
  hipLaunchKernelGGL(ou::k_dots, dim3(ou::DOT_BLOCKS, nvec), dim3(ou::DOT_THREADS), 0, st, a, b, n, partial);
  PAT_TRY(last_error());
  hipLaunchKernelGGL(ou::k_dot_final, dim3((nvec + 63) / 64), dim3(64), 0, st, partial, nvec, out);
  return last_error();
}

// x = Xi_M^{-1} b by preconditioned conjugate gradients (box vectors in the scratch).
int ou_pcg(const pat_ou* o, hipStream_t st, int nvec, char* ws, const OuLayout& L, double tol, int maxit,
           int* iters) {
  float* b = reinterpret_cast<float*>(ws + L.b);
  float* x = reinterpret_cast<float*>(ws + L.x);
  float* r = reinterpret_cast<float*>(ws + L.r);
  float* z = reinterpret_cast<float*>(ws + L.z);
  float* p = reinterpret_cast<float*>(ws + L.p);
  float* Ap = reinterpret_cast<float*>(ws + L.Ap);
  float2* W = reinterpret_cast<float2*>(ws + L.W);
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* sc = reinterpret_cast<double*>(ws + L.sc);
  double* dots = reinterpret_cast<double*>(ws + L.dots);
  const int64_t n = (int64_t)o->nby * o->nbx, tot = n * nvec;
  const size_t vb = (size_t)tot * sizeof(float);
  PAT_TRY(fill_zero(st, x, vb));
  PAT_TRY(copy_dev(st, b, r, vb));
  std::vector<double> bb((size_t)nvec), rr((size_t)nvec);
  PAT_TRY(ou_dots(o, st, nvec, b, b, partial, dots));
  if (hipMemcpyAsync(bb.data(), dots, nvec * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PAT_EHIP;
  PAT_TRY(ou_circ(o, st, nvec, r, o->s_pre, W, z));
  PAT_TRY(copy_dev(st, z, p, vb));
  PAT_TRY(ou_dots(o, st, nvec, r, z, partial, sc));   // rz
  const int vb1 = (nvec + 63) / 64;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    PAT_TRY(ou_circ(o, st, nvec, p, o->s_op, W, Ap));
    PAT_TRY(ou_dots(o, st, nvec, p, Ap, partial, sc + nvec));   // pAp
    hipLaunchKernelGGL(ou::k_cg_alpha, dim3(vb1), dim3(64), 0, st, sc, nvec);
    hipLaunchKernelGGL(ou::k_cg_update, dim3(grid_blocks(tot)), dim3(256), 0, st, nvec, n, sc, p, Ap, x, r);
    PAT_TRY(last_error());
    if (it % 8 == 0 || it == maxit) {   // convergence test on the host every 8 iterations
      PAT_TRY(ou_dots(o, st, nvec, r, r, partial, dots));
      if (hipMemcpyAsync(rr.data(), dots, nvec * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return PAT_EHIP;
      bool done = true;
      for (int v = 0; v < nvec; ++v) done = done && rr[v] <= tol * tol * bb[v];
      if (done) break;
    }
    PAT_TRY(ou_circ(o, st, nvec, r, o->s_pre, W, z));
    PAT_TRY(ou_dots(o, st, nvec, r, z, partial, sc + 4 * nvec));   // rz_new
    hipLaunchKernelGGL(ou::k_cg_beta, dim3(vb1), dim3(64), 0, st, sc, nvec);
    hipLaunchKernelGGL(ou::k_cg_dir, dim3(grid_blocks(tot)), dim3(256), 0, st, nvec, n, sc, z, p);
    PAT_TRY(last_error());
  }
  if (iters) *iters = std::min(it, maxit);
  return PAT_OK;
}

// 1/2 sum_v w_v dots[v] -> *J (one thread, fixed order)
__global__ void k_ou_energy(const double* __restrict__ dots, const float* __restrict__ w, int nvec, double* J) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int v = 0; v < nvec; ++v) s += 0.5 * (double)w[v] * dots[v];
    *J = s;
  }
}

}  // namespace

extern "C" {

const char* pat_status_string(int s) {
  switch (s) {
    case PAT_OK: return "ok";
    case PAT_EINVAL: return "invalid argument";
    case PAT_EUNSUPPORTED: return "unsupported size";
    case PAT_EWORKSPACE: return "workspace too small or not filled by a recording pat_forward";
    case PAT_EHIP: return "HIP runtime error";
    case PAT_ENONFINITE: return "non-finite value in an output (check mode)";
    default: return "unknown status";
  }
}

int pat_plan_create(const pat_grid* g, int32_t K, int32_t m, const double* sensor_xy, pat_plan** out) {
  if (!g || !out || !sensor_xy) return PAT_EINVAL;
  *out = nullptr;
  if (g->nx <= 0 || g->ny <= 0 || g->nt <= 0 || K <= 0 || m <= 0 || g->pml < 0 || !(g->dx > 0) ||
      !(g->dt > 0) || !(g->c_ref > 0) || !(g->rho0 > 0) || !(g->pml_alpha >= 0))
    return PAT_EINVAL;
  if (2 * g->pml >= g->nx || 2 * g->pml >= g->ny) return PAT_EINVAL;
  if (!supported(g->nx) || !supported(g->ny) || K > 64) return PAT_EUNSUPPORTED;
  const int nx = g->nx, ny = g->ny, nh = nx / 2 + 1;

  // --- sensors: bilinear taps on cell centres (Sec. 2.2)
  std::vector<GatherEnt> gent;
  struct Tap { int row, ix, sensor; float w; };
  std::vector<Tap> taps;
  for (int s = 0; s < m; ++s) {
    const double fx = sensor_xy[2 * s] / g->dx + nx / 2.0 - 0.5;
    const double fy = sensor_xy[2 * s + 1] / g->dx + ny / 2.0 - 0.5;
    if (!std::isfinite(fx) || !std::isfinite(fy)) return PAT_EINVAL;
    const int i0 = (int)std::floor(fx), j0 = (int)std::floor(fy);
    if (i0 < 0 || j0 < 0 || i0 + 1 > nx - 1 || j0 + 1 > ny - 1) return PAT_EINVAL;
    const double tx = fx - i0, ty = fy - j0;
    gent.push_back({j0, i0, s, 0, (float)((1 - tx) * (1 - ty)), (float)(tx * (1 - ty))});
    gent.push_back({j0 + 1, i0, s, 1, (float)((1 - tx) * ty), (float)(tx * ty)});
    taps.push_back({j0, i0, s, (float)((1 - tx) * (1 - ty))});
    taps.push_back({j0, i0 + 1, s, (float)(tx * (1 - ty))});
    taps.push_back({j0 + 1, i0, s, (float)((1 - tx) * ty)});
    taps.push_back({j0 + 1, i0 + 1, s, (float)(tx * ty)});
  }
  std::stable_sort(gent.begin(), gent.end(), [](const GatherEnt& a, const GatherEnt& b) { return a.row < b.row; });
  std::vector<int32_t> grs(ny + 1, 0);
  for (const auto& e : gent) grs[e.row + 1]++;
  for (int y = 0; y < ny; ++y) grs[y + 1] += grs[y];
  std::stable_sort(taps.begin(), taps.end(), [](const Tap& a, const Tap& b) {
    return a.row != b.row ? a.row < b.row : a.ix < b.ix;
  });
  std::vector<ScatterPix> spix;
  std::vector<ScatterTap> stap;
  for (size_t i = 0; i < taps.size();) {
    size_t j = i;
    ScatterPix px{};
    px.row = taps[i].row;
    px.ix = taps[i].ix;
    px.start = (int32_t)stap.size();
    while (j < taps.size() && taps[j].row == taps[i].row && taps[j].ix == taps[i].ix) {
      if (j - i < 4) {
        px.sensor[j - i] = taps[j].sensor;
        px.w[j - i] = taps[j].w;
      }
      stap.push_back({taps[j].sensor, taps[j].w});
      ++j;
    }
    px.count = (int32_t)(j - i);
    spix.push_back(px);
    i = j;
  }
  std::vector<int32_t> srs(ny + 1, 0);
  for (const auto& e : spix) srs[e.row + 1]++;
  for (int y = 0; y < ny; ++y) srs[y + 1] += srs[y];

  // --- FFT twiddles, staggered derivative factors, kappa, PML
  std::vector<float2> twx(nx), twy(ny), exp_(nh), exm(nh), eyp(ny), eym(ny);
  for (int j = 0; j < nx; ++j) twx[j] = make_float2((float)std::cos(2 * M_PI * j / nx), (float)-std::sin(2 * M_PI * j / nx));
  for (int j = 0; j < ny; ++j) twy[j] = make_float2((float)std::cos(2 * M_PI * j / ny), (float)-std::sin(2 * M_PI * j / ny));
  for (int i = 0; i < nh; ++i) { exp_[i] = shift_factor(i, nx, g->dx, +1); exm[i] = shift_factor(i, nx, g->dx, -1); }
  for (int i = 0; i < ny; ++i) { eyp[i] = shift_factor(i, ny, g->dx, +1); eym[i] = shift_factor(i, ny, g->dx, -1); }
  std::vector<float> kap((size_t)ny * nh);
  for (int e = 0; e < ny; ++e) {
    const double ky = wavenumber(e, ny, g->dx);
    for (int i = 0; i < nh; ++i) {
      const double kx = wavenumber(i, nx, g->dx);
      const double arg = g->c_ref * std::sqrt(kx * kx + ky * ky) * g->dt / 2.0;
      kap[(size_t)i * ny + e] = (float)(arg == 0.0 ? 1.0 : std::sin(arg) / arg);   // column-major: [nh][ny]
    }
  }
  std::vector<float> ax, asx, ax2, asx2, wfx, ay, asy, ay2, asy2, wfy;
  pml_axis(*g, nx, ax, asx, ax2, asx2, wfx);
  pml_axis(*g, ny, ay, asy, ay2, asy2, wfy);

  // --- one device blob
  struct Piece { const void* src; size_t bytes; size_t off; };
  std::vector<Piece> pieces;
  size_t total = 0;
  auto add = [&](const void* src, size_t bytes) {
    pieces.push_back({src, bytes, total});
    total += align256(std::max<size_t>(bytes, 4));
    return pieces.size() - 1;
  };
  size_t i_twx = add(twx.data(), nx * sizeof(float2)), i_twy = add(twy.data(), ny * sizeof(float2));
  size_t i_exp = add(exp_.data(), nh * sizeof(float2)), i_exm = add(exm.data(), nh * sizeof(float2));
  size_t i_eyp = add(eyp.data(), ny * sizeof(float2)), i_eym = add(eym.data(), ny * sizeof(float2));
  size_t i_kap = add(kap.data(), kap.size() * sizeof(float));
  size_t i_ax = add(ax.data(), nx * 4), i_asx = add(asx.data(), nx * 4), i_ax2 = add(ax2.data(), nx * 4),
         i_asx2 = add(asx2.data(), nx * 4), i_wfx = add(wfx.data(), nx * 4);
  size_t i_ay = add(ay.data(), ny * 4), i_asy = add(asy.data(), ny * 4), i_ay2 = add(ay2.data(), ny * 4),
         i_asy2 = add(asy2.data(), ny * 4), i_wfy = add(wfy.data(), ny * 4);
  size_t i_grs = add(grs.data(), grs.size() * 4), i_gent = add(gent.data(), gent.size() * sizeof(GatherEnt));
  size_t i_srs = add(srs.data(), srs.size() * 4), i_spix = add(spix.data(), spix.size() * sizeof(ScatterPix));
  size_t i_stap = add(stap.data(), stap.size() * sizeof(ScatterTap));
  size_t i_red = add(nullptr, RED_BLOCKS * sizeof(double));
  size_t i_flag = add(nullptr, sizeof(int32_t));

  pat_plan* p = new (std::nothrow) pat_plan();
  if (!p) return PAT_EHIP;
  p->g = *g;
  p->K = K;
  p->m = m;
  p->nh = nh;
  p->fast = fast_size(nx) && fast_size(ny) && !std::getenv("PAT_GENERIC_KERNELS");
  p->nhs = p->fast ? nx / 2 : nh;
  // 4 datasets per block: g_c traffic 2 B/pt instead of 8; 1, 2 and 8 per
  // block measured slower at 512^2 x 8
  p->kb = !p->fast ? 1 : (K >= 4 ? 4 : (K >= 2 ? 2 : 1));
  p->gsl = (K + p->kb - 1) / p->kb;
  if (hipMalloc(&p->dev, total) != hipSuccess) {
    delete p;
    return PAT_EHIP;
  }
  std::vector<char> host(total, 0);
  for (const auto& pc : pieces)
    if (pc.src) std::memcpy(host.data() + pc.off, pc.src, pc.bytes);
  if (hipMemcpy(p->dev, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->dev);
    delete p;
    return PAT_EHIP;
  }
  char* d = static_cast<char*>(p->dev);
  auto P = [&](size_t i) { return static_cast<void*>(d + pieces[i].off); };
  Tables& t = p->tb;
  t.tw_x = (const float2*)P(i_twx); t.tw_y = (const float2*)P(i_twy);
  t.ex_p = (const float2*)P(i_exp); t.ex_m = (const float2*)P(i_exm);
  t.ey_p = (const float2*)P(i_eyp); t.ey_m = (const float2*)P(i_eym);
  t.kappa = (const float*)P(i_kap);
  t.ax = (const float*)P(i_ax); t.asx = (const float*)P(i_asx); t.ax2 = (const float*)P(i_ax2);
  t.asx2 = (const float*)P(i_asx2); t.wfx = (const float*)P(i_wfx);
  t.ay = (const float*)P(i_ay); t.asy = (const float*)P(i_asy); t.ay2 = (const float*)P(i_ay2);
  t.asy2 = (const float*)P(i_asy2); t.wfy = (const float*)P(i_wfy);
  t.g_row_start = (const int32_t*)P(i_grs); t.g_ent = (const GatherEnt*)P(i_gent);
  t.s_row_start = (const int32_t*)P(i_srs); t.s_pix = (const ScatterPix*)P(i_spix);
  t.s_tap = (const ScatterTap*)P(i_stap);
  t.nx = nx; t.ny = ny; t.nh = nh; t.K = K; t.m = m; t.nt = g->nt;
  p->red = (double*)P(i_red);
  p->flag = (int32_t*)P(i_flag);
  p->check_finite = std::getenv("PAT_CHECK_FINITE") != nullptr;
  *out = p;
  return PAT_OK;
}

int pat_plan_destroy(pat_plan* p) {
  if (!p) return PAT_EINVAL;
  drop_graphs(p);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->dev) (void)hipFree(p->dev);
  delete p;
  return PAT_OK;
}

int pat_workspace_size(const pat_plan* p, int32_t ckpt_every, size_t* bytes) {
  if (!p || !bytes || ckpt_every < 0) return PAT_EINVAL;
  *bytes = make_layout(p, ckpt_every).total;
  return PAT_OK;
}

int pat_forward(pat_plan* p, const float* c, const float* p0, float* data, void* ws, size_t ws_bytes,
                int32_t ckpt_every, int32_t record, void* stream) {
  if (!p || !c || !p0 || !data || !ws || ckpt_every < 0) return PAT_EINVAL;
  const Layout L = make_layout(p, ckpt_every);
  if (ws_bytes < L.total) return PAT_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const pat_grid& g = p->g;
  FwdArgs a;
  a.c = c;
  a.ux = at<float>(ws, L.ux); a.uy = at<float>(ws, L.uy); a.rx = at<float>(ws, L.rx); a.ry = at<float>(ws, L.ry);
  a.SA = at<float2>(ws, L.SA); a.SB = at<float2>(ws, L.SB);
  a.dpart = at<float>(ws, L.dpart);
  a.ctl = at<StepCtl>(ws, L.ctl);
  const bool store_all = record && ckpt_every == 0;
  const bool ckpt = record && ckpt_every > 0;
  a.hist_base = store_all ? at<float>(ws, L.hist) : nullptr;
  if (record) p->recorded = false;
  auto body = [](pat_plan* pp, hipStream_t s2, const FwdArgs& aa, int cnt) { return fwd_steps(pp, s2, aa, cnt); };

  PAT_TRY(set_ctl(st, a.ctl, 1 | 4, -1, 0, 0));
  PAT_TRY(launch_fwd_init(p, st, c, p0, a.rx, a.ry, a.hist_base, a.dpart, a.SA));
  const int steps = g.nt - 1;
  int n = 0;
  while (n < steps) {
    if (ckpt && n > 0 && n % ckpt_every == 0) {
      const int slot = n / ckpt_every - 1;
      char* ck = at<char>(ws, L.ckpt) + (size_t)slot * (4 * align256(L.F) + align256(L.Sp));
      PAT_TRY(copy_dev(st, a.ux, ck, L.F));
      PAT_TRY(copy_dev(st, a.uy, ck + align256(L.F), L.F));
      PAT_TRY(copy_dev(st, a.rx, ck + 2 * align256(L.F), L.F));
      PAT_TRY(copy_dev(st, a.ry, ck + 3 * align256(L.F), L.F));
      PAT_TRY(copy_dev(st, a.SA, ck + 4 * align256(L.F), L.Sp));
    }
    int cnt = std::min(kChunk, steps - n);
    if (ckpt) cnt = std::min(ckpt_every - n % ckpt_every, steps - n);
    PAT_TRY(run_steps(p, st, a, cnt, 1, body));
    n += cnt;
  }
  const int64_t rows = (int64_t)p->K * g.nt;
  hipLaunchKernelGGL(k_sensor_finalize, dim3(grid_blocks(rows * p->m)), dim3(256), 0, st, a.dpart, data, rows, p->m);
  PAT_TRY(last_error());
  if (record) {
    p->recorded = true;
    p->rec_ws = ws;
    p->rec_c = c;
    p->rec_p0 = p0;
    p->rec_ckpt = ckpt_every;
  }
  if (p->check_finite) return check_outputs(p, st, {{data, rows * p->m}});
  return PAT_OK;
}

int pat_history_field(const pat_plan* p, const void* ws, int32_t n, const float** field) {
  if (!p || !ws || !field || n < 0 || n >= p->g.nt) return PAT_EINVAL;
  *field = nullptr;
  if (!p->recorded || p->rec_ws != ws || p->rec_ckpt != 0) return PAT_EWORKSPACE;
  const Layout L = make_layout(p, 0);
  *field = at<const float>(const_cast<void*>(ws), L.hist + (size_t)n * L.F);
  return PAT_OK;
}

int pat_misfit(pat_plan* p, const float* data, const float* y, const float* w, float* resid, double* J,
               void* stream) {
  if (!p || !data || !y || !w || !resid || !J) return PAT_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t per_k = (int64_t)p->g.nt * p->m;
  hipLaunchKernelGGL(k_misfit, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, data, y, w, resid, p->red, per_k, p->K);
  PAT_TRY(last_error());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RED_THREADS), 0, st, p->red, RED_BLOCKS, J, 0.5);
  return last_error();
}

int pat_adjoint_gradient(pat_plan* p, const float* c, const float* p0, const float* resid, float* g_p0, float* g_c,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!p || !c || !p0 || !resid || !g_p0 || !g_c || !ws) return PAT_EINVAL;
  if (!p->recorded || p->rec_ws != ws || p->rec_c != c || p->rec_p0 != p0) return PAT_EWORKSPACE;
  const int s = p->rec_ckpt;
  const Layout L = make_layout(p, s);
  if (ws_bytes < L.total) return PAT_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const pat_grid& g = p->g;
  const double nrm = 1.0 / ((double)g.nx * (double)g.ny);
  AdjArgs a;
  a.c = c;
  a.hist_base = at<float>(ws, L.hist);
  a.resid = resid;
  a.uhx = at<float>(ws, L.uhx); a.uhy = at<float>(ws, L.uhy); a.rhx = at<float>(ws, L.rhx);
  a.rhy = at<float>(ws, L.rhy); a.gck = at<float>(ws, L.gck);
  a.SC = at<float2>(ws, L.SC); a.SD = at<float2>(ws, L.SD);
  a.ctl = at<StepCtl>(ws, L.ctl);
  auto abody = [](pat_plan* pp, hipStream_t s2, const AdjArgs& aa, int cnt) { return adj_steps(pp, s2, aa, cnt); };
  auto fbody = [](pat_plan* pp, hipStream_t s2, const FwdArgs& aa, int cnt) { return fwd_steps(pp, s2, aa, cnt); };
  // adjoint state starts at zero (fill kernels: no memset nodes)
  PAT_TRY(fill_zero(st, a.uhx, L.F));
  PAT_TRY(fill_zero(st, a.uhy, L.F));
  PAT_TRY(fill_zero(st, a.rhx, L.F));
  PAT_TRY(fill_zero(st, a.rhy, L.F));
  PAT_TRY(fill_zero(st, a.gck, L.F));
  PAT_TRY(fill_zero(st, a.SC, L.Sp));
  PAT_TRY(fill_zero(st, a.SD, L.Sp));
  PAT_TRY(set_ctl(st, a.ctl, 2 | 4, 0, g.nt, 0));

  int n = g.nt - 1;   // next adjoint step
  if (s == 0) {
    while (n >= 1) {
      const int cnt = std::min(kChunk, n);
      PAT_TRY(run_steps(p, st, a, cnt, 2, abody));
      n -= cnt;
    }
  } else {
    FwdArgs f;
    f.c = c;
    f.ux = at<float>(ws, L.ux); f.uy = at<float>(ws, L.uy); f.rx = at<float>(ws, L.rx); f.ry = at<float>(ws, L.ry);
    f.SA = at<float2>(ws, L.SA); f.SB = at<float2>(ws, L.SB);
    f.hist_base = at<float>(ws, L.hist);   // the segment buffer: slot j holds level n0 + 1 + j
    f.dpart = nullptr;
    f.ctl = a.ctl;
    while (n >= 1) {
      const int n0 = ((n - 1) / s) * s;
      // recompute p^{n0+1 .. n} from the checkpoint at n0 into the segment buffer
      PAT_TRY(set_ctl(st, a.ctl, 1 | 4, n0 - 1, 0, n0 + 1));
      if (n0 == 0) {
        PAT_TRY(launch_fwd_init(p, st, c, p0, f.rx, f.ry, nullptr, nullptr, f.SA));
      } else {
        const int slot = n0 / s - 1;
        const char* ck = at<char>(ws, L.ckpt) + (size_t)slot * (4 * align256(L.F) + align256(L.Sp));
        PAT_TRY(copy_dev(st, ck, f.ux, L.F));
        PAT_TRY(copy_dev(st, ck + align256(L.F), f.uy, L.F));
        PAT_TRY(copy_dev(st, ck + 2 * align256(L.F), f.rx, L.F));
        PAT_TRY(copy_dev(st, ck + 3 * align256(L.F), f.ry, L.F));
        PAT_TRY(copy_dev(st, ck + 4 * align256(L.F), f.SA, L.Sp));
      }
      PAT_TRY(run_steps(p, st, f, n - n0, 3, fbody));
      PAT_TRY(run_steps(p, st, a, n - n0, 2, abody));
      n = n0;
    }
  }
  PAT_TRY(launch_col<COL_SUMM>(p, st, a.SC, a.SD, (float)(g.dt / g.rho0 * nrm), nullptr, 0));
  PAT_TRY(launch_adj_final(p, st, c, p0, resid, a.rhx, a.rhy, a.gck, g_p0, a.SC));
  const int64_t npix = (int64_t)g.ny * g.nx;
  hipLaunchKernelGGL(k_reduce_k, dim3(grid_blocks(npix)), dim3(256), 0, st, a.gck, g_c, p->gsl, npix);
  PAT_TRY(last_error());
  if (p->check_finite) return check_outputs(p, st, {{g_p0, (int64_t)p->K * npix}, {g_c, npix}});
  return PAT_OK;
}

int pat_project_update(int64_t n, float* x, const float* d, float alpha, const float* lo, const float* hi,
                       float lo_s, float hi_s, void* stream) {
  if (n < 0 || (n > 0 && (!x || !d))) return PAT_EINVAL;
  if (n == 0) return PAT_OK;
  hipLaunchKernelGGL(k_project_update, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, x, d,
                     alpha, lo, hi, lo_s, hi_s);
  return last_error();
}

int pat_free_part(int64_t n, const float* x, const float* g, const float* lo, const float* hi, const float* v,
                  float* out, void* stream) {
  if (n <= 0 || !x || !g || !lo || !hi || !v || !out) return PAT_EINVAL;
  hipLaunchKernelGGL(k_free_part, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, x, g, lo,
                     hi, v, out);
  return last_error();
}

int pat_axpby(int64_t n, float a, const float* x, float b, const float* y, float* out, void* stream) {
  if (n <= 0 || !x || !out) return PAT_EINVAL;
  hipLaunchKernelGGL(k_axpby, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, a, x, b, y,
                     out);
  return last_error();
}

int pat_mul(int64_t n, const float* x, const float* s, float* out, void* stream) {
  if (n <= 0 || !x || !s || !out) return PAT_EINVAL;
  hipLaunchKernelGGL(k_mul, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, x, s, out);
  return last_error();
}

int pat_prolong(int32_t nchan, const float* coarse, int32_t nxc, int32_t nyc, float* fine, int32_t nxf, int32_t nyf,
                void* stream) {
  if (nchan <= 0 || nyc <= 0 || nxc <= 0 || nyf <= 0 || nxf <= 0 || !coarse || !fine) return PAT_EINVAL;
  const int64_t n = (int64_t)nchan * nyf * nxf;
  hipLaunchKernelGGL(k_prolong, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), nchan, coarse,
                     nyc, nxc, fine, nyf, nxf);
  return last_error();
}

int pat_prolong_phys(int32_t nchan, const float* coarse, int32_t nxc, int32_t nyc, double dxc, float* fine,
                     int32_t nxf, int32_t nyf, double dxf, void* stream) {
  if (nchan <= 0 || nyc <= 0 || nxc <= 0 || nyf <= 0 || nxf <= 0 || !coarse || !fine || !(dxc > 0.0) ||
      !(dxf > 0.0))
    return PAT_EINVAL;
  const int64_t n = (int64_t)nchan * nyf * nxf;
  hipLaunchKernelGGL(k_prolong_phys, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), nchan,
                     coarse, nyc, nxc, dxc, fine, nyf, nxf, dxf);
  return last_error();
}

int pat_time_interp(int32_t nlead, int32_t nt_src, int32_t m, const float* y, double dt_src, float* out,
                    int32_t nt_dst, double dt_dst, void* stream) {
  if (nlead <= 0 || nt_src <= 0 || m <= 0 || nt_dst <= 0 || !y || !out || !(dt_src > 0) || !(dt_dst > 0))
    return PAT_EINVAL;
  const int64_t n = (int64_t)nlead * nt_dst * m;
  hipLaunchKernelGGL(k_time_interp, dim3(grid_blocks(n)), dim3(256), 0, static_cast<hipStream_t>(stream), nlead,
                     nt_src, m, y, dt_src, out, nt_dst, dt_dst);
  return last_error();
}

size_t pat_lbfgs_scratch_bytes(int32_t npairs) {
  return (size_t)(RED_BLOCKS + 2 * std::max(npairs, 0) + 2) * sizeof(double);
}

static int dot_into(hipStream_t st, int64_t n, const float* a, const float* b, double* partial, double* out) {
  hipLaunchKernelGGL(k_dot_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, a, b, n, partial);
  PAT_TRY(last_error());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, out, 1.0);
  return last_error();
}

int pat_absmax(int64_t n, const float* x, double* out, void* scratch, void* stream) {
  if (n <= 0 || !x || !out || !scratch) return PAT_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(scratch);
  hipLaunchKernelGGL(k_absmax_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, x, n, partial);
  PAT_TRY(last_error());
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, out);
  return last_error();
}

int pat_dot(int64_t n, const float* a, const float* b, double* out, void* scratch, void* stream) {
  if (n <= 0 || !a || !b || !out || !scratch) return PAT_EINVAL;
  return dot_into(static_cast<hipStream_t>(stream), n, a, b, static_cast<double*>(scratch), out);
}

}  // extern "C"

namespace {

// Alg. 1 on the stream, with `scr` holding pat_lbfgs_scratch_bytes(np) bytes.
int lbfgs_two_loop(hipStream_t st, int64_t n, const float* g, int32_t np, const float* const* s,
                   const float* const* y, float* d, double* scr) {
  double* partial = scr;
  double* sc = partial + RED_BLOCKS;
  if (d != g) PAT_TRY(copy_dev(st, g, d, (size_t)n * sizeof(float)));
  if (np == 0) return PAT_OK;
  const int blocks = grid_blocks(n);
  for (int j = 0; j < np; ++j) PAT_TRY(dot_into(st, n, y[j], s[j], partial, sc + j));
  for (int j = np - 1; j >= 0; --j) {
    PAT_TRY(dot_into(st, n, s[j], d, partial, sc + 2 * np));
    hipLaunchKernelGGL(k_lbfgs_loop1, dim3(blocks), dim3(256), 0, st, n, d, y[j], sc, np, j);
    PAT_TRY(last_error());
  }
  PAT_TRY(dot_into(st, n, y[np - 1], y[np - 1], partial, sc + 2 * np + 1));
  hipLaunchKernelGGL(k_lbfgs_h0, dim3(blocks), dim3(256), 0, st, n, d, sc, np);
  PAT_TRY(last_error());
  for (int j = 0; j < np; ++j) {
    PAT_TRY(dot_into(st, n, y[j], d, partial, sc + 2 * np));
    hipLaunchKernelGGL(k_lbfgs_loop2, dim3(blocks), dim3(256), 0, st, n, d, s[j], sc, np, j);
    PAT_TRY(last_error());
  }
  return PAT_OK;
}

int lbfgs_args_ok(int64_t n, const float* g, int32_t np, const float* const* s, const float* const* y,
                  const float* d) {
  if (n <= 0 || !g || !d || np < 0 || (np > 0 && (!s || !y))) return PAT_EINVAL;
  for (int j = 0; j < np; ++j)
    if (!s[j] || !y[j]) return PAT_EINVAL;
  return PAT_OK;
}

// ----------------------------------------------------------------------------
// Library-owned scratch of the allocation-free two-loop recursion: one static
// device array (every GPU that runs the library holds its own copy for the
// life of the process).  Host code never passes the array's name to a kernel:
// its device address on the current GPU comes from hipGetSymbolAddress, taken
// once per device and kept.
// ----------------------------------------------------------------------------
namespace noalloc {
constexpr int kMaxDevices = 64;
constexpr size_t kDoubles = RED_BLOCKS + 2 * PAT_LBFGS_NOALLOC_MAX_PAIRS + 2;
static __device__ __align__(256) double scratch[kDoubles];
std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PAT_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PAT_EHIP;
    g_addr[dev] = static_cast<double*>(ptr);
  }
  *out = g_addr[dev];
  return PAT_OK;
}
}  // namespace noalloc

}  // namespace

extern "C" {

int pat_lbfgs_direction(int64_t n, const float* g, int32_t np, const float* const* s, const float* const* y, float* d,
                        void* scratch, void* stream) {
  PAT_TRY(lbfgs_args_ok(n, g, np, s, y, d));
  if (!scratch) return PAT_EINVAL;
  return lbfgs_two_loop(static_cast<hipStream_t>(stream), n, g, np, s, y, d, static_cast<double*>(scratch));
}

int pat_lbfgs_direction_noalloc(int64_t n, const float* g, int32_t np, const float* const* s,
                                const float* const* y, float* d, void* stream) {
  PAT_TRY(lbfgs_args_ok(n, g, np, s, y, d));
  if (np > PAT_LBFGS_NOALLOC_MAX_PAIRS) return PAT_EUNSUPPORTED;
  double* scr = nullptr;
  PAT_TRY(noalloc::scratch_address(&scr));
  return lbfgs_two_loop(static_cast<hipStream_t>(stream), n, g, np, s, y, d, scr);
}

int pat_plan_set_tile(pat_plan* p, int32_t col_tile) {
  if (!p || (col_tile != 0 && col_tile != 8)) return PAT_EINVAL;
  if (col_tile != p->col_tile) {   // captured graphs hold the old kernels
    drop_graphs(p);
    p->col_tile = col_tile;
  }
  return PAT_OK;
}

int pat_plan_set_col_order(pat_plan* p, int32_t order) {
  if (!p || order < 0 || order > 2) return PAT_EINVAL;
  if (order != p->col_order) {   // captured graphs hold the old kernels
    drop_graphs(p);
    p->col_order = order;
  }
  return PAT_OK;
}

int pat_batch_release(void) {
  int status = PAT_OK;
  batch_free(g_batch);
  g_batch = nullptr;
  for (hipStream_t s : g_pool) {
    if (hipStreamSynchronize(s) != hipSuccess || hipStreamDestroy(s) != hipSuccess) status = PAT_EHIP;
  }
  g_pool.clear();
  return status;
}

int pat_batch_gradient(int32_t nprob, const pat_problem* probs, int32_t nstreams, void* stream) {
  if (nprob <= 0 || !probs || nstreams <= 0 || nstreams > 16) return PAT_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t sig = 1469598103934665603ull;
  sig = fnv(sig, &nstreams, sizeof(nstreams));
  for (int i = 0; i < nprob; ++i) {
    const pat_problem& pr = probs[i];
    if (!pr.plan || !pr.c || !pr.p0 || !pr.y || !pr.w || !pr.data || !pr.resid || !pr.J || !pr.g_p0 || !pr.g_c ||
        !pr.ws)
      return PAT_EINVAL;
    for (int j = 0; j < i; ++j)
      if (probs[j].plan == pr.plan || probs[j].ws == pr.ws) return PAT_EINVAL;   // one job per plan and workspace
    if (pr.ws_bytes < make_layout(pr.plan, 0).total) return PAT_EWORKSPACE;
    sig = fnv(sig, &pr, sizeof(pr));
    sig = fnv(sig, &pr.plan->tb, sizeof(Tables));
    sig = fnv(sig, &pr.plan->g, sizeof(pat_grid));
    const int shape[3] = {pr.plan->K, pr.plan->kb, pr.plan->fast ? 1 : 0};
    sig = fnv(sig, shape, sizeof(shape));
  }
  if (!g_batch || g_batch->sig != sig) {   // a new set of problems: new slot tables and graphs
    batch_free(g_batch);
    g_batch = new (std::nothrow) BatchContext();
    if (!g_batch) return PAT_EHIP;
    g_batch->sig = sig;
    const int sb = batch_build(g_batch, nprob, probs, nstreams);
    if (sb != PAT_OK) {
      batch_free(g_batch);
      g_batch = nullptr;
      return sb;
    }
  }
  BatchContext* ctx = g_batch;
  for (auto& b : ctx->probs) b.pr.plan->recorded = false;   // the batch overwrites every workspace
  int ns = 0;
  for (const auto& cl : ctx->classes) ns = std::max(ns, cl.stream + 1);
  PAT_TRY(pool_streams(ns));
  // fork: every class stream waits for the work already queued on the caller's stream
  hipEvent_t fork;
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return PAT_EHIP;
  std::vector<hipEvent_t> done((size_t)ns, nullptr);
  int status = PAT_OK;
  if (hipEventRecord(fork, st) != hipSuccess) status = PAT_EHIP;
  for (int s = 0; s < ns && status == PAT_OK; ++s)
    if (hipStreamWaitEvent(g_pool[s], fork, 0) != hipSuccess) status = PAT_EHIP;
  for (const auto& cl : ctx->classes) {
    if (status != PAT_OK) break;
    status = batch_class(ctx, cl, g_pool[cl.stream]);
  }
  // join: the caller's stream waits for every class stream
  for (int s = 0; s < ns; ++s) {
    if (hipEventCreateWithFlags(&done[s], hipEventDisableTiming) != hipSuccess) {
      status = PAT_EHIP;
      continue;
    }
    if (hipEventRecord(done[s], g_pool[s]) != hipSuccess || hipStreamWaitEvent(st, done[s], 0) != hipSuccess)
      status = PAT_EHIP;
  }
  (void)hipEventDestroy(fork);
  for (auto e : done)
    if (e) (void)hipEventDestroy(e);
  return status;
}

int pat_trace_start(int32_t every) {
  if (every <= 0) return PAT_EINVAL;
  if (!g_trace.created) {
    g_trace.ev.resize((size_t)PAT_PASS_KINDS * kTraceCap * 2);
    for (auto& e : g_trace.ev)
      if (hipEventCreate(&e) != hipSuccess) return PAT_EHIP;
    g_trace.created = true;
  }
  for (int k = 0; k < PAT_PASS_KINDS; ++k) {
    g_trace.seen[k] = 0;
    g_trace.used[k] = 0;
  }
  g_trace.every = every;
  g_trace.on = true;
  return PAT_OK;
}

int pat_trace_stop(void) {
  g_trace.on = false;
  return PAT_OK;
}

int pat_trace_read(int32_t kind, int64_t* count, double* total_ms) {
  if (kind < 0 || kind >= PAT_PASS_KINDS || !count || !total_ms) return PAT_EINVAL;
  double tot = 0.0;
  for (int i = 0; i < g_trace.used[kind]; ++i) {
    float ms = 0.f;
    hipEvent_t a = g_trace.ev[((size_t)kind * kTraceCap + i) * 2];
    hipEvent_t b = g_trace.ev[((size_t)kind * kTraceCap + i) * 2 + 1];
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) return PAT_EHIP;
    tot += ms;
  }
  *count = g_trace.used[kind];
  *total_ms = tot;
  return PAT_OK;
}


int pat_ou_create(int32_t ny, int32_t nx, double dx, double tau, const uint8_t* mask, pat_ou** out) {
  if (!out || ny <= 0 || nx <= 0 || !(dx > 0.0) || !(tau > 0.0)) return PAT_EINVAL;
  *out = nullptr;
  // bounding box of the mask
  int y0 = ny, y1 = -1, x0 = nx, x1 = -1;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      if (!mask || mask[(size_t)y * nx + x]) {
        y0 = std::min(y0, y); y1 = std::max(y1, y); x0 = std::min(x0, x); x1 = std::max(x1, x);
      }
  if (y1 < 0) return PAT_EINVAL;   // empty mask
  const int nby = y1 - y0 + 1, nbx = x1 - x0 + 1;
  const int need = 2 * std::max(nby, nbx) - 1;
  static const int sizes[] = {32, 36, 40, 48, 64, 81, 84, 96, 125, 128, 160, 175, 192, 243, 256, 375, 384, 512};
  int L = 0;
  for (int cand : sizes)
    if (cand >= need) { L = cand; break; }
  if (!L) return PAT_EUNSUPPORTED;
  // twiddles and the spectrum of the kernel on the wrapped offsets (float64 cosine sums:
  // the embedded kernel is even along both axes, so its DFT is real)
  std::vector<float2> tw((size_t)L);
  std::vector<double> cosv((size_t)L);
  for (int j = 0; j < L; ++j) {
    tw[j] = make_float2((float)std::cos(2 * M_PI * j / L), (float)-std::sin(2 * M_PI * j / L));
    cosv[j] = std::cos(2 * M_PI * j / L);
  }
  std::vector<double> e((size_t)L * L), A((size_t)L * L, 0.0), S((size_t)L * L, 0.0);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const double dy = std::min(y, L - y), dxw = std::min(x, L - x);
      e[(size_t)y * L + x] = std::exp(-dx * std::sqrt(dy * dy + dxw * dxw) / tau);
    }
  for (int y = 0; y < L; ++y)
    for (int k = 0; k < L; ++k) {
      double acc = 0.0;
      for (int x = 0; x < L; ++x) acc += e[(size_t)y * L + x] * cosv[((size_t)k * x) % L];
      A[(size_t)y * L + k] = acc;
    }
  for (int ky = 0; ky < L; ++ky)
    for (int kx = 0; kx < L; ++kx) {
      double acc = 0.0;
      for (int y = 0; y < L; ++y) acc += A[(size_t)y * L + kx] * cosv[((size_t)ky * y) % L];
      S[(size_t)ky * L + kx] = acc;
    }
  double smax = 0.0;
  for (double v : S) smax = std::max(smax, v);
  std::vector<float> sop((size_t)L * L), spre((size_t)L * L);
  for (size_t i = 0; i < S.size(); ++i) {
    sop[i] = (float)S[i];
    spre[i] = (float)(1.0 / std::max(S[i], 1e-6 * smax));
  }
  std::vector<uint8_t> bm((size_t)nby * nbx);
  for (int y = 0; y < nby; ++y)
    for (int x = 0; x < nbx; ++x) bm[(size_t)y * nbx + x] = !mask || mask[(size_t)(y0 + y) * nx + x0 + x] ? 1 : 0;
  const size_t o_tw = 0, o_op = align256(L * sizeof(float2)), o_pre = o_op + align256((size_t)L * L * 4),
               o_m = o_pre + align256((size_t)L * L * 4), total = o_m + align256(bm.size());
  pat_ou* o = new (std::nothrow) pat_ou();
  if (!o) return PAT_EHIP;
  if (hipMalloc(&o->dev, total) != hipSuccess) {
    delete o;
    return PAT_EHIP;
  }
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + o_tw, tw.data(), tw.size() * sizeof(float2));
  std::memcpy(host.data() + o_op, sop.data(), sop.size() * 4);
  std::memcpy(host.data() + o_pre, spre.data(), spre.size() * 4);
  std::memcpy(host.data() + o_m, bm.data(), bm.size());
  if (hipMemcpy(o->dev, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(o->dev);
    delete o;
    return PAT_EHIP;
  }
  char* d = static_cast<char*>(o->dev);
  o->tw = reinterpret_cast<float2*>(d + o_tw);
  o->s_op = reinterpret_cast<float*>(d + o_op);
  o->s_pre = reinterpret_cast<float*>(d + o_pre);
  o->mask = reinterpret_cast<uint8_t*>(d + o_m);
  o->ny = ny; o->nx = nx; o->oy = y0; o->ox = x0; o->nby = nby; o->nbx = nbx; o->L = L;
  *out = o;
  return PAT_OK;
}

int pat_ou_destroy(pat_ou* o) {
  if (!o) return PAT_EINVAL;
  if (o->dev) (void)hipFree(o->dev);
  delete o;
  return PAT_OK;
}

int pat_ou_scratch_bytes(const pat_ou* o, int32_t nvec, size_t* bytes) {
  if (!o || nvec <= 0 || !bytes) return PAT_EINVAL;
  *bytes = ou_layout(o, nvec).total;
  return PAT_OK;
}

int pat_ou_apply(pat_ou* o, int32_t nvec, const float* v, float* out, void* scratch, size_t scratch_bytes,
                 void* stream) {
  if (!o || nvec <= 0 || !v || !out || !scratch) return PAT_EINVAL;
  const OuLayout L = ou_layout(o, nvec);
  if (scratch_bytes < L.total) return PAT_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(scratch);
  float* b = reinterpret_cast<float*>(ws + L.b);
  float* y = reinterpret_cast<float*>(ws + L.x);
  const int64_t n = (int64_t)nvec * o->nby * o->nbx;
  hipLaunchKernelGGL(ou::k_gather, dim3(grid_blocks(n)), dim3(256), 0, st, v, nvec, o->ny, o->nx, o->oy, o->ox,
                     o->nby, o->nbx, o->mask, 0.0f, nullptr, b);
  PAT_TRY(last_error());
  PAT_TRY(ou_circ(o, st, nvec, b, o->s_op, reinterpret_cast<float2*>(ws + L.W), y));
  const int64_t ng = (int64_t)nvec * o->ny * o->nx;
  hipLaunchKernelGGL(ou::k_scatter, dim3(grid_blocks(ng)), dim3(256), 0, st, y, nvec, o->ny, o->nx, o->oy, o->ox,
                     o->nby, o->nbx, nullptr, out);
  return last_error();
}

int pat_ou_prior(pat_ou* o, int32_t nvec, const float* z, const float* eta, const float* inv_var, float* grad,
                 double* J, double tol, int32_t maxit, void* scratch, size_t scratch_bytes, int32_t* iters,
                 void* stream) {
  if (!o || nvec <= 0 || !z || !eta || !inv_var || !grad || !J || !scratch || !(tol > 0.0) || maxit <= 0)
    return PAT_EINVAL;
  const OuLayout L = ou_layout(o, nvec);
  if (scratch_bytes < L.total) return PAT_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(scratch);
  float* b = reinterpret_cast<float*>(ws + L.b);
  float* x = reinterpret_cast<float*>(ws + L.x);
  const int64_t n = (int64_t)nvec * o->nby * o->nbx;
  hipLaunchKernelGGL(ou::k_gather, dim3(grid_blocks(n)), dim3(256), 0, st, z, nvec, o->ny, o->nx, o->oy, o->ox,
                     o->nby, o->nbx, o->mask, 1.0f, eta, b);
  PAT_TRY(last_error());
  int it = 0;
  PAT_TRY(ou_pcg(o, st, nvec, ws, L, tol, maxit, &it));
  if (iters) *iters = it;
  // J = sum_v 1/2 inv_var_v (b_v . x_v); grad = inv_var_v x_v on the grid
  double* dots = reinterpret_cast<double*>(ws + L.dots);
  PAT_TRY(ou_dots(o, st, nvec, b, x, reinterpret_cast<double*>(ws + L.partial), dots));
  hipLaunchKernelGGL(k_ou_energy, dim3(1), dim3(64), 0, st, dots, inv_var, nvec, J);
  PAT_TRY(last_error());
  const int64_t ng = (int64_t)nvec * o->ny * o->nx;
  hipLaunchKernelGGL(ou::k_scatter, dim3(grid_blocks(ng)), dim3(256), 0, st, x, nvec, o->ny, o->nx, o->oy, o->ox,
                     o->nby, o->nbx, inv_var, grad);
  return last_error();
}

}  // extern "C"
