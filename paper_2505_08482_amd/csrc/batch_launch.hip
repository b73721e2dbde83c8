// batch_launch.hip — launchers of the batched passes (batch_kernels.hpp), in a
// translation unit of their own so that their template instantiations compile
// beside the rest of the library.
#include <hip/hip_runtime.h>

#include "batch_kernels.hpp"

namespace pat {
namespace {

#define PAT_BATCH_FAST(X) X(32) X(64) X(128) X(256) X(512)
// every length of the any-radix family (also power-of-two sides of
// non-square grids, and power-of-two grids run with that family)
#define PAT_BATCH_GENERIC(X)                                                                              \
  X(32) X(36) X(40) X(48) X(64) X(81) X(84) X(96) X(125) X(128) X(160) X(175) X(192) X(243) X(256) X(375) \
  X(384) X(512) X(768)

int launched() { return hipGetLastError() == hipSuccess ? 0 : -4; }

template <int MODE>
int col(bool fast_family, int ny, const BatchSlot* s, int ns, int blocks, hipStream_t st) {
  if (fast_family) {
    switch (ny) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    hipLaunchKernelGGL((fast::kb_col<N, MODE, fast::Cfg<N>::TC, false>), dim3(blocks),                      \
                       dim3(fast::Cfg<N>::TC * fast::Cfg<N>::T), 0, st, s, ns);                             \
    return launched();
      PAT_BATCH_FAST(X)
#undef X
      default: return -2;
    }
  }
  switch (ny) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    hipLaunchKernelGGL((kb_gcol<N, MODE>), dim3(blocks), dim3(ColCfg<N>::BLOCK), 0, st, s, ns);              \
    return launched();
    PAT_BATCH_GENERIC(X)
#undef X
    default: return -2;
  }
}

}  // namespace

int batch_launch_col(int mode, bool fast_family, int ny, const BatchSlot* s, int ns, int blocks, hipStream_t st) {
  switch (mode) {
    case COL_GRAD1: return col<COL_GRAD1>(fast_family, ny, s, ns, blocks, st);
    case COL_PAIRP: return col<COL_PAIRP>(fast_family, ny, s, ns, blocks, st);
    case COL_PAIRM: return col<COL_PAIRM>(fast_family, ny, s, ns, blocks, st);
    case COL_SUMM: return col<COL_SUMM>(fast_family, ny, s, ns, blocks, st);
    default: return -2;
  }
}

int batch_launch_row(int kind, bool fast_family, int nx, const BatchSlot* s, int ns, int blocks, hipStream_t st) {
  if (fast_family) {
    switch (nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    if (kind == BK_FWD_U) hipLaunchKernelGGL(fast::kb_fwd_u<N>, dim3(blocks), dim3(64), 0, st, s, ns);        \
    else if (kind == BK_FWD_RHO) hipLaunchKernelGGL(fast::kb_fwd_rho<N>, dim3(blocks), dim3(64), 0, st, s, ns); \
    else hipLaunchKernelGGL(fast::kb_adj_u<N>, dim3(blocks), dim3(64), 0, st, s, ns);                         \
    return launched();
      PAT_BATCH_FAST(X)
#undef X
      default: return -2;
    }
  }
  switch (nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    if (kind == BK_FWD_U) hipLaunchKernelGGL(kb_gfwd_u<N>, dim3(blocks), dim3(256), 0, st, s, ns);            \
    else if (kind == BK_FWD_RHO) hipLaunchKernelGGL(kb_gfwd_rho<N>, dim3(blocks), dim3(256), 0, st, s, ns);   \
    else hipLaunchKernelGGL(kb_gadj_u<N>, dim3(blocks), dim3(256), 0, st, s, ns);                             \
    return launched();
    PAT_BATCH_GENERIC(X)
#undef X
    default: return -2;
  }
}

int batch_launch_adj_rho(bool fast_family, int nx, int kb, const BatchSlot* s, int ns, int blocks, hipStream_t st) {
  if (fast_family) {
    switch (nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    switch (kb) {                                                                                             \
      case 8: hipLaunchKernelGGL((fast::kb_adj_rho<N, 8>), dim3(blocks), dim3(512), 0, st, s, ns); break;     \
      case 4: hipLaunchKernelGGL((fast::kb_adj_rho<N, 4>), dim3(blocks), dim3(256), 0, st, s, ns); break;     \
      case 2: hipLaunchKernelGGL((fast::kb_adj_rho<N, 2>), dim3(blocks), dim3(128), 0, st, s, ns); break;     \
      default: hipLaunchKernelGGL((fast::kb_adj_rho<N, 1>), dim3(blocks), dim3(64), 0, st, s, ns); break;     \
    }                                                                                                         \
    return launched();
      PAT_BATCH_FAST(X)
#undef X
      default: return -2;
    }
  }
  switch (nx) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    hipLaunchKernelGGL(kb_gadj_rho<N>, dim3(blocks), dim3(256), 0, st, s, ns);                               \
    return launched();
    PAT_BATCH_GENERIC(X)
#undef X
    default: return -2;
  }
}

}  // namespace pat
