// batch_slot.hpp — one problem of a batched launch (batch_kernels.hpp): the
// host fills these, the batched kernels read them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave_kernels.hpp"

namespace pat {

// One problem of a batched launch.
struct BatchSlot {
  Tables tb;
  // forward state (as in a single-problem forward solve)
  const float* c;
  float *ux, *uy, *rx, *ry;
  float2 *SA, *SB;
  float* hist_base;
  float* dpart;
  // adjoint state
  const float* resid;
  float *uhx, *uhy, *rhx, *rhy, *gck;
  float2 *SC, *SD;
  StepCtl* ctl;
  float sc_grad;      // dt / rho0 / (nx ny): gradient and divergence-sum column passes
  float sc_div;       // dt rho0 / (nx ny): the other two column passes
  int32_t b_col;      // first block of this problem in a column-pass launch
  int32_t b_row;      // ... in a row-pass launch
  int32_t b_adj;      // ... in an adjoint-density launch (its group of slots)
  int32_t pad;
};

// Launch one batched pass over `ns` slots (`blocks` blocks in all) on `st`
// (batch_launch.hip).  mode: a column-pass mode of wave_kernels.hpp; kind:
// BK_FWD_U, BK_FWD_RHO or BK_ADJ_U; kb: datasets per block of the adjoint
// density pass (power-of-two family).  Returns 0, or -2 for a size without
// batched kernels, or -4 for a launch error.
enum BatchRowKind { BK_FWD_U = 0, BK_FWD_RHO = 1, BK_ADJ_U = 2 };
int batch_launch_col(int mode, bool fast, int ny, const BatchSlot* s, int ns, int blocks, hipStream_t st);
int batch_launch_row(int kind, bool fast, int nx, const BatchSlot* s, int ns, int blocks, hipStream_t st);
int batch_launch_adj_rho(bool fast, int nx, int kb, const BatchSlot* s, int ns, int blocks, hipStream_t st);

}  // namespace pat
