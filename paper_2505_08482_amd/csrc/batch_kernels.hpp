// batch_kernels.hpp — one launch advances many independent problems.
//
// Problems of one transform family and grid size share a launch: the blocks
// of a launch are the concatenation of every problem's blocks (in problem
// order), each problem described by a slot in device memory (its tables, its
// state and spectra, its step counters, and where its blocks start in each
// kind of launch).  A block finds its slot by a scan over the slots' block
// starts (uniform: scalar loads) and runs the same device body as the
// single-problem kernel, with its block index relative to its problem, so a
// problem computes exactly the bits it computes alone.  The datasets of a
// problem share c (eq. (2)); different problems share nothing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_slot.hpp"
#include "fast_kernels.hpp"
#include "wave_kernels.hpp"

namespace pat {

// Device view of a slot with every pointer in the global address space: a
// pointer loaded from memory is otherwise generic and its loads and stores
// become flat instructions; converted back to the bodies' plain pointers, the
// compiler still knows they address global memory.
#define PAT_GLOBAL __attribute__((address_space(1)))
struct TablesG {
  const float2 PAT_GLOBAL *tw_x, *tw_y, *ex_p, *ex_m, *ey_p, *ey_m;
  const float PAT_GLOBAL *kappa, *ax, *asx, *ax2, *asx2, *wfx, *ay, *asy, *ay2, *asy2, *wfy;
  const int32_t PAT_GLOBAL* g_row_start;
  const GatherEnt PAT_GLOBAL* g_ent;
  const int32_t PAT_GLOBAL* s_row_start;
  const ScatterPix PAT_GLOBAL* s_pix;
  const ScatterTap PAT_GLOBAL* s_tap;
  int32_t nx, ny, nh, K, m, nt;
};
struct BatchSlotG {
  TablesG tb;
  const float PAT_GLOBAL* c;
  float PAT_GLOBAL *ux, *uy, *rx, *ry;
  float2 PAT_GLOBAL *SA, *SB;
  float PAT_GLOBAL* hist_base;
  float PAT_GLOBAL* dpart;
  const float PAT_GLOBAL* resid;
  float PAT_GLOBAL *uhx, *uhy, *rhx, *rhy, *gck;
  float2 PAT_GLOBAL *SC, *SD;
  StepCtl PAT_GLOBAL* ctl;
  float sc_grad, sc_div;
  int32_t b_col, b_row, b_adj, pad;
};
static_assert(sizeof(TablesG) == sizeof(Tables), "device view of Tables");
static_assert(sizeof(BatchSlotG) == sizeof(BatchSlot), "device view of BatchSlot");

// A slot in registers with plain pointers (as the single-problem kernels see
// their arguments).
struct SlotView {
  Tables tb;
  const float* c;
  float *ux, *uy, *rx, *ry;
  float2 *SA, *SB;
  float* hist_base;
  float* dpart;
  const float* resid;
  float *uhx, *uhy, *rhx, *rhy, *gck;
  float2 *SC, *SD;
  StepCtl* ctl;
  float sc_grad, sc_div;
  int32_t b_col, b_row, b_adj;
};

#define PAT_P(T, x) ((T)(x))
__device__ __forceinline__ SlotView load_slot(const BatchSlot* __restrict__ s, int j) {
  const BatchSlotG g = reinterpret_cast<const BatchSlotG*>(s)[j];
  SlotView v;
  v.tb.tw_x = PAT_P(const float2*, g.tb.tw_x); v.tb.tw_y = PAT_P(const float2*, g.tb.tw_y);
  v.tb.ex_p = PAT_P(const float2*, g.tb.ex_p); v.tb.ex_m = PAT_P(const float2*, g.tb.ex_m);
  v.tb.ey_p = PAT_P(const float2*, g.tb.ey_p); v.tb.ey_m = PAT_P(const float2*, g.tb.ey_m);
  v.tb.kappa = PAT_P(const float*, g.tb.kappa);
  v.tb.ax = PAT_P(const float*, g.tb.ax); v.tb.asx = PAT_P(const float*, g.tb.asx);
  v.tb.ax2 = PAT_P(const float*, g.tb.ax2); v.tb.asx2 = PAT_P(const float*, g.tb.asx2);
  v.tb.wfx = PAT_P(const float*, g.tb.wfx);
  v.tb.ay = PAT_P(const float*, g.tb.ay); v.tb.asy = PAT_P(const float*, g.tb.asy);
  v.tb.ay2 = PAT_P(const float*, g.tb.ay2); v.tb.asy2 = PAT_P(const float*, g.tb.asy2);
  v.tb.wfy = PAT_P(const float*, g.tb.wfy);
  v.tb.g_row_start = PAT_P(const int32_t*, g.tb.g_row_start);
  v.tb.g_ent = PAT_P(const GatherEnt*, g.tb.g_ent);
  v.tb.s_row_start = PAT_P(const int32_t*, g.tb.s_row_start);
  v.tb.s_pix = PAT_P(const ScatterPix*, g.tb.s_pix);
  v.tb.s_tap = PAT_P(const ScatterTap*, g.tb.s_tap);
  v.tb.nx = g.tb.nx; v.tb.ny = g.tb.ny; v.tb.nh = g.tb.nh; v.tb.K = g.tb.K; v.tb.m = g.tb.m; v.tb.nt = g.tb.nt;
  v.c = PAT_P(const float*, g.c);
  v.ux = PAT_P(float*, g.ux); v.uy = PAT_P(float*, g.uy); v.rx = PAT_P(float*, g.rx); v.ry = PAT_P(float*, g.ry);
  v.SA = PAT_P(float2*, g.SA); v.SB = PAT_P(float2*, g.SB);
  v.hist_base = PAT_P(float*, g.hist_base);
  v.dpart = PAT_P(float*, g.dpart);
  v.resid = PAT_P(const float*, g.resid);
  v.uhx = PAT_P(float*, g.uhx); v.uhy = PAT_P(float*, g.uhy);
  v.rhx = PAT_P(float*, g.rhx); v.rhy = PAT_P(float*, g.rhy); v.gck = PAT_P(float*, g.gck);
  v.SC = PAT_P(float2*, g.SC); v.SD = PAT_P(float2*, g.SD);
  v.ctl = PAT_P(StepCtl*, g.ctl);
  v.sc_grad = g.sc_grad; v.sc_div = g.sc_div;
  v.b_col = g.b_col; v.b_row = g.b_row; v.b_adj = g.b_adj;
  return v;
}
#undef PAT_P

enum BatchRange { BR_COL = 0, BR_ROW = 1, BR_ADJ = 2 };

template <int R>
__device__ __forceinline__ int32_t range_start(const BatchSlot& s) {
  return R == BR_COL ? s.b_col : (R == BR_ROW ? s.b_row : s.b_adj);
}

// Slot of block `bid`: the last slot whose range starts at or before it.
template <int R>
__device__ __forceinline__ int slot_of(const BatchSlot* __restrict__ s, int ns, int bid) {
  int j = 0;
  while (j + 1 < ns && range_start<R>(s[j + 1]) <= bid) ++j;
  return j;
}

// ---------------------------------------------------------------------------
// Power-of-two family (fast_kernels.hpp)
// ---------------------------------------------------------------------------
namespace fast {

template <int N, int MODE, int TC, bool SEQ>
__global__ __launch_bounds__(TC * Cfg<N>::T) void kb_col(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_COL>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  constexpr bool FWD = MODE == COL_GRAD1 || MODE == COL_PAIRM;
  constexpr bool FIRST = MODE == COL_GRAD1 || MODE == COL_SUMM;   // first pass of a step
  int32_t* step = MODE == COL_GRAD1 ? &sl.ctl->fwd_n : (MODE == COL_SUMM ? &sl.ctl->adj_n : nullptr);
  fast::k_col_body<N, MODE, TC, SEQ>(blockIdx.x - sl.b_col, sl.tb, FWD ? sl.SA : sl.SC, FWD ? sl.SB : sl.SD,
                               FIRST ? sl.sc_grad : sl.sc_div, step, MODE == COL_GRAD1 ? +1 : -1);
}

template <int N>
__global__ __launch_bounds__(64) void kb_fwd_u(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  fast::k_fwd_u_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.ux, sl.uy, sl.SA, sl.SB, sl.ctl);
}

template <int N>
__global__ __launch_bounds__(64) void kb_fwd_rho(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  fast::k_fwd_rho_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.c, sl.rx, sl.ry, sl.hist_base, sl.dpart, sl.SA, sl.SB,
                    sl.ctl);
}

template <int N, int KB>
__global__ __launch_bounds__(64 * KB) void kb_adj_rho(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ADJ>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  fast::k_adj_rho_body<N, KB>(blockIdx.x - sl.b_adj, sl.tb, sl.c, sl.hist_base, sl.resid, sl.rhx, sl.rhy, sl.gck, sl.SC,
                        sl.SD, sl.ctl);
}

template <int N>
__global__ __launch_bounds__(64) void kb_adj_u(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  fast::k_adj_u_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.uhx, sl.uhy, sl.SC, sl.SD, sl.ctl);
}

}  // namespace fast

// ---------------------------------------------------------------------------
// Any-radix family (wave_kernels.hpp)
// ---------------------------------------------------------------------------
template <int N, int MODE>
__global__ __launch_bounds__(ColCfg<N>::BLOCK) void kb_gcol(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_COL>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  constexpr bool FWD = MODE == COL_GRAD1 || MODE == COL_PAIRM;
  constexpr bool FIRST = MODE == COL_GRAD1 || MODE == COL_SUMM;
  int32_t* step = MODE == COL_GRAD1 ? &sl.ctl->fwd_n : (MODE == COL_SUMM ? &sl.ctl->adj_n : nullptr);
  pat::k_col_body<N, MODE>(blockIdx.x - sl.b_col, sl.tb, FWD ? sl.SA : sl.SC, FWD ? sl.SB : sl.SD,
                      FIRST ? sl.sc_grad : sl.sc_div, step, MODE == COL_GRAD1 ? +1 : -1);
}

template <int N>
__global__ __launch_bounds__(256) void kb_gfwd_u(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  pat::k_fwd_u_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.ux, sl.uy, sl.SA, sl.SB, sl.ctl);
}

template <int N>
__global__ __launch_bounds__(256) void kb_gfwd_rho(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  pat::k_fwd_rho_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.c, sl.rx, sl.ry, sl.hist_base, sl.dpart, sl.SA, sl.SB,
                    sl.ctl);
}

template <int N>
__global__ __launch_bounds__(256) void kb_gadj_rho(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ADJ>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  pat::k_adj_rho_body<N>(blockIdx.x - sl.b_adj, sl.tb, sl.c, sl.hist_base, sl.resid, sl.rhx, sl.rhy, sl.gck, sl.SC,
                    sl.SD, sl.ctl);
}

template <int N>
__global__ __launch_bounds__(256) void kb_gadj_u(const BatchSlot* __restrict__ s, int ns) {
  const int j = slot_of<BR_ROW>(s, ns, blockIdx.x);
  const SlotView sl = load_slot(s, j);
  pat::k_adj_u_body<N>(blockIdx.x - sl.b_row, sl.tb, sl.uhx, sl.uhy, sl.SC, sl.SD, sl.ctl);
}

}  // namespace pat
