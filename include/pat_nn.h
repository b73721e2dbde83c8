/*
 * pat_nn.h — C ABI of the learned fine-level start (libpat.so, gfx950).
 *
 * Sec. 3.1 starts every finer multigrid level from the coarse iterate,
 * linearly interpolated.  The learned start proposes the sound speed of the
 * finest level instead: a small U-Net reads the coarse sound speed and the
 * summed initial-pressure gradient (interpolated onto the fine grid) and adds a
 * correction to the interpolated sound speed; plain gradient iterations then
 * continue from it (and remain the fallback).  The network is not part of the
 * paper; these calls are its layers, forward and backward, and the training
 * update, so that it is trained on the GPU by the library's own kernels.
 *
 * Conventions (beyond those of pat.h, whose status codes these calls return):
 *  - "bf16" arrays are uint16_t holding bfloat16 values (the upper 16 bits of
 *    an IEEE float32, rounded to nearest even).  Dense contractions multiply
 *    bf16 operands on the matrix cores and accumulate in float32.
 *  - Activations are channels-last: [B][H][W][ld] with the C channels of an
 *    operand starting at the pointer given (a channel slice of a wider buffer,
 *    e.g. one half of a concatenation).  C, ld and every slice offset must be
 *    multiples of 8 and activation / weight pointers 16-byte aligned.
 *  - Convolution weights are [cout][9][cin], tap t = 3 (di + 1) + (dj + 1) for
 *    the input offset (di, dj) in {-1, 0, 1}^2 (row, column); zero padding.
 *  - All pointers are DEVICE pointers owned by the caller; calls are
 *    asynchronous on `stream` and deterministic (no floating-point atomics).
 */
#ifndef PAT_NN_H
#define PAT_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 3x3 convolution, zero padding, same size:
 *   v[p][o] = sum_{t,c} x[p + offset_t][c] w[o][t][c] (+ bias[o] if bias),
 *   v = max(v, 0) if relu;  v += y[p][o] if accumulate (the old bf16 value);
 *   v = 0 where mask[p][o] <= 0 if mask (mask [B*H*W][ldm], bf16);  y = bf16(v).
 * x: [B*H*W][ldx] bf16 (cin channels), y: [B*H*W][ldy] bf16 (cout channels).
 * The forward layer uses bias and relu; the data gradient of a layer is this
 * call on the gradient of its output with the weights from
 * pat_nn_conv3x3_flip and, when its input is a ReLU output, that input as mask.
 * Requires cin % 8 == 0, cout >= 1, B, H, W >= 1, ldx >= cin, ldy >= cout.
 * y must not overlap x. */
int pat_nn_conv3x3(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t ldx, int32_t cin,
                   const uint16_t* w, const float* bias, uint16_t* y, int32_t ldy, int32_t cout,
                   int32_t relu, int32_t accumulate, const uint16_t* mask, int32_t ldm, void* stream);

/* Weights of the transposed convolution: wt[c][t][o] = w[o][8 - t][c]
 * (wt is [cin][9][cout] bf16). */
int pat_nn_conv3x3_flip(int32_t cout, int32_t cin, const uint16_t* w, uint16_t* wt, void* stream);

/* Scratch (bytes) of pat_nn_conv3x3_wgrad for these sizes. */
int pat_nn_wgrad_scratch_bytes(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout, size_t* bytes);

/* Weight and bias gradients of a 3x3 convolution:
 *   dw[o][t][c] = sum_p dy[p][o] x[p + offset_t][c],  db[o] = sum_p dy[p][o]
 * with dy the gradient wrt the layer's pre-activation output ([B*H*W][ldy]
 * bf16, cout channels) and x its input ([B*H*W][ldx] bf16, cin channels).
 * dw: [cout][9][cin] float32, db: [cout] float32 or NULL.  Pixel partial sums
 * are reduced in a fixed order.  Requires cin % 8 == 0, cout % 8 == 0. */
int pat_nn_conv3x3_wgrad(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t ldx, int32_t cin,
                         const uint16_t* dy, int32_t ldy, int32_t cout, float* dw, float* db, void* scratch,
                         size_t scratch_bytes, void* stream);

/* 2x2 average pooling: y[b][i][j] = mean of x[b][2i..2i+1][2j..2j+1];
 * x [B][H][W][ldx], y [B][H/2][W/2][ldy], H and W even. */
int pat_nn_avgpool2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* x, int32_t ldx, uint16_t* y,
                    int32_t ldy, void* stream);

/* Adjoint of pat_nn_avgpool2: dx[b][i][j] = dy[b][i/2][j/2] / 4 (+ the old dx if
 * accumulate), zero where mask <= 0 (mask [B][H][W][ldm] or NULL).  dx is the
 * fine [B][H][W][ldx] array, dy the coarse one. */
int pat_nn_avgpool2_backward(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* dy, int32_t ldy,
                             uint16_t* dx, int32_t ldx, const uint16_t* mask, int32_t ldm, int32_t accumulate,
                             void* stream);

/* Nearest-neighbour 2x upsampling: y[b][i][j] = x[b][i/2][j/2]; y is the fine
 * [B][H][W][ldy] array, x the coarse [B][H/2][W/2][ldx] one. */
int pat_nn_upsample2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* x, int32_t ldx, uint16_t* y,
                     int32_t ldy, void* stream);

/* Adjoint of pat_nn_upsample2: dx[b][i][j] = sum of dy over the four fine
 * pixels of coarse pixel (i, j), zero where mask <= 0 (coarse mask or NULL). */
int pat_nn_upsample2_backward(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* dy, int32_t ldy,
                              uint16_t* dx, int32_t ldx, const uint16_t* mask, int32_t ldm, void* stream);

/* 1x1 output head: r[p] = b[0] + sum_c w[c] x[p][c]; x [P][ldx] bf16, w [C]
 * bf16, b float32 scalar, r [P] float32. */
int pat_nn_head(int64_t P, int32_t C, const uint16_t* x, int32_t ldx, const uint16_t* w, const float* b, float* r,
                void* stream);

/* Scratch (bytes) of pat_nn_head_backward for C channels. */
size_t pat_nn_head_scratch_bytes(int32_t C);

/* Gradients of the head given dr = dL/dr [P]: dx[p][c] = [x[p][c] > 0] w[c] dr[p]
 * (the gradient wrt the pre-activation of the ReLU layer that produced x;
 * bf16 [P][lddx]), dw[c] = sum_p dr[p] x[p][c], db[0] = sum_p dr[p] (float32).
 * Requires C to divide 256. */
int pat_nn_head_backward(int64_t P, int32_t C, const uint16_t* x, int32_t ldx, const uint16_t* w, const float* dr,
                         uint16_t* dx, int32_t lddx, float* dw, float* db, void* scratch, size_t scratch_bytes,
                         void* stream);

/* Scratch (bytes) of pat_nn_masked_mse. */
size_t pat_nn_mse_scratch_bytes(void);

/* Masked squared loss over B images sharing mask [H*W] (uint8, nonzero = in):
 * out[0] = L = sum_masked (r - t)^2 / (2 n), out[1] = n (masked pixels x B),
 * both float64; dr = [mask] (r - t) / n (float32 [B][H][W]). */
int pat_nn_masked_mse(int32_t B, int64_t hw, const float* r, const float* t, const uint8_t* mask, float* dr,
                      double* out, void* scratch, size_t scratch_bytes, void* stream);

/* One Adam step (Kingma & Ba, 2015) at step count `step` >= 1 over n float32
 * parameters w with gradient g and moments m, v (updated in place):
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps);
 * w_bf16 (or NULL) receives the rounded copy of w used by the kernels. */
int pat_nn_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, int32_t step, float lr,
                float b1, float b2, float eps, void* stream);

/* Round n float32 values to bf16. */
int pat_nn_to_bf16(int64_t n, const float* a, uint16_t* b, void* stream);

/* Scratch (bytes) of pat_nn_pack_input. */
size_t pat_nn_pack_scratch_bytes(void);

/* Network input of one image of H x W pixels from the interpolated coarse
 * sound speed c_up [H][W] and K interpolated initial-pressure gradients
 * g_up [K][H][W]:
 *   x[p] = ((c - shift) / scale, sum_k g_k / max_p |sum_k g_k|, 0 x 6) (bf16 [H][W][8]),
 *   base[p] = c (float32), target[p] = (c_true - c) / scale if c_true (float32).
 * sym in 0..7 applies one symmetry of the square to every output (source
 * pixel of output (i, j): rows flipped if bit 0, columns flipped if bit 1, then
 * transposed if bit 2; bit 2 requires H == W). */
int pat_nn_pack_input(int32_t H, int32_t W, int32_t K, const float* c_up, const float* g_up, const float* c_true,
                      int32_t sym, float shift, float scale, uint16_t* x, float* base, float* target,
                      void* scratch, size_t scratch_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PAT_NN_H */
