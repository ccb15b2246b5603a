/*
 * msl_nn.h -- C ABI of the learned-initialiser kernels in libmsl.
 *
 * The reconstruction of arXiv 2212.01253 (Sec. 4.1) starts ADAM from an
 * initial guess.  These kernels train and run a small convolutional network
 * that maps a far-field log-intensity image to an initial delta cross-section
 * (a learned initial guess; not part of the paper).  Matrix products run on
 * the MI355X matrix cores in bfloat16 with float32 accumulation.
 *
 * Layouts: activations are float32 [C][B][H][W] (channel-major, so a
 * convolution is one matrix product over all images of a batch); bfloat16
 * values are uint16_t holding the upper half of the IEEE float32 pattern,
 * rounded to nearest even.  All arrays are caller-owned DEVICE memory; every
 * call only enqueues on hip_stream.  Arguments are validated on the host; on
 * an error nothing is enqueued and msl_last_error() (msl.h) describes it.
 */
#ifndef MSL_NN_H
#define MSL_NN_H

#include <stddef.h>
#include <stdint.h>

#include "msl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[m][n] = beta * C[m][n] + sum_k op(A)[m][k] op(B)[k][n] (+ bias[m]) (then max(0, .) if relu).
 * op(A)[m][k] = transA ? A[k * lda + m] : A[m * lda + k]   (bfloat16)
 * op(B)[k][n] = transB ? B[n * ldb + k] : B[k * ldb + n]   (bfloat16)
 * C float32 with row stride ldc; C16 (optional) receives C rounded to bfloat16 with the same
 * stride; bias (optional) float32 [M].  M, N, K >= 1. */
msl_status msl_nn_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                            const uint16_t* B, int32_t ldb, int32_t transB, float* C, int32_t ldc, float beta,
                            const float* bias, int32_t relu, uint16_t* C16, void* hip_stream);

/* The same product without beta, bias or activation, its K range split into `splits` parts that
 * run side by side (for small M x N and long K, such as weight gradients): part s writes its
 * partial product to partials + s * M * N (float32 [splits][M][N], caller-owned scratch), then a
 * fixed-order sum over the parts writes C.  1 <= splits <= 4096. */
msl_status msl_nn_gemm_bf16_splitk(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                                   const uint16_t* B, int32_t ldb, int32_t transB, float* C, int32_t ldc,
                                   int32_t splits, float* partials, void* hip_stream);

/* 3x3 patches, zero padding 1, stride 1 or 2: x float32 [C][B][H][W] ->
 * col bfloat16 [C*9][B*Ho*Wo] with Ho = H/stride, Wo = W/stride (H, W divisible by stride);
 * row c*9 + 3*(dy+1) + (dx+1), column (b*Ho + i)*Wo + j holds x[c][b][stride*i+dy][stride*j+dx]. */
msl_status msl_nn_im2col3x3(int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const float* x,
                            uint16_t* col, void* hip_stream);

/* Adjoint of msl_nn_im2col3x3: dx[c][b][y][x] = sum of the col entries that sampled it
 * (col float32 [C*9][B*Ho*Wo]); dx is overwritten. */
msl_status msl_nn_col2im3x3(int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const float* col,
                            float* dx, void* hip_stream);

/* Scratch the two calls below need for their packed weights: bfloat16 elements (16 pad16(Co) pad16(C),
 * pad16 rounding up to a multiple of 16), or 0 for invalid sizes. */
int64_t msl_nn_conv3x3_scratch_elems(int32_t Co, int32_t C);

/* 3x3 convolution, zero padding 1, stride 1 or 2, as an implicit matrix-core product on halo tiles
 * (no patch matrix in memory):
 * y[o][b][i][j] = act(sum_c sum_t w16[o][9c + t] bf16(x[c][b][s i + dy][s j + dx]) + bias[o]),
 * t = 3 (dy + 1) + (dx + 1); x [C][B][H][W] float32 (x_bf16 0) or bfloat16 bits (x_bf16 1: used
 * as is, the same product as float32 x holding those values), w16 bfloat16 [Co][9C], bias float32
 * [Co] or NULL, relu 0/1, y [Co][B][H/s][W/s] float32 (y_bf16 0) or bfloat16 bits (y_bf16 1: the
 * float32 result rounded to nearest even; an activation stored for the next layer, which rounds
 * its input to bfloat16 anyway).  The products and sums are those of msl_nn_gemm_bf16 with the
 * patch matrix, in another order (over taps, then channels in chunks of 16), so the two agree to
 * float32 rounding.  wscratch: device, 16-byte aligned, msl_nn_conv3x3_scratch_elems(Co, C)
 * bfloat16 elements, overwritten (the weights in [Co][9][pad16(C)] order); the call reads w16 once
 * per call, not once per tile. */
msl_status msl_nn_conv3x3(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const uint16_t* w16,
                          const void* x, int32_t x_bf16, const float* bias, int32_t relu, void* y, int32_t y_bf16,
                          uint16_t* wscratch, void* hip_stream);

/* Its input gradient, also implicit: dx[c][b][y][x] = sum over o and taps t of w16[o][9c + t] dy16[o][b][i][j]
 * where s i + dy = y and s j + dx = x (dy16 bfloat16 [Co][B][H/s][W/s]; dx float32 [C][B][H][W],
 * overwritten).  Runs on halo tiles with the weights repacked into wscratch (required): stride 1 as
 * a convolution of dy16 with the weights transposed and rotated by 180 degrees; stride 2 (dx 8-byte
 * aligned) split by the parity of (y, x) into a 2x2 convolution of dy16 with 4 C rows (zero weights
 * where a parity class has no tap).  A stride-2 call with dx not 8-byte aligned runs as an implicit
 * product over the patch columns instead.  accumulate 1: dx += the gradient instead of dx = (the
 * gradient of a layer whose input also feeds a skip connection; needs the halo path). */
msl_status msl_nn_conv3x3_adjoint(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride,
                                  const uint16_t* w16, const uint16_t* dy16, float* dx, int32_t accumulate,
                                  uint16_t* wscratch, void* hip_stream);

/* Its weight gradient, implicit as well: dw[o][9c + t] = sum over output pixels p of dy16[o][p] times the
 * patch value (c, t) at p (x float32 rounded to bfloat16 as in the forward, or with x_bf16 1 bfloat16
 * bits used as is: the same result as float32 x holding those values); the pixel sum is split into at
 * most `splits` parts written to partials (float32 [splits][Co][9C], caller-owned scratch) and then
 * summed in a fixed order into dw (float32 [Co][9C]).  When the output width W/s is a multiple of 8 the parts
 * are ranges of 128/s-pixel halo tiles (as many parts as fill the GPU, at most `splits`), otherwise
 * ranges of pixels of the patch-column product (msl_nn_gemm_bf16_splitk of dy16 and the patch
 * matrix, bit for bit).  1 <= splits <= 4096. */
msl_status msl_nn_conv3x3_weight_grad(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride,
                                     const uint16_t* dy16, const void* x, int32_t x_bf16, float* dw, int32_t splits,
                                     float* partials, void* hip_stream);

/* Nearest 2x upsampling [C][B][H][W] -> [C][B][2H][2W] (y may be a channel slice of a larger
 * array: it is written at y with the [C][B][2H][2W] layout; x and y float32, or bfloat16 bits with
 * bf16 1, copied unchanged), and its adjoint (float32, sum of the four). */
msl_status msl_nn_upsample2(int32_t C, int32_t B, int32_t H, int32_t W, const void* x, void* y, int32_t bf16,
                            void* hip_stream);
msl_status msl_nn_upsample2_adjoint(int32_t C, int32_t B, int32_t H, int32_t W, const float* dy, float* dx,
                                    void* hip_stream);

/* Row pooling by f: x [B][H][W] -> y [B][H/f][W], y = mean of f consecutive rows; and its adjoint. */
msl_status msl_nn_rowpool(int32_t B, int32_t H, int32_t W, int32_t f, const float* x, float* y, void* hip_stream);
msl_status msl_nn_rowpool_adjoint(int32_t B, int32_t H, int32_t W, int32_t f, const float* dy, float* dx,
                                  void* hip_stream);

/* Summaries of each image row for the network's global head: x float32 [B][H][W], f16 bfloat16
 * [B][3H] with v[r] = mean over all W columns of row r, v[H + r] = x[b][r][W/2] (the centre column:
 * zero transverse momentum in an fftshifted far field), v[2H + r] = mean of the seven columns
 * W/2-3 .. W/2+3 (float32 sums in ascending column order), and f16[b][i] = bfloat16((v[i] -
 * shift[i]) * scale[i]); shift and scale float32 [3H] (normalisation; each may be NULL: 0 and 1).
 * W >= 8. */
msl_status msl_nn_row_features(int32_t B, int32_t H, int32_t W, const float* x, const float* shift,
                               const float* scale, uint16_t* f16, void* hip_stream);

/* The head's output broadcast along the columns: y[b][r][z] += p[r][b] (p float32 [R][B], y float32
 * [B][R][W]); and its adjoint dp[r][b] = sum over z of dy[b][r][z] (ascending z; dp overwritten). */
msl_status msl_nn_add_row_bias(int32_t B, int32_t R, int32_t W, const float* p, float* y, void* hip_stream);
msl_status msl_nn_row_bias_adjoint(int32_t B, int32_t R, int32_t W, const float* dy, float* dp, void* hip_stream);

/* Elementwise helpers over n floats: dy[i] = y[i] > 0 ? dy[i] : 0 (ReLU backward);
 * y[i] += x[i]; y16[i] = bfloat16(x[i]). */
msl_status msl_nn_relu_adjoint(int64_t n, const float* y, float* dy, void* hip_stream);
msl_status msl_nn_add(int64_t n, const float* x, float* y, void* hip_stream);
msl_status msl_nn_to_bf16(int64_t n, const float* x, uint16_t* y16, void* hip_stream);

/* One layer's output gradient made ready for its backward products, in one pass over dy (float32
 * [M][N], read only): g = dy where y > 0, else 0 (the ReLU adjoint; y [M][N] float32, or bfloat16
 * bits with y_bf16 1, or NULL for no activation); dy16[m][n] = bfloat16(g) and bias_grad[m] = sum_n g (fixed-order sums, as
 * msl_nn_rowsum; parts: float32 scratch of at least 64 M).  dy16 equals msl_nn_relu_adjoint then
 * msl_nn_to_bf16 bit for bit; bias_grad is msl_nn_rowsum of g summed in another fixed order. */
msl_status msl_nn_grad_prep(int32_t M, int32_t N, const void* y, int32_t y_bf16, const float* dy, uint16_t* dy16,
                            float* bias_grad, float* parts, void* hip_stream);

/* out[m] = sum_n X[m * N + n] (float32 sums of float32 rows, bias gradients), in a fixed order:
 * 64 partial sums per row into parts (float32 [M][64], caller-owned scratch), then their sum. */
msl_status msl_nn_rowsum(int32_t M, int32_t N, const float* X, float* out, float* parts, void* hip_stream);

/* Mean squared error over n values: loss_out[0] (double, device) = sum (p - t)^2 / n,
 * grad[i] = 2 (p - t) / n (float32; may be NULL).  The sum is FP64 in a fixed order: 256 chunk
 * sums into parts (double, device scratch of at least 256), then their sum. */
msl_status msl_nn_mse(int64_t n, const float* pred, const float* target, float* grad, double* loss_out,
                      double* parts, void* hip_stream);

/* ADAM step over n float32 weights (as msl_region_adam_step, without the clamp), then the
 * bfloat16 copy w16 of the new weights (may be NULL); t >= 1. */
msl_status msl_nn_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w16, float lr,
                       float beta1, float beta2, float eps, int32_t t, void* hip_stream);

/* out[i] = a * log(x[i] + eps) + b (float32; the network's input map of an intensity image). */
msl_status msl_nn_logmap(int64_t n, const float* x, float eps, float a, float b, float* out, void* hip_stream);

/* ---- training samples: slice pools of bars on a substrate, rendered on the device ----
 * Sample i has nf[i] boxes (at most MSL_NN_MAX_BOXES) and np[i] pool slices.  Box f of sample
 * i is boxes[(i * MSL_NN_MAX_BOXES + f) * 8 + 0..7] = {x0, x1, y0, y1, z0, z1, delta, beta}
 * (slice range [x0, x1), rows [y0, y1), columns [z0, z1), as floats holding integers and the
 * two values); pool slice u of sample i starts at slice cuts[i * MSL_NN_MAX_CUTS + u].  Pool
 * slice u is the substrate (rows [0, substrate_rows): sub_delta, sub_beta; zero above) with
 * every box active at its first slice written over it in order.  Pools are written at
 * pool_delta + pool_off[i] * ny * nz (float32 [np[i]][ny][nz]; the same for pool_beta).
 * All arrays device memory. */
#define MSL_NN_MAX_BOXES 64
#define MSL_NN_MAX_CUTS 132
msl_status msl_nn_render_pools(int32_t n_samples, int32_t ny, int32_t nz, int32_t substrate_rows, float sub_delta,
                               float sub_beta, const float* boxes, const int32_t* nf, const int32_t* cuts,
                               const int32_t* np, const int64_t* pool_off, int32_t max_pool, float* pool_delta,
                               float* pool_beta, void* hip_stream);

/* Length-weighted mean of pool slices over a box of rows: for every sample i,
 * out[i][r][z] = scale * sum_u w[i * MSL_NN_MAX_CUTS + u] * pool[pool_off[i] + u][y0 + r][z]
 * for r < rows, u < np[i] (out float32 [n_samples][rows][nz]). */
msl_status msl_nn_pool_average(int32_t n_samples, int32_t ny, int32_t nz, int32_t y0, int32_t rows,
                               const float* w, const int32_t* np, const int64_t* pool_off, int32_t max_pool,
                               const float* pool, float scale, float* out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MSL_NN_H */
