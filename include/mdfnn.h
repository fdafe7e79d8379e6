/*
 * mdfnn.h -- C ABI of the layer kernels of the convolutional encoder-decoder
 * that predicts steady cavity fields (P, u, v, grad u) for warm-starting the
 * MDF-LBM solver of include/mdf.h.  None of this is in the paper: the
 * network only proposes an initial state; the solver (eq. 3-21) decides the
 * result, and a warm start is built from the predicted fields with the
 * inverse of eq. 3-16 (MDF_INIT_FIELDS_GRAD).
 *
 * Conventions
 * -----------
 * - Activations are NHWC: x[b][y][x][c], c fastest.  "bf16" buffers hold
 *   bfloat16 bit patterns (uint16_t); stores round to nearest even.
 *   Products are taken on the gfx950 matrix cores (BF16 in, FP32 accumulate).
 * - 3x3 convolutions use zero padding 1 and stride 1.  Weights are
 *   w[cout][tap][cin] with tap = 3 * (dy + 1) + (dx + 1), i.e. the output
 *   at pixel (y, x) is  bias[co] + sum_{tap, ci} w[co][tap][ci] x[y+dy][x+dx][ci].
 * - Channel counts must be multiples of 32 for the 3x3 kernels (pad the
 *   input with zero channels); the 1x1 head takes any cin/cout <= 32.
 * - All pointers are device pointers owned by the caller; every call is
 *   enqueued on `stream` (hipStream_t, NULL = null stream) and returns 0 on
 *   success, -1 (MDFNN_EINVAL) on invalid sizes or null pointers (nothing
 *   launched), -3 (MDFNN_EDEVICE) on a launch error.
 * - Scratch buffers are caller-owned; their size is given by the matching
 *   *_scratch_bytes() query.
 */
#ifndef MDFNN_H
#define MDFNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDFNN_OK 0
#define MDFNN_EINVAL (-1)
#define MDFNN_ETOOBIG (-2)
#define MDFNN_EDEVICE (-3)

/* y = act(conv3x3(concat(x1, x2)) + bias).  x1: [B,H,W,c1], x2: [B,H,W,c2]
 * or NULL with c2 = 0 (the input channels are x1's then x2's); w: bf16
 * [cout][9][c1+c2]; bias: fp32 [cout] or NULL.  relu != 0 applies max(0, .).
 * Output: y_bf16 [B,H,W,cout] (if not NULL) and/or y_f32 (if not NULL).
 * mask (bf16, [B,H,W,cout], or NULL): the output is multiplied by
 * (mask > 0), the derivative of a ReLU whose output is `mask` (used by the
 * data gradient).  c1, c2, cout multiples of 32 (c2 may be 0). */
int mdfnn_conv3x3_fwd(const uint16_t *x1, int c1, const uint16_t *x2, int c2, const uint16_t *w,
                      const float *bias, int B, int H, int W, int cout, int relu,
                      const uint16_t *mask, uint16_t *y_bf16, float *y_f32, void *stream);

/* Data gradient of a 3x3 convolution: the weights of the transposed
 * convolution, wt[ci][tap][co] = w[co][8 - tap][ci] (bf16).  w: [cout][9][cin]. */
int mdfnn_conv3x3_flip(const uint16_t *w, int cout, int cin, uint16_t *wt, void *stream);

/* Weight gradient of y = conv3x3(concat(x1, x2)):
 *   dw[co][tap][ci] = sum_{b,y,x} dy[b][y][x][co] * xin[b][y+dy][x+dx][ci]
 * in FP32, plus the bias gradient db[co] = sum dy (if db not NULL).
 * dy: bf16 [B,H,W,cout].  dw: fp32 [cout][9][c1+c2] (overwritten).
 * scratch: mdfnn_wgrad_scratch_bytes(B, H, W, c1 + c2, cout) bytes. */
size_t mdfnn_wgrad_scratch_bytes(int B, int H, int W, int cin, int cout);
int mdfnn_conv3x3_wgrad(const uint16_t *x1, int c1, const uint16_t *x2, int c2, const uint16_t *dy,
                        int B, int H, int W, int cout, float *dw, float *db, void *scratch,
                        void *stream);

/* 2x2 average pooling (H, W even): y[b][i][j][c] = mean of the 2x2 block.
 * Backward: dx[b][y][x][c] = dy[b][y/2][x/2][c] / 4 (H, W: the input size). */
int mdfnn_avgpool2_fwd(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, void *stream);
int mdfnn_avgpool2_bwd(const uint16_t *dy, int B, int H, int W, int C, uint16_t *dx, void *stream);

/* Nearest 2x upsampling: y[b][y][x][c] = x[b][y/2][x/2][c] (output 2H x 2W).
 * Backward: dx[b][i][j][c] = sum of dy over the 2x2 block. */
int mdfnn_upsample2_fwd(const uint16_t *x, int B, int H, int W, int C, uint16_t *y, void *stream);
int mdfnn_upsample2_bwd(const uint16_t *dy, int B, int H, int W, int C, uint16_t *dx, void *stream);

/* out = (a + b) * (mask > 0) over n bf16 elements; b and mask may be NULL
 * (then omitted).  out may alias a.  The mask form is the derivative of a
 * ReLU whose output is `mask`. */
int mdfnn_add(const uint16_t *a, const uint16_t *b, const uint16_t *mask, long long n, uint16_t *out,
              void *stream);

/* 1x1 head in FP32: y[p][o] = bias[o] + sum_c w[o][c] x[p][c], x bf16
 * [P][cin], w fp32 [cout][cin], y fp32 [P][cout]; cin, cout <= 32. */
int mdfnn_head_fwd(const uint16_t *x, int P, int cin, const float *w, const float *bias, int cout,
                   float *y, void *stream);
/* Backward of the head: dx (bf16 [P][cin], may be NULL), dw (fp32
 * [cout][cin]) and db (fp32 [cout]), from dy (fp32 [P][cout]).  mask (bf16
 * [P][cin] or NULL) multiplies dx by (mask > 0).  scratch:
 * mdfnn_head_scratch_bytes(P, cin, cout) bytes. */
size_t mdfnn_head_scratch_bytes(int P, int cin, int cout);
int mdfnn_head_bwd(const uint16_t *x, const float *dy, int P, int cin, const float *w, int cout,
                   const uint16_t *mask, uint16_t *dx, float *dw, float *db, void *scratch,
                   void *stream);

/* Weighted mean squared error over P pixels and C channels:
 *   L = sum_{p,c} wt[p] (y - t)^2 / (sum_p wt[p] * C),
 * with its gradient dy = dL/dy (fp32 [P][C]); loss (fp32 scalar, device)
 * accumulated deterministically.  wt: fp32 [P] (e.g. 1 on fluid nodes,
 * 0 on solid ones).  scratch: mdfnn_loss_scratch_bytes(P) bytes. */
size_t mdfnn_loss_scratch_bytes(int P);
int mdfnn_mse(const float *y, const float *t, const float *wt, int P, int C, float *dy, float *loss,
              void *scratch, void *stream);

/* mdfnn_mse without a scratch argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same kernels and the same results as
 * mdfnn_mse; the partial sums live in a static device array of
 * 2 * ceil(MDFNN_MSE_NOALLOC_MAX_P / 256) + 2 floats (256 KiB) that each
 * GPU the library runs on holds until the process ends.  The call allocates
 * nothing: on its first use on a device it only looks up that array's
 * address (hipGetSymbolAddress) with the device current.  Every call on one
 * GPU shares the array: calls that overlap on one GPU (on different
 * streams, or from several threads) race; calls on one stream are ordered.
 * Returns MDFNN_ETOOBIG (nothing launched) when P > MDFNN_MSE_NOALLOC_MAX_P,
 * MDFNN_EINVAL on null pointers or sizes < 1, MDFNN_EDEVICE on a HIP error. */
#define MDFNN_MSE_NOALLOC_MAX_P (1 << 23)
int mdfnn_mse_noalloc(const float *y, const float *t, const float *wt, int P, int C, float *dy,
                      float *loss, void *stream);

/* Adam update with FP32 master weights (Kingma & Ba): for n parameters,
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * then p_bf16 = bf16(p) if p_bf16 is not NULL.  t >= 1 is the step count. */
int mdfnn_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
               float eps, int t, uint16_t *p_bf16, void *stream);

/* fp32 -> bf16 (round to nearest even) and bf16 -> fp32 conversions. */
int mdfnn_to_bf16(const float *x, long long n, uint16_t *y, void *stream);
int mdfnn_to_f32(const uint16_t *x, long long n, float *y, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MDFNN_H */
