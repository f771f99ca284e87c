/*
 * unet.h -- C ABI of the learned crosstalk filter kernels in librtm.so.
 *
 * A 3-D U-Net maps an RTM image made with one random-boundary realisation
 * (image condition of Eq. (3); random boundary of the section on wavefield
 * reconstruction) to the average over many realisations, in which the
 * boundary crosstalk, uncorrelated between realisations, has cancelled.
 * The network is a project extension of the method.  These entry points are
 * its layers, forward and backward; the training loop composes them.
 *
 * Conventions
 *  - Activations are channels-last: element (n, z, y, x, c) of a tensor with
 *    extents (N, D, H, W, C) sits at ((((n*D + z)*H + y)*W + x)*C + c).
 *  - bfloat16 values are stored as uint16_t (the upper half of the float32
 *    bit pattern); conversions round to nearest even.
 *  - Convolutions are 3x3x3 cross-correlations with one cell of zero padding
 *    (output size = input size):
 *        y[p, o] = b[o] + sum_{t, i} w[o, t, i] x[p + off(t), i],
 *    tap t = (kz*3 + ky)*3 + kx, off(t) = (kz-1, ky-1, kx-1) in (z, y, x).
 *    Master weights are float32 [Cout][27][Cin].
 *  - Channel counts of a convolution must be 16, 32, 64 or 128, or the pair
 *    (Cin, Cout) must be (1, 16) or (16, 1): the network's one-channel input
 *    and output layers, which run on the vector units (too few products per
 *    voxel for the matrix cores); the others run as bfloat16 MFMA.
 *  - Pointers are device pointers unless stated; device buffers belong to
 *    the caller; nothing is allocated.  Every call is asynchronous on
 *    `stream` (a hipStream_t, NULL = default stream) unless stated.
 *  - Return 0 (RTM_OK) or a negative RTM_* code from rtm.h, with a message
 *    from rtm_last_error().  All checks run on the host before any launch;
 *    on error nothing is launched.
 */
#ifndef UNET_H
#define UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Extents of one convolution: N samples of D x H x W voxels, Cin -> Cout. */
typedef struct {
    int32_t n, d, h, w;
    int32_t cin, cout;
} unet_conv_desc_t;

/* Packs master weights w (float32 [Cout][27][Cin]) into the two bfloat16
 * layouts the convolution kernels read: w_fwd [Cout][27*Cin] (same order)
 * and w_bwd [Cin][27*Cout] with w_bwd[i][t*Cout + o] = w[o][26 - t][i] (the
 * spatially flipped, channel-transposed kernel of the input gradient).
 * Either output may be NULL. */
int unet_weight_pack(const unet_conv_desc_t *desc, const float *w, uint16_t *w_fwd, uint16_t *w_bwd, void *stream);

/* One layer of unet_weight_pack_many. */
typedef struct {
    const float *w;
    int32_t cin, cout;
    uint16_t *w_fwd, *w_bwd;
} unet_pack_item_t;

/* unet_weight_pack for `count` layers (1 .. UNET_PACK_MAX, host array) in
 * one launch: the same bits as one call per layer. */
#define UNET_PACK_MAX 16
int unet_weight_pack_many(int32_t count, const unet_pack_item_t *items, void *stream);

/* Forward convolution on bfloat16 operands with float32 accumulation
 * (MFMA), plus a fused epilogue.  For each output (p, o) with o < y_channels
 * (for y) or o < Cout (for r and out):
 *     a = acc + (bias ? bias[o] : 0);   if (relu) a = max(a, 0)
 *     y[p*y_channels + o] = a                       (float32, if y)
 *     r[p*Cout + o] = bf16(a)                       (if r)
 *     out[p*Cout + o] = bf16(a + (skip ? skip[p*Cout + o] : 0))   (if out)
 * x: bfloat16 [N][D][H][W][Cin]; w_fwd from unet_weight_pack; skip: bfloat16
 * [..][Cout] or NULL.  1 <= y_channels <= Cout.  Outputs must not alias
 * inputs.  x and w_fwd must be 16-byte aligned; for the (1, 16) pair also
 * y, r, out and skip (stored and read as 16-byte vectors). */
int unet_conv3d_fwd(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *w_fwd, const float *bias,
                    int32_t relu, const uint16_t *skip, float *y, int32_t y_channels, uint16_t *r, uint16_t *out,
                    void *stream);

/* Input gradient: dx[q, i] = sum_{t, o} w[o, t, i] dy[q - off(t), o], as the
 * forward kernel applied to dy with w_bwd.  dy: bfloat16 [..][Cout];
 * dx: float32 [..][Cin].  dy and w_bwd must be 16-byte aligned; for the
 * (16, 1) pair also dx. */
int unet_conv3d_dgrad(const unet_conv_desc_t *desc, const uint16_t *dy, const uint16_t *w_bwd, float *dx,
                      void *stream);

/* unet_conv3d_dgrad, and in the same pass the gradient through the ReLU of
 * the layer below, whose stored output is `mask` (bfloat16 [..][Cin]):
 *     g_out[q, i] = bf16(dx[q, i]) if mask[q, i] > 0, else 0
 * (bfloat16 [..][Cin]; what unet_relu_grad gives for g1 = dx alone, bit for
 * bit).  mask and g_out 16-byte aligned, Cin a multiple of 8. */
int unet_conv3d_dgrad_relu(const unet_conv_desc_t *desc, const uint16_t *dy, const uint16_t *w_bwd, float *dx,
                           const uint16_t *mask, uint16_t *g_out, void *stream);

/* Workspace of unet_conv3d_wgrad in bytes (host only, no device work). */
int unet_wgrad_ws_bytes(const unet_conv_desc_t *desc, size_t *bytes);

/* Weight and bias gradients: dw[o][t][i] = sum_p dy[p, o] x[p + off(t), i]
 * (float32 [Cout][27][Cin]) and db[o] = sum_p dy[p, o] (float32 [Cout], or
 * NULL).  x: bfloat16 [..][Cin]; dy: bfloat16 [..][Cout].  Split-K partial
 * sums go to the workspace and are reduced in a fixed order: the result is
 * bitwise reproducible.  Overwrites dw and db. */
int unet_conv3d_wgrad(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy, float *dw, float *db,
                      void *ws, size_t ws_bytes, void *stream);

/* unet_conv3d_wgrad in two halves, so that a training step can reduce the
 * split-K partials of all its layers in one pass at the end of the backward
 * pass instead of one pass per layer.
 *
 * unet_conv3d_wgrad_partial writes the partial sums of one layer into ws
 * (same size and alignment rules as unet_conv3d_wgrad; one workspace per
 * layer whose reduction is still pending).  unet_wgrad_reduce_many then
 * reduces `count` layers (1 .. UNET_WGRAD_MAX, host array of items) in two
 * launches: for each item, dw and db (db may be NULL) get the same bits
 * unet_conv3d_wgrad would give for the same desc, x and dy.  An item's ws
 * must hold that layer's partials (written on the same stream, or ordered
 * before this call by the caller) and must not be shared with another item:
 * the reduction keeps its chunk sums in ws. */
int unet_conv3d_wgrad_partial(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy, void *ws,
                              size_t ws_bytes, void *stream);

typedef struct {
    unet_conv_desc_t desc;
    void *ws;
    size_t ws_bytes;
    float *dw, *db;
} unet_wgrad_item_t;

#define UNET_WGRAD_MAX 16
int unet_wgrad_reduce_many(int32_t count, const unet_wgrad_item_t *items, void *stream);

/* Network input: x[v][c] = bf16(img[v] * scale) for c == 0, 0 for c > 0;
 * img float32 [nvox], x bfloat16 [nvox][channels]. */
int unet_embed(int64_t nvox, int32_t channels, const float *img, float scale, uint16_t *x, void *stream);

/* Mean over 2x2x2 blocks: x bfloat16 (N, D, H, W, C) -> y bfloat16
 * (N, D/2, H/2, W/2, C).  D, H and W must be even. */
int unet_pool2(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const uint16_t *x, uint16_t *y, void *stream);

/* Nearest-neighbour upsampling: x bfloat16 (N, D, H, W, C) -> y bfloat16
 * (N, 2D, 2H, 2W, C). */
int unet_up2(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const uint16_t *x, uint16_t *y, void *stream);

/* Adjoint of unet_up2: g_coarse (N, D, H, W, C) = sum over each 2x2x2 block
 * of g_fine (N, 2D, 2H, 2W, C); float32. */
int unet_up2_bwd(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g_fine, float *g_coarse,
                 void *stream);

/* unet_up2_bwd, and in the same pass the gradient through the ReLU of the
 * coarse level, whose stored output is `mask` (bfloat16, extents of
 * g_coarse): g_out = bf16(g_coarse) where mask > 0, else 0 (what
 * unet_relu_grad gives for g1 = g_coarse alone, bit for bit). */
int unet_up2_bwd_relu(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g_fine, float *g_coarse,
                      const uint16_t *mask, uint16_t *g_out, void *stream);

/* Gradient through a ReLU whose stored output is `mask` (bfloat16, same
 * extents (N, D, H, W, C)):
 *     out[v, c] = bf16((g1[v, c] + (g2 ? g2[v, c] : 0)
 *                      + (g_pool ? g_pool[parent(v), c] / 8 : 0)) * (mask[v, c] > 0))
 * where g_pool has extents (N, D/2, H/2, W/2, C) (the adjoint of unet_pool2
 * fused in); g1 float32; g2, g_pool float32 or NULL. */
int unet_relu_grad(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g1, const float *g2,
                   const float *g_pool, const uint16_t *mask, uint16_t *out, void *stream);

/* Workspace of unet_mse in bytes (host only). */
int unet_mse_ws_bytes(int64_t nvox, size_t *bytes);

/* Residual output and loss: out[v] = img[v] + y[v]; loss = mean((out -
 * target)^2) accumulated in float64 in a fixed order; gy[v][0] =
 * bf16(2 (out[v] - target[v]) / nvox) and gy[v][c > 0] = 0 (bfloat16
 * [nvox][channels]).  out may be NULL; gy may be NULL; target may be NULL
 * (then only out is produced).  If loss (host pointer) is non-NULL the call
 * synchronises the stream and stores the loss there. */
int unet_mse(int64_t nvox, int32_t channels, const float *img, const float *y, const float *target, float *out,
             uint16_t *gy, double *loss, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba) on n float32 parameters with bias correction
 * for step number `step` (>= 1): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  The
 * moments and the update are float32; 1 - b1, 1 - b2 and the corrections
 * are formed in double from the double arguments. */
int unet_adam(int64_t n, float *p, const float *g, float *m, float *v, double lr, double b1, double b2, double eps,
              int32_t step, void *stream);

/* Kernel choice of unet_conv3d_fwd and unet_conv3d_dgrad, process-wide:
 * with lds = 1 (the default) convolutions of at most 32 input and 32
 * output channels, and of 64 input and 32 output channels, on grids at
 * least 64 voxels wide and large enough for 256 workgroups of 64 x 4 x
 * (4 to 16) output voxels stage their input in LDS
 * (one load per activation instead of one per tap); lds = 0 runs every
 * layer on the direct kernel.  Both compute each output element by the same sequence of
 * matrix-core operations, so results are equal bit for bit; the switch is
 * for tests and measurement.  unet_get_conv_lds reads it back. */
int unet_set_conv_lds(int32_t lds);
int unet_get_conv_lds(int32_t *lds);

#ifdef __cplusplus
}
#endif

#endif /* UNET_H */
