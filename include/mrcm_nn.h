/*
 * Learned warm start for the conjugate-gradient local solves (MRCM_PCG in
 * mrcm.h).  A small 3D convolutional network maps, per right-hand-side column
 * of a subdomain, two channels on the subdomain's cell grid -- the centred
 * log-permeability and the right-hand side scaled to a largest magnitude of
 * one -- to the column's solution up to a scale (the MBFs of (2.25), the
 * particular solution of (2.26)).  Its output, written into the MBF layout by
 * mrcm_nn_scatter, is the starting guess mrcm_options.pcg_x0, scaled in the
 * solver by pcg_x0_scale.  The paper has no learned component; this is an
 * addition on top of its local problems.
 *
 * These calls are the network's kernels and the exchange of data with an
 * MBF handle; the network's parameters, activations and optimiser state are
 * the caller's device buffers.  Tensors are FP32 (loss FP64), layout
 * [batch][channel][d][h][w] with w fastest.  For a subdomain the grid is its
 * local row order viewed as [n2][n1][n0] (mrcm_subdomain_info: the extents
 * along ax[2], ax[1], ax[0]), so one column of the MBFs is one [d][h][w]
 * sample.  Every call is asynchronous on the given HIP stream.
 * Errors: MRCM_EINVAL (null pointer, non-positive size, channels above 16),
 * MRCM_EUNSUPPORTED, MRCM_ENOMEM, MRCM_EHIP.
 */
#ifndef MRCM_NN_H
#define MRCM_NN_H

#include "mrcm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Largest channel count of one convolution (input or output). */
int32_t mrcm_conv3d_max_channels(void);

/*
 * y = conv(x, w) + bias: 3x3x3 cross-correlation with dilation (taps at
 * offsets -dilation, 0, +dilation along each axis) and zero padding, output
 * of the input's size.  x [batch][cin][d][h][w], weights [cout][cin][3][3][3]
 * (taps kd, kh, kw), bias [cout] or NULL, y [batch][cout][d][h][w].
 * relu != 0: y = max(y, 0).  mask (optional, shaped like y): y = 0 where
 * mask <= 0.
 */
mrcm_status mrcm_conv3d_forward(const float *x, const float *weights, const float *bias, float *y,
                                const float *mask, int32_t batch, int32_t cin, int32_t cout, int32_t d,
                                int32_t h, int32_t w, int32_t dilation, int32_t relu, void *stream);

/*
 * Gradients of y = conv(x, w) + bias (same dilation) for a given dL/dy:
 *  dw [cout][cin][27], db [cout] (or NULL): sums over the batch and the grid;
 *  dx [batch][cin][d][h][w] (or NULL to skip): the transposed convolution of
 *    dy, zeroed where dx_mask <= 0 when dx_mask (shaped like x) is given --
 *    with dx_mask = x this applies the derivative of the ReLU that produced x.
 * wt: workspace of cout*cin*27 floats for the transposed weights (needed when
 * dx is requested).  Sums are taken in a fixed order (reproducible).
 */
mrcm_status mrcm_conv3d_backward(const float *x, const float *weights, const float *dy, float *dx, float *dw,
                                 float *db, float *wt, const float *dx_mask, int32_t batch, int32_t cin,
                                 int32_t cout, int32_t d, int32_t h, int32_t w, int32_t dilation, void *stream);

/*
 * Mean squared error over n entries: *loss = sum (y - t)^2 / n (one FP64
 * value in device memory), dy = 2 (y - t) / n.  workspace: 1024 doubles.
 */
mrcm_status mrcm_mse(const float *y, const float *t, float *dy, double *loss, double *workspace, int64_t n,
                     void *stream);

/*
 * mrcm_mse without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training or serving
 * loops, harnesses that forbid hipMalloc).  The same kernels and the same
 * result, bitwise, as mrcm_mse; the partial sums live in the library's own
 * static array of 1024 doubles (8 KiB) per GPU, which every call on that GPU
 * shares and which the GPU keeps until the process ends.  Calls that overlap
 * on one GPU (on different streams, or from different threads) race on that
 * array; calls in stream order do not.  Allocates nothing: no hipMalloc,
 * hipFree or allocating library routine.  Errors: MRCM_EINVAL (null pointer,
 * n <= 0, or n > MRCM_MSE_NOALLOC_MAX_N), MRCM_EHIP.
 */
#define MRCM_MSE_NOALLOC_MAX_N ((int64_t)1 << 40)
mrcm_status mrcm_mse_noalloc(const float *y, const float *t, float *dy, double *loss, int64_t n, void *stream);

/*
 * The encoder-decoder network (the learned form as specified: BF16 weights,
 * FP32 accumulation).  Activations are FP32, channels last:
 * [batch][d][h][w][c] with c fastest.  Master weights are FP32 [cout][cin][27]
 * (taps kd*9 + kh*3 + kw, as mrcm_conv3d_forward's [cout][cin][3][3][3]);
 * a convolution uses them packed to bfloat16 (round to nearest, ties to
 * even) by mrcm_unet_pack:
 *   wf [pad(cout)][27][pad(cin)]  forward weights,
 *   wt [pad(cin)][27][pad(cout)]  the spatially flipped transpose, which makes
 *                                 mrcm_unet_conv compute dL/dx,
 * pad(c) = mrcm_unet_padded(c), c rounded up to 16; at most
 * mrcm_unet_max_channels() (128) channels.
 */
int32_t mrcm_unet_max_channels(void);
int32_t mrcm_unet_padded(int32_t c);
mrcm_status mrcm_unet_pack(const float *w, uint16_t *wf, uint16_t *wt, int32_t cin, int32_t cout, void *stream);

/*
 * y = conv(x, w) + bias: zero-padded 3x3x3 cross-correlation with x and w
 * rounded to bfloat16 and the products summed in FP32 on the matrix cores
 * (implicit GEMM on v_mfma_f32_16x16x16_bf16).  relu != 0: y = max(y, 0);
 * mask (shaped like y, optional): y = 0 where mask <= 0.  With x = dL/dy and
 * the packed transpose wt (cin and cout exchanged) it gives dL/dx.
 */
mrcm_status mrcm_unet_conv(const float *x, const uint16_t *wf, const float *bias, float *y, const float *mask,
                           int32_t batch, int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t relu,
                           void *stream);

/*
 * Weight gradients of y = conv(x, w) + b for a given dL/dy, in FP32:
 * dw [cout][cin][27] = correlation of dy with bfloat16(x) (the operand the
 * forward pass used), db [cout] (or NULL) = sum of dy over the batch and the
 * grid.  workspace: mrcm_unet_wgrad_workspace(...) floats.  The partial sums
 * are added in a fixed order (reproducible).
 */
int64_t mrcm_unet_wgrad_workspace(int32_t batch, int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout);
mrcm_status mrcm_unet_wgrad(const float *x, const float *dy, float *dw, float *db, float *workspace, int32_t batch,
                            int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout, void *stream);

/*
 * Average over 2x2 cells of (d, h) (d, h even; output d/2 x h/2 x w), and
 * nearest upsampling by two over (d, h) (input d x h x w, output 2d x 2h x w);
 * backward != 0: the adjoint (x the gradient at the output, y that at the
 * input).  mrcm_unet_relu_mask: g = 0 where out <= 0.
 */
mrcm_status mrcm_unet_pool(const float *x, float *y, int32_t batch, int32_t d, int32_t h, int32_t w, int32_t c,
                           int32_t backward, void *stream);
mrcm_status mrcm_unet_upsample(const float *x, float *y, int32_t batch, int32_t d, int32_t h, int32_t w, int32_t c,
                               int32_t backward, void *stream);
mrcm_status mrcm_unet_relu_mask(float *g, const float *out, int64_t n, void *stream);

/* [batch][c][voxels] -> [batch][voxels][c] (mrcm_nn_features' inputs to
 * channels last). */
mrcm_status mrcm_nn_channels_last(const float *in, float *out, int32_t batch, int32_t c, int64_t voxels, void *stream);

/*
 * One Adam step (Kingma and Ba, 2015) on n parameters at step t >= 1:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 */
mrcm_status mrcm_adam_step(float *p, const float *g, float *m, float *v, int32_t n, int32_t t, float lr,
                           float b1, float b2, float eps, void *stream);

/*
 * Network samples of the listed subdomains (host array subs, n_subs entries,
 * all with the same grid): sample s = (position of l in subs, column c) in
 * that order, i.e. the columns of subs[0] first.  From the handle's current
 * build:
 *  inp [samples][2][d][h][w]: log kx minus its mean over the subdomain, and
 *       the column's right-hand side divided by its largest magnitude;
 *  tgt [samples][1][d][h][w] (or NULL): the column's solution X divided by
 *       its root mean square (zero columns stay zero).
 * The right-hand sides are formed again into the handle's refinement buffer
 * (allocated on first use), once per build: later calls on the same build
 * reuse them, so a workload may be gathered a few subdomains at a time.
 */
mrcm_status mrcm_nn_features(mrcm_mbfs *mbfs, const int32_t *subs, int32_t n_subs, float *inp, float *tgt,
                             void *stream);

/*
 * x0 (MBF layout, as mrcm_options.pcg_x0) for the listed subdomains from the
 * network's outputs out [samples][d][h][w] in the order of
 * mrcm_nn_features; entries of other subdomains are left as they are.
 */
mrcm_status mrcm_nn_scatter(mrcm_mbfs *mbfs, const int32_t *subs, int32_t n_subs, const float *out, double *x0,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MRCM_NN_H */
