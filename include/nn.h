/*
 * nn.h -- C ABI of the warm-start network in libtt.so.
 *
 * A 3-D U-Net predicts the factor tau of the traveltime T = T0 * tau (the
 * multiplicative factorisation of Sec. 3.1) from the model, so that the fast
 * sweeping solve of Eq. (4) starts close to its fixed point.  These entry points
 * are its layers' forward and backward passes and the optimiser.
 *
 * Conventions
 *   - Every array is caller-owned DEVICE memory; nothing is retained or freed.
 *   - Activations and activation gradients are bf16 (uint16_t storage,
 *     round-to-nearest-even), channels last: [npos][c_total] with npos =
 *     nbatch * D * H * W positions in (n, z, y, x) order; a layer reads or writes
 *     the channel range [c_off, c_off + c) of a buffer with c_total channels
 *     (this is how skip connections are concatenated without copies).
 *   - Weights, biases, their gradients and optimiser state are fp32.  3^3
 *     convolution weights are [27][cin][cout] with tap t = (dz+1)*9 + (dy+1)*3 +
 *     (dx+1); up-sampling weights [8][cin][cout] with child s = a*4 + b*2 + c.
 *   - D, H, W >= 1; 3^3 convolutions pad with zeros.  cin of a 3^3 convolution
 *     is a multiple of 16 (pad input features with zero channels and zero
 *     weights); cout is a multiple of 16 and at most 64.
 *   - Every call only enqueues work on `stream` (a hipStream_t, NULL = default).
 *   - Returns 0, or -1 (invalid argument, host-checked) / -2 (HIP error); see
 *     tt_last_error().
 */
#ifndef NN_H
#define NN_H

#include <stddef.h>
#include <stdint.h>

#include "tt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Warm-start feature and target scaling (fixed parts of the model's definition):
 *   feature 0 = (s / s0 - 1) * NN_FEAT_S      (s0 = slowness constant of the source)
 *   feature 1 = xi * NN_FEAT_A, feature 2 = eta * NN_FEAT_A
 *   feature 3 = |X - X_s| * NN_FEAT_D         (straight distance to the source, km)
 *   target    = (tau - 1) * NN_TARGET_SCALE                                        */
#define NN_FEAT_S 5.0
#define NN_FEAT_A 25.0
#define NN_FEAT_D 0.01
#define NN_TARGET_SCALE 10.0

/* Range of the initial tau that nn_warm_init hands to the solver: a
 * prediction outside it is clamped (a NaN becomes 1), so that a poor network
 * costs iterations only. */
#define NN_TAU_INIT_MIN 0.25
#define NN_TAU_INIT_MAX 4.0

/* Scratch of nn_mse: loss holds 2 + 2 * NN_MSE_MAX_BLOCKS floats. */
#define NN_MSE_MAX_BLOCKS 1024
#define NN_MSE_LOSS_FLOATS (2 + 2 * NN_MSE_MAX_BLOCKS)

/* fp32 -> bf16 conversion of n values. */
int nn_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream);

/* bf16 -> fp32 conversion of n values. */
int nn_from_bf16(const uint16_t* x, int64_t n, float* y, void* stream);

/* Pack fp32 weights W[27][cin][cout] into the bf16 operand fragments used by
 * the matrix-core convolution (size 27*cin*cout bf16).  flip = 1 packs the
 * weights of the data-gradient convolution instead (tap mirrored, cin and cout
 * exchanged: a [27][cout][cin] fragment set). */
int nn_conv3_pack(const float* W, int cin, int cout, int flip, uint16_t* frag, void* stream);

/* y = act(conv3(x) + bias) over [nbatch][D][H][W] positions on matrix cores
 * (bf16 operands, fp32 accumulation).  act = ReLU if relu != 0.  bias may be
 * NULL.  frag from nn_conv3_pack(flip = 0), or flip = 1 for data gradients. */
int nn_conv3_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cx_total, int cx_off, int cin,
                 const uint16_t* frag, const float* bias, int cout, int relu, uint16_t* y, int cy_total,
                 int cy_off, void* stream);

/* Weight and bias gradients of a 3^3 convolution: gW[27][cin][cout] =
 * sum_p x[p + d_t][ci] gz[p][co], gb[co] = sum_p gz[p][co] (fp32, overwritten).
 * work: fp32 scratch of nn_conv3_wgrad_work(...) bytes. */
size_t nn_conv3_wgrad_work(int nbatch, int D, int H, int W, int cin, int cout);
int nn_conv3_wgrad(const uint16_t* x, int nbatch, int D, int H, int W, int cx_total, int cx_off, int cin,
                   const uint16_t* gz, int cg_total, int cg_off, int cout, float* gW, float* gb, float* work,
                   size_t work_bytes, void* stream);

/* g_out = g * (y > 0) (ReLU backward from the layer's output y), bf16. */
int nn_relu_mask(const uint16_t* g, const uint16_t* y, int64_t npos, int c_total, int c_off, int c,
                 uint16_t* g_out, int co_total, int co_off, void* stream);

/* 2^3 max pooling (D, H, W even) and its backward: the gradient goes to the
 * first maximal child in (z, y, x) order; accumulate != 0 adds to gx. */
int nn_pool_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int c_total, int c_off, int c, uint16_t* y,
                void* stream);
int nn_pool_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int c_total, int c_off,
                int c, uint16_t* gx, int accumulate, void* stream);

/* 2^3 stride-2 transposed convolution from [D][H][W] to [2D][2H][2W]:
 * y[2p + s][o] = b[o] + sum_i x[p][i] Wup[s][i][o] (fp32 weights and
 * arithmetic; x is [npos][cin] contiguous), and its backward (gx bf16, may be
 * NULL; gW[8][cin][cout], gb[cout] fp32 overwritten; work as for
 * nn_up_wgrad_work). */
int nn_up_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cin, const float* Wup, const float* b,
              int cout, uint16_t* y, int cy_total, int cy_off, void* stream);
size_t nn_up_wgrad_work(int nbatch, int D, int H, int W, int cin, int cout);
int nn_up_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int cin, int cout,
              int cg_total, int cg_off, const float* Wup, uint16_t* gx, float* gW, float* gb, float* work,
              size_t work_bytes, void* stream);

/* 1x1 head: y[p] = b + sum_i x[p][i] w[i] (fp32 out, cin <= 127), and its
 * backward (gx bf16, may be NULL; gw[cin], gb[1] fp32 overwritten; work as for
 * nn_head_work). */
int nn_head_fwd(const uint16_t* x, int64_t npos, int cin, const float* w, const float* b, float* y, void* stream);
size_t nn_head_work(int64_t npos, int cin);
int nn_head_bwd(const uint16_t* x, const float* gy, int64_t npos, int cin, const float* w, uint16_t* gx,
                float* gw, float* gb, float* work, size_t work_bytes, void* stream);

/* Weighted mean squared error: loss[0] = sum m (y - t)^2 / max(sum m, 1),
 * loss[1] = max(sum m, 1), gy = 2 m (y - t) / max(sum m, 1) (m = 1 where mask is
 * NULL).  loss must hold NN_MSE_LOSS_FLOATS floats (the tail is scratch).  The
 * sums run in a fixed order (deterministic). */
int nn_mse(const float* y, const float* t, const float* mask, int64_t n, float* loss, float* gy, void* stream);

/* Adam step (bias-corrected) on n fp32 parameters; step >= 1. */
int nn_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float beta1, float beta2,
            float eps, void* stream);

/* ------------------------------------------------------------------ U-Net
 * Four levels with channels ch[0..3] (multiples of 16, ch[3] <= 64, 2 ch[l] <= 64
 * for l < 3): two 3^3 convolutions with ReLU per level, 2^3 max pooling down,
 * 2^3 stride-2 transposed convolutions up, skip concatenation [up, skip], 1x1
 * head.  in_ch real input features (<= 16) are read from a 16-channel input;
 * channels in_ch..15 are ignored.
 *
 * Parameters are one fp32 array in this order, each convolution W [27][ci][co]
 * then b [co]: e1a (in_ch -> c0), e1b, e2a (c0 -> c1), e2b, e3a (c1 -> c2), e3b,
 * bna (c2 -> c3), bnb, d3a (2 c2 -> c2), d3b, d2a (2 c1 -> c1), d2b, d1a (2 c0 -> c0),
 * d1b; then the up-samplings W [8][ci][co], b [co]: u3 (c3 -> c2), u2 (c2 -> c1),
 * u1 (c1 -> c0); then head w [c0], b [1].  Gradients use the same layout. */
typedef struct {
    int32_t ch[4];
    int32_t in_ch;
} nn_unet_cfg;

/* Number of fp32 parameters / bf16 fragment elements (0 if cfg is invalid). */
size_t nn_unet_nparams(const nn_unet_cfg* cfg);
size_t nn_unet_nfrag(const nn_unet_cfg* cfg);

/* Workspace bytes for a batch of nbatch inputs of D x H x W (multiples of 8);
 * train != 0 adds the gradient buffers that nn_unet_backward needs. */
size_t nn_unet_workspace(const nn_unet_cfg* cfg, int nbatch, int D, int H, int W, int train);

/* Round the parameters into the convolution fragments (forward and
 * data-gradient); call after every parameter update. */
int nn_unet_pack(const nn_unet_cfg* cfg, const float* params, uint16_t* frag, void* stream);

/* y [nbatch][D][H][W] (fp32) from x [nbatch][D][H][W][16] (bf16).  The
 * activations stay in ws for a following nn_unet_backward when train != 0
 * (ws then sized with train = 1). */
int nn_unet_forward(const nn_unet_cfg* cfg, const float* params, const uint16_t* frag, const uint16_t* x, int nbatch,
                    int D, int H, int W, float* y, void* ws, size_t ws_bytes, int train, void* stream);

/* Gradient of sum(gy * y) for every parameter (overwrites grad), using the
 * activations of the last nn_unet_forward(train = 1) on the same x and ws. */
int nn_unet_backward(const nn_unet_cfg* cfg, const float* params, const uint16_t* frag, const uint16_t* x,
                     const float* gy, int nbatch, int D, int H, int W, float* grad, void* ws, size_t ws_bytes,
                     void* stream);

/* ------------------------------------------------------------- warm start
 * The network runs on the coarse nodes (stride * z, stride * y, stride * x) of
 * the solver grid, padded with zeros to D x H x W (each >= (n - 1) / stride + 1).
 *
 * nn_warm_features: feat [nsrc][D][H][W][16] bf16 (features above, zero outside
 *   the grid and in channels 4..15).  src_pos [nsrc][3] in axis coordinates,
 *   src_par [nsrc][3] (s0, xi0, eta0) as from tt_source_params.
 * nn_warm_target: target [nsrc][D][H][W] = (tau - 1) * NN_TARGET_SCALE at the
 *   coarse nodes of tau [nsrc][N], 0 outside; mask (may be NULL) 1 inside, 0 outside.
 * nn_warm_init: tau_init [nsrc][N] = 1 + pred / NN_TARGET_SCALE, interpolated
 *   trilinearly from the coarse nodes (held constant past the last one) and
 *   clamped to [NN_TAU_INIT_MIN, NN_TAU_INIT_MAX]. */
int nn_warm_features(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
                     const double* src_pos, const double* src_par, int32_t stride, int32_t D, int32_t H, int32_t W,
                     uint16_t* feat, void* stream);
int nn_warm_target(const tt_grid* grid, int32_t nsrc, const double* tau, int32_t stride, int32_t D, int32_t H,
                   int32_t W, float* target, float* mask, void* stream);
int nn_warm_init(const tt_grid* grid, int32_t nsrc, const float* pred, int32_t stride, int32_t D, int32_t H, int32_t W,
                 double* tau_init, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NN_H */
