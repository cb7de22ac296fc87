/*
 * uotnet.h -- C ABI of the learned warm start for the unbalanced Beckmann OT
 * prox solver (AMD Instinct MI355X, gfx950).
 *
 * The paper's solver is meant to run warm-started inside outer solvers
 * (Sec. III-B, cost analysis: warm starts and early termination; Sec. IV-A:
 * prox variables initialised to zero and cached between calls).  This
 * library adds a learned start: a small encoder-decoder maps an image pair
 * (p, q) to an initial flux (Mx, My) and dual a, from which the residual is
 * completed as r = D M + q - p so that the start satisfies the constraint.
 * The plain cold-start solver remains the fallback, and its stopping rule
 * decides convergence either way.
 *
 * Network (U-Net, NHWC BF16 activations and weights, FP32 accumulation on
 * the matrix cores, FP32 master weights and Adam moments):
 *   level 0:  conv3x3(in -> ch0) ReLU, conv3x3(ch0 -> ch0) ReLU        = e0
 *   level l:  2x2 average pool, conv(ch_{l-1} -> ch_l) ReLU, conv ReLU = e_l
 *   decoder:  2x nearest upsample, concat with e_l (upsampled first),
 *             conv(ch_{l+1} + ch_l -> ch_l) ReLU, conv(ch_l -> ch_l) ReLU
 *   head:     conv3x3(ch0 -> 3), no activation
 * Inputs: channel 0 = in_scale * p, channel 1 = in_scale * q.  Outputs are
 * normalised targets: (s_flux Mx, s_flux My, s_dual a).  Loss: mean over
 * pixels and batch of the squared error summed over the three channels.
 *
 * Parameters are exchanged with the host in this layout: for every conv in
 * the order enc0a, enc0b, enc1a, enc1b, ..., dec(L-2)a, dec(L-2)b, ...,
 * dec0a, dec0b, head: the weights w[cout][3][3][cin] (row-major) followed by
 * the bias[cout], all FP32.
 *
 * Ownership and errors as in uot.h: device pointers belong to the caller,
 * the handle owns its buffers, status codes only, synchronous calls.
 */
#ifndef UOTNET_H
#define UOTNET_H

#include <stdint.h>

#include "uot.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uotnet uotnet;

typedef struct uotnet_config {
  int32_t height, width;  /* image size; multiples of 2^(levels-1)            */
  int32_t levels;         /* 2..4                                              */
  int32_t ch[4];          /* widths per level, multiples of 8                  */
  int32_t batch_max;      /* largest batch of forward / train_step             */
  uint64_t seed;          /* He-normal initialisation seed                     */
} uotnet_config;

/* Creates the network on the current device, bound to hip_stream (NULL: a
 * private stream).  Weights are He-normal, biases zero. */
uot_status uotnet_create(const uotnet_config *cfg, void *hip_stream, uotnet **out);
void uotnet_destroy(uotnet *net);

/* Number of FP32 values in the host parameter layout above. */
int64_t uotnet_num_params(const uotnet *net);
uot_status uotnet_get_params(uotnet *net, float *host, int64_t n);
/* Replaces the parameters and resets the optimiser state. */
uot_status uotnet_set_params(uotnet *net, const float *host, int64_t n);

/* Forward pass on B pairs (packed planes of height*width pixels each) and
 * conversion to a solver start for DIST: Mx = out0 / s_flux, My = out1 /
 * s_flux (zero on the last column / row), a = out2 / s_dual, r = D M + dst
 * - src.  packed: device state planes (Mx, My, a, r) of B pairs. */
uot_status uotnet_warm_state(uotnet *net, int32_t B, const float *src, const float *dst, float in_scale,
                             float s_flux, float s_dual, uot_state *packed);

/* One training step on B pairs against solver targets (three packed device
 * planes Mx, My, a): forward, loss, backward, Adam (lr; beta1 0.9, beta2
 * 0.999, eps 1e-8).  *loss (host) receives the loss before the update. */
uot_status uotnet_train_step(uotnet *net, int32_t B, const float *src, const float *dst, float in_scale,
                             const float *tMx, const float *tMy, const float *ta, float s_flux, float s_dual,
                             float lr, double *loss);

/* Gradients of the last train step, in the host parameter layout. */
uot_status uotnet_get_grads(uotnet *net, float *host, int64_t n);

/* One convolution on raw device tensors, for layer-level checks:
 *   op 0: out[N][H][W][Cout] = conv3x3(X, W) + bias (ReLU if relu), FP32
 *   op 1: out[N][H][W][Cin]  = input gradient of conv3x3 for output grad G
 *   op 2: out[Cout][9][Cin]  = weight gradient for output grad G, input X
 * X: bf16 [N][H][W][Cin]; Wt: bf16 [Cout][9][Cin]; G: bf16 [N][H][W][Cout];
 * Cin and Cout multiples of 8; bias may be NULL. */
uot_status uotnet_conv(int32_t op, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout, const uint16_t *X,
                       const uint16_t *Wt, const uint16_t *G, const float *bias, int32_t relu, float *out,
                       void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* UOTNET_H */
