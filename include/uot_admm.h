/*
 * uot_admm.h -- C ABI of the ADMM solvers of Sec. IV that call the UOT prox
 * (Lee, Bertrand and Rozell, "Parallel Unbalanced Optimal Transport
 * Regularization for Large-scale Imaging Problems"), for AMD Instinct MI355X.
 *
 * UOT-DF (Sec. IV-A, eqs. UOT-DF and BPDN+UOT-DF, Algorithm 2): one frame of
 * the dynamic filter,
 *
 *     s* = argmin_{s >= 0}  1/2 ||y - Phi s||^2 + lam ||s||_1 + kappa V_mu(s, s0),
 *
 * with Phi diagonal (phi = its diagonal; NULL = identity, the denoising case
 * of the paper's run-time study) and s0 the prediction of the frame.  ADMM
 * splits s = x = z (multipliers a, b, penalty rho); one iteration runs
 *
 *     s <- max(((x + a) + (z + b)) / 2 - lam / (2 rho), 0)
 *     x <- (phi y + rho (s - a)) / (phi^2 + rho)
 *     z <- prox_{(kappa/rho) V_mu(., s0)}(s - b): `prox_iters` passes of
 *          Algorithm 1 in the one-argument-fixed mode (eq.
 *          Prox_UOT_specialcase), warm-started from the previous ADMM
 *          iteration's prox state
 *     a <- a + x - s,   b <- b + z - s
 *
 * and stops when ||[x - s; z - s]|| < eps and rho ||[x - x_prev; z - z_prev]||
 * < eps (tested every check_every iterations) or at max_iter.
 *
 * Readings where the paper is silent or inconsistent:
 *   - the s-step minimises the augmented Lagrangian the paper writes, which
 *     holds both penalty blocks; the printed line keeps only the x-block,
 *     with which the iteration converges to the transport-free least-squares
 *     point (s = y for Phi = I).  The l1 threshold is lam / (2 rho).
 *   - V_mu is symmetric in its two arguments, so the z-prox of V_mu(z, s0) is
 *     the one-argument-fixed prox with s0 held.
 *   - every variable, and the prox state, starts at zero (Algorithm 2).
 *
 * Memory layout: every plane is FP32, ny rows of nx pixels, x fastest.
 * Ownership: y, phi, s0 and s are DEVICE pointers owned by the caller; the
 * handle owns its workspace (the ADMM and prox states) and is bound to one
 * stream and device; not thread-safe.
 * Errors: uot_status codes of uot.h; argument checks run before device work.
 */
#ifndef UOT_ADMM_H
#define UOT_ADMM_H

#include <stdint.h>

#include "uot.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uotdf_params {
  int32_t nx, ny;
  int32_t balanced;     /* 1: balanced transport (W instead of V_mu; the r plane is dropped) */
  int32_t residual_p;   /* 1 or 2, as in uot_params                                          */
  int32_t bc;           /* 0 zero flux (default), 1 literal boundary                         */
  double kappa;         /* weight of the transport term, > 0                                  */
  double mu;            /* growth/decay weight of V_mu, > 0 (unbalanced)                      */
  double lam;           /* l1 weight (BPDN+UOT-DF), >= 0; 0 = UOT-DF                          */
  double rho;           /* ADMM penalty, > 0                                                  */
  int32_t prox_iters;   /* Algorithm-1 passes per ADMM iteration, >= 1                        */
  int32_t max_iter;     /* ADMM iteration cap, >= 1                                           */
  int32_t check_every;  /* ADMM iterations between residual tests, >= 1                       */
  double eps;           /* residual threshold (the paper uses 1e-3); <= 0 runs max_iter         */
  uint32_t flags;       /* UOT_NO_GRAPH: launch directly instead of replaying graphs           */
} uotdf_params;

typedef struct uotdf_report {
  int32_t iters;        /* ADMM iterations run                                                */
  int32_t converged;    /* 1 if both residuals fell below eps                                 */
  double r_primal;      /* ||[x - s; z - s]|| at the last test                                */
  double r_dual;        /* rho ||[x - x_prev; z - z_prev]|| at the last test                  */
  double seconds;       /* wall time of the call                                              */
  double ms_per_iter;   /* device time per ADMM iteration, from events around the windows     */
} uotdf_report;

typedef struct uotdf_handle uotdf_handle;

/* Validates *prm without touching the GPU. */
uot_status uotdf_check_params(const uotdf_params *prm);

/* Creates a handle for one grid size on the current device, bound to
 * hip_stream (a hipStream_t; NULL = a stream the handle creates and owns,
 * which synchronises with the null stream). */
uot_status uotdf_create(const uotdf_params *prm, void *hip_stream, uotdf_handle **out);

/* Solves one frame: y (observation), phi (diagonal of Phi, or NULL),
 * s0 (prediction, >= 0) are read; s (output) receives the estimate.  Every
 * variable starts at zero.  Synchronous. */
uot_status uotdf_solve(uotdf_handle *h, const float *y, const float *phi, const float *s0, float *s,
                       uotdf_report *rep);

/* Copies the ADMM planes x, z, a, b left by the last solve into caller-owned
 * device buffers of nx*ny floats (any may be NULL).  Synchronous. */
uot_status uotdf_copy_planes(uotdf_handle *h, float *x, float *z, float *a, float *b);

void uotdf_destroy(uotdf_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* UOT_ADMM_H */
