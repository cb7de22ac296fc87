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
 *     holds both penalty blocks; the printed update keeps only the x-block,
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
  double prox_tau_ratio;/* tau1 / tau2 of the prox passes, the product kept at 0.98 / ||K||^2;
                           0 = 1 (equal steps).  The paper tunes its steps by search; an
                           inexact, warm-started prox is sensitive to this ratio              */
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

/*
 * RPCA+UOT-DF (Sec. IV-B, eq. RPCA_UOTDF, Algorithm 3): separation of T
 * frames y_t = Phi_t (s_t + l_t) + noise into a sparse part S >= 0, coupled
 * across consecutive frames by unbalanced transport, and a low-rank part
 * L >= 0:
 *
 *   min 1/2 sum_t ||y_t - Phi_t (s_t + l_t)||^2 + lam ||S||_1 + gam ||L||_*
 *       + kappa sum_{t<T} V_mu(s_t, s_{t+1})
 *
 * by ADMM with the splitting X = S + L, Tn = L, z_t = s_t, w_{t+1} = s_{t+1}
 * (multipliers A, D, b, c); one iteration runs the steps of Algorithm 3:
 * the s-step (one-sided l1 shrink of the sigma-weighted average), the L-step,
 * the x-step (diagonal Phi), the singular-value threshold of L + D, the full
 * prox of every frame pair ((kappa/rho) V_mu at (s_t - b_t, s_{t+1} - c_{t+1}),
 * `prox_iters` warm-started passes of Algorithm 1 over the batch of T - 1
 * pairs), and the multiplier steps.  Stops when the stacked constraint
 * violations ||[X - S - L; L - Tn; z - s; w - s]|| and rho times the stacked
 * changes ||[dX; dTn; dz; dw]|| are both below eps.
 *
 * Readings: the x-step carries rho on (s + l - a) and the A-step subtracts L
 * (both as the augmented Lagrangian the paper writes gives them; the printed
 * updates differ).  The singular-value threshold goes through the T x T Gram
 * matrix of L + D, whose eigenvectors a parallel Jacobi method finds,
 * started from the previous iteration's.
 *
 * Signed sparse part (Sec. IV-B, eq. RPCA_UOTDF_PN; signed_sparse = 1):
 * S = S+ - S- with S+, S- >= 0, an l1 term on each and an OT term for each
 * sign, kappa sum_t (V_mu(s+_t, s+_{t+1}) + V_mu(s-_t, s-_{t+1})).  The paper
 * gives no algorithm for it; the splitting is Algorithm 3's with the sparse
 * block in two signs (X = S+ - S- + L, one z, w pair per sign), minimised in
 * the order S+, S-, L, X, Tn, the prox of all 2 (T - 1) pairs as one batch,
 * then the multipliers.  The stacked residuals include both signs.
 *
 * Layout: frames packed back to back, frame t at element t * nx * ny; y and
 * phi hold T frames, S and L (outputs) T frames.  2 <= frames <= 64.
 */
typedef struct rpca_params {
  int32_t nx, ny, frames;
  int32_t balanced, residual_p, bc;
  double lam;           /* l1 weight of S, >= 0                                             */
  double gam;           /* nuclear-norm weight of L, >= 0                                   */
  double kappa, mu;     /* transport weight (> 0) and growth/decay weight (> 0, unbalanced) */
  double rho;           /* ADMM penalty, > 0                                                */
  int32_t prox_iters, max_iter, check_every;
  double eps;           /* residual threshold (the paper uses 1e-4); <= 0 runs max_iter      */
  uint32_t flags;       /* UOT_NO_GRAPH                                                      */
  double prox_tau_ratio;/* tau1 / tau2 of the prox passes (as in uotdf_params); 0 = 1       */
  int32_t signed_sparse;/* 0: S >= 0 (Algorithm 3); 1: S = S+ - S- (eq. RPCA_UOTDF_PN)      */
  int32_t reserved;
} rpca_params;

typedef struct rpca_report {
  int32_t iters, converged;
  double r_primal, r_dual;
  double seconds;       /* wall time of the call                                            */
  double ms_per_iter;   /* device time per ADMM iteration                                   */
  int32_t jacobi_sweeps;/* sweeps of the last eigensolve                                    */
  int32_t reserved;
} rpca_report;

typedef struct rpca_handle rpca_handle;

uot_status rpca_check_params(const rpca_params *prm);
uot_status rpca_create(const rpca_params *prm, void *hip_stream, rpca_handle **out);
/* y, phi (may be NULL): device, T frames; S, L (may be NULL): device outputs,
 * T frames (S = S+ - S- with signed_sparse).  Every variable starts at zero.
 * Synchronous. */
uot_status rpca_solve(rpca_handle *h, const float *y, const float *phi, float *S, float *L, rpca_report *rep);
/* Copies the split variables and multipliers after the last solve into
 * caller-owned device buffers (X, Tn, A, D: T frames; Z, W, B, C: the pair
 * planes, T - 1 frames, or 2 (T - 1) with signed_sparse: the + pairs, then
 * the - pairs; any may be NULL).  Synchronous. */
uot_status rpca_copy_planes(rpca_handle *h, float *X, float *Tn, float *A, float *D, float *Z, float *W, float *B,
                            float *C);
/* Copies S+ and S- (T frames each; S- is zero without signed_sparse) into
 * caller-owned device buffers (either may be NULL).  Synchronous. */
uot_status rpca_copy_sparse(rpca_handle *h, float *Sp, float *Sm);
void rpca_destroy(rpca_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* UOT_ADMM_H */
