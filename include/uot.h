/*
 * uot.h -- C ABI of the unbalanced Beckmann optimal-transport prox solver
 * for AMD Instinct MI355X (gfx950).
 *
 * The solver runs the primal-dual proximal iteration of Lee, Bertrand and
 * Rozell, "Parallel Unbalanced Optimal Transport Regularization for
 * Large-scale Imaging Problems" (Sec. III-B, Algorithm 1), on a 2-D pixel
 * grid with a 2-vector flux per pixel.  One constraint operator serves all
 * modes:
 *
 *     K(z) = D M - x0 + x1 - r          (D = discrete divergence, Sec. II-A)
 *
 *   UOT_DIST        x0 = src = p, x1 = dst = q are fixed; the iteration
 *                   evaluates V_mu(p, q) = min ||M||_{2,1} + mu ||r||_p^p
 *                   s.t. K = 0  (eq. Unbal_OT_beckman; balanced: eq. OT_beckman)
 *   UOT_PROX        the prox of V_mu at (p0, p1) = (src, dst) with step rho,
 *                   over x0, x1 >= 0 (eq. Prox_UOT)
 *   UOT_PROX_FIXED  the prox with the first argument held at s = src and the
 *                   second argument's prox centre p = dst (eq.
 *                   Prox_UOT_specialcase), over x1 >= 0
 *
 * Readings where the paper is silent or ambiguous:
 *   - rho is the prox step of the prox definition (weight 1/(2 rho)), so
 *     the x-update uses theta = tau1 / (rho + tau1).
 *   - bc = 0 (default): zero flux through the right and top edges
 *     (Mx[:, nx-1] = My[ny-1, :] = 0); bc = 1: the literal text, those
 *     entries are free.
 *   - stopping rule: rel_res = max(||K z^k|| / (||x0^k|| + ||x1^k||),
 *     ||(z^{k-1}-z^k)/tau1 - K*(a^{k-1}-a^k)|| / ||K* a^k||) <= tol,
 *     tested every check_every iterations.
 *   - default steps tau1 = 0.99 s / ||K||, tau2 = 0.99 / (s ||K||) with
 *     ||K||^2 = lambda_max(D D*) + (number of identity blocks of K), which
 *     keeps tau1 tau2 ||K||^2 = 0.98 < 1 (Theorem 1), and s the image scale
 *     of the pair: the largest |pixel| of src and dst (1 if both are zero).
 *     The problem is 1-homogeneous (images scaled by t scale M and r by t
 *     and leave a unchanged), so tying tau1 / tau2 to s^2 makes the
 *     iterates of scaled images the scaled iterates.  The paper tunes its
 *     steps by search and fixes no rule;
 *     UOT_ADAPTIVE_STEPS keeps the product tau1 tau2 and rebalances the
 *     ratio at every check by residual balancing (adaptive primal-dual
 *     hybrid gradient, Goldstein, Li and Yuan): when the relative
 *     stationarity residual exceeds 1.5x the relative feasibility residual,
 *     tau1 /= (1 - alpha) and tau2 *= (1 - alpha), and the reverse in the
 *     opposite case; alpha starts at 0.5 and shrinks by 0.95 per change.
 *
 * Memory layout: every image and state plane is FP32, ny rows of nx pixels
 * with x fastest (element j*nx + i is pixel (i, j), the paper's column-major
 * vec with i first); a row stride (pitch) larger than nx may be given.
 *
 * Ownership: every image and state pointer is a DEVICE pointer owned by the
 * caller.  The library never frees, reallocates or keeps them past a call.
 * A handle owns only its workspace (the second copy of the state used for
 * ping-pong, reduction buffers, the captured graphs, tile lists); it is bound
 * to one HIP stream and one device and is not thread-safe.
 *
 * Errors: every entry point returns a uot_status; no C++ exception crosses
 * the ABI.  Argument and shape checks run before any device work.  Input
 * values (non-finite, negative) are checked on the device before the first
 * iteration.  Reaching max_iter is a report status, not an error.
 */
#ifndef UOT_H
#define UOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum uot_status {
  UOT_OK = 0,
  UOT_ERR_ARG = 1,        /* a parameter is out of range or a pointer is NULL      */
  UOT_ERR_SHAPE = 2,      /* grid sizes / offsets inconsistent                     */
  UOT_ERR_STEP = 3,       /* tau1 * tau2 * ||K||^2 >= 1 (Theorem 1)                */
  UOT_ERR_NONFINITE = 4,  /* NaN or Inf in an input image or a warm-start state    */
  UOT_ERR_NEGATIVE = 5,   /* negative pixel in an input image                      */
  UOT_ERR_DEVICE = 6,     /* a HIP call failed or no usable GPU                    */
  UOT_ERR_OOM = 7,        /* workspace allocation failed                           */
  UOT_ERR_MASS = 8,       /* balanced mode, zero-flux boundary, unequal masses     */
  UOT_ERR_TOO_LARGE = 9   /* uot_solve_noalloc: the problem exceeds its scratch    */
} uot_status;

enum { UOT_DIST = 0, UOT_PROX = 1, UOT_PROX_FIXED = 2 };

/* uot_report.status */
enum { UOT_CONVERGED = 0, UOT_MAX_ITER = 1, UOT_DIVERGED = 2 };

/* uot_params.flags */
#define UOT_WARM_START   0x1u  /* start from the caller's state instead of zeros      */
#define UOT_ALLOW_SIGNED 0x4u  /* DIST only: accept negative pixels in src/dst        */
#define UOT_UNSAFE_STEPS 0x8u  /* skip the tau1 tau2 ||K||^2 < 1 check (testing only)  */
#define UOT_NO_GRAPH     0x10u /* launch kernels directly instead of replaying graphs */
#define UOT_AUTOTUNE     0x20u /* time the tile shapes on first use of a size class   */
#define UOT_ADAPTIVE_STEPS 0x40u /* rebalance tau1/tau2 at each check (needs tol > 0)  */
#define UOT_WARM_FALLBACK 0x100u /* with UOT_WARM_START: a pair whose warm state holds a
                                    non-finite value starts from zeros (its report says
                                    cold_start) instead of failing the call               */
#define UOT_RECORD_HISTORY 0x80u /* keep (iterations, rel_res) of every check of the last
                                    solve, per pair (uot_history); the checks then run
                                    every window even with tol <= 0, and the host waits
                                    for each window                                      */

typedef struct uot_params {
  int32_t nx, ny;       /* grid of uot_solve (ignored by uot_solve_batched)           */
  int32_t mode;         /* UOT_DIST, UOT_PROX or UOT_PROX_FIXED                       */
  int32_t balanced;     /* 1: drop r (the balanced variant)                           */
  int32_t residual_p;   /* 1 (mu ||r||_1) or 2 (mu ||r||_2^2)                         */
  int32_t bc;           /* 0 zero flux (default), 1 literal boundary                  */
  double mu;            /* growth/decay weight mu > 0 (unbalanced only)               */
  double rho;           /* prox step rho > 0 (PROX modes)                             */
  double tau1, tau2;    /* primal / dual steps; 0 (both) selects the scaled default
                           0.99 s/||K||, 0.99/(s ||K||) per pair (see above)          */
  int32_t max_iter;     /* iteration cap, >= 0                                        */
  int32_t check_every;  /* iterations between convergence checks (rounded up to even) */
  double tol;           /* stop when rel_res <= tol; <= 0 runs exactly max_iter       */
  uint32_t flags;       /* UOT_* flags above                                          */
  int32_t tile_rows;    /* kernel shape: 0 = autotuned / heuristic; 4, 8, 16, 32 rows per
                           64-wide tile; 116 / 132 = the 16- / 32-row vectorised kernel;
                           316 / 332 = the same with non-temporal stores (for states
                           larger than the last-level cache).  The vectorised shapes
                           take any row layout; they run at full speed when every row
                           starts on a 16-byte boundary (see pitch).
                           1000 * T + rows (4004, 4008, 2016, 4016, 8016, 4032, 8032):
                           temporally blocked, up to T iterations per launch on
                           64 x rows tiles with a T-pixel halo; the last iteration
                           before each convergence check runs in the single-step
                           kernel of the same rows (100 + rows; 4 / 8 for 4004 / 4008).  Every
                           shape computes bit-identical iterates                         */
  int32_t pitch;        /* row stride of uot_solve's planes in elements; 0 = nx.  A
                           pitch rounded up to a multiple of 4 puts every row on a
                           16-byte boundary; the padding is never read or written   */
  int32_t norm;         /* flux norm: UOT_NORM_ISO (0) the paper's l2,1 sum of
                           per-pixel ||(Mx, My)||_2 (eq. Unbal_OT_beckman);
                           UOT_NORM_ANISO (1) the l1,1 sum of |Mx| + |My| (the
                           anisotropic variant: grid min-cost flow).  Changes the
                           flux prox (group vs component shrink), the flux norm in
                           objectives and the dual feasibility (||.||_2 vs ||.||_inf)
                           of the certified bounds                                   */
  int32_t max_groups;   /* upper bound on the workgroups of the persistent launches (the
                           fused iteration, the check, set-up and copy kernels walk the
                           tile list with a fixed grid); rounded down to a multiple of 8
                           (the XCD count), at least 8.  0 = as many as fill the device.
                           Results do not depend on it: every tile is computed alike by
                           whichever workgroup visits it                              */
} uot_params;

enum { UOT_NORM_ISO = 0, UOT_NORM_ANISO = 1 };

/* Device planes of one state.  Required planes by mode:
 *   DIST: Mx, My, a (+ r unless balanced)      PROX: + x0, x1     PROX_FIXED: + x1
 * Unused planes may be NULL. */
typedef struct uot_state {
  float *Mx, *My, *r, *a, *x0, *x1;
} uot_state;

/* Host-side report of one solve (one pair). */
typedef struct uot_report {
  int32_t iters;       /* iterations run                                               */
  int32_t status;      /* UOT_CONVERGED, UOT_MAX_ITER or UOT_DIVERGED                  */
  double rel_res;      /* stopping-rule residual at the last iterate                   */
  double rel_gap;      /* (primal - dual) / |primal|; NaN where no bound is available  */
  double primal;       /* certified upper bound on the optimal value                   */
  double dual;         /* certified lower bound on the optimal value                   */
  double feas;         /* ||K z|| at the last iterate                                  */
  double objective;    /* objective of the raw iterate (no feasibility repair)         */
  double seconds;      /* wall time of the call                                        */
  double tau1, tau2;   /* steps actually used                                          */
  int32_t tile_rows;   /* kernel shape that ran (a tile_rows code; 0 if no iteration)  */
  int32_t cold_start;  /* 1: UOT_WARM_FALLBACK replaced a non-finite warm state by zeros */
} uot_report;

typedef struct uot_handle uot_handle;

/* Validates *prm without touching the GPU.  Returns UOT_OK or the error a
 * uot_create call would return for these parameters. */
uot_status uot_check_params(const uot_params *prm);

/* ||K||^2 for a grid and mode (proof of Theorem 1): lambda_max(D D*) + the
 * number of identity blocks of K.  Host only; returns -1 on bad arguments. */
double uot_knorm2(int32_t nx, int32_t ny, int32_t mode, int32_t balanced, int32_t bc);

/* Creates a handle bound to hip_stream (a hipStream_t; NULL: the handle
 * creates and owns a stream of its own) on the current device.  *out is set
 * to NULL on error.  With the environment variable UOT_PROFILE set at this
 * call, every uot_solve / uot_solve_batched of the handle writes one line
 * per check window (its GPU time from events, the iterations so far, the
 * live and stopped pairs) plus a setup and an end line: UOT_PROFILE=1 to
 * stderr, any other value except 0 appended to the file it names.  The host
 * then waits for every window, so profiled solves run slower. */
uot_status uot_create(const uot_params *prm, void *hip_stream, uot_handle **out);

/* One grid of nx x ny (from the params).  src/dst: device images (see the
 * modes above).  st: caller-owned device state; zeroed first unless
 * UOT_WARM_START.  On return st holds the last iterate and *rep (host) the
 * report.  The call is synchronous with respect to the host. */
uot_status uot_solve(uot_handle *h, const float *src, const float *dst, uot_state *st,
                     uot_report *rep);

/* B independent pairs of uneven sizes, solved together (the T-1 frame-pair
 * problems of Sec. IV-B are one such batch).  nx, ny, offset are HOST
 * arrays of length B; pair b occupies elements [offset[b], offset[b] +
 * nx[b]*ny[b]) of src, dst and of every plane of *packed (ranges must not
 * overlap).  reps: host array of B reports.  Each pair gets its own steps
 * (from its own ||K||) unless tau1/tau2 are given, and stops on its own. */
uot_status uot_solve_batched(uot_handle *h, int32_t B, const int32_t *nx, const int32_t *ny,
                             const int64_t *offset, const float *src, const float *dst,
                             uot_state *packed, uot_report *reps);

/* uot_solve_batched with a row stride per pair: pixel (x, y) of pair b is
 * element offset[b] + y * pitch[b] + x; pitch (HOST, length B, each >= nx[b])
 * may be NULL (pitch = nx).  Pair b spans [offset[b], offset[b] + pitch[b] *
 * (ny[b] - 1) + nx[b]); spans must not overlap.  The padding between rows is
 * never read or written.  Rows starting on 16-byte boundaries (pitches and
 * offsets multiples of 4) let the fused kernel move every pixel with 16-byte
 * accesses; that is the layout to choose for batches of arbitrary widths. */
uot_status uot_solve_batched_pitched(uot_handle *h, int32_t B, const int32_t *nx, const int32_t *ny,
                                     const int32_t *pitch, const int64_t *offset, const float *src,
                                     const float *dst, uot_state *packed, uot_report *reps);

/* Evaluates the report fields (rel_res against prev if prev != NULL, the
 * certified gap, feasibility, objective) of a given state without iterating.
 * Uses the handle's grid. */
uot_status uot_objective(uot_handle *h, const float *src, const float *dst, const uot_state *st,
                         const uot_state *prev, uot_report *out);

/* The convergence history of the last uot_solve / uot_solve_batched on this
 * handle made with UOT_RECORD_HISTORY: for pair `pair`, the iteration count
 * and rel_res (as in uot_report) at every check while the pair was running,
 * the final evaluation included.  Writes min(n, cap) records into the host
 * arrays iters and rel_res (either may be NULL) and the total into *n.
 * UOT_ERR_ARG for a pair outside the last solve or no recorded solve. */
uot_status uot_history(uot_handle *h, int32_t pair, int32_t *iters, double *rel_res, int32_t cap, int32_t *n);

/* Douglas-Rachford splitting of the same problem: a projection-based
 * alternative to Algorithm 1 (Sec. II-B lists Douglas-Rachford among the
 * proximal first-order methods; the paper builds on the primal-dual one).  With G the separable terms of the
 * objective (flux norm, residual penalty, the prox quadratic and x >= 0)
 * and the constraint K z = b (K z = D M - x0 + x1 - r over the terms of the
 * mode; DIST: b = p - q; PROX_FIXED: b = s), one iteration is
 *   z = prox_{gamma G}(w),  y = P(2 z - w),  w <- w + y - z,
 * with P the exact projection onto {K z = b}: y = u - K^T phi,
 * (n I + D D*) phi = K u - b, n the identity blocks of K, solved by the
 * orthonormal DCT-II of the zero-flux grid (the pseudo-inverse when n = 0).
 * One grid (uot_params nx, ny, contiguous rows), zero-flux boundary only
 * (bc = 0); mode, balanced, residual_p, norm, mu, rho, max_iter,
 * check_every, tol and UOT_NO_GRAPH as for uot_solve; w starts at zero.
 * Stops when ||y - z|| <= tol max(1, ||z||) at a check or at max_iter.
 * st receives z (the planes the mode needs; a is not used).  gamma > 0 is
 * the DR step.  Synchronous. */
typedef struct uot_dr_report {
  int32_t iters, status;    /* UOT_CONVERGED / UOT_MAX_ITER / UOT_DIVERGED          */
  double fixed_point_res;   /* ||y - z|| / max(1, ||z||) at the last check         */
  double objective;         /* G(z)                                                */
  double infeasibility;     /* ||K z - b||                                         */
  double seconds;           /* wall time of the call                               */
  double ms_per_iter;       /* device time per iteration                           */
} uot_dr_report;

uot_status uot_dr_solve(uot_handle *h, const float *src, const float *dst, uot_state *st, double gamma,
                        uot_dr_report *rep);

/* Neumann-Poisson solve (alpha I + D D*) phi = rhs on an nx x ny grid with
 * the zero-flux boundary (D D* is the grid Laplacian with Neumann ends; the
 * orthonormal DCT-II diagonalises it, eigenvalues 4 sin^2(pi kx/(2 nx)) +
 * 4 sin^2(pi ky/(2 ny))).  alpha >= 0; at alpha = 0 the constant mode is
 * dropped (phi has zero mean, rhs is projected to zero mean).  rhs, phi:
 * device planes of nx*ny floats (may not alias).  Synchronous. */
uot_status uot_poisson(uot_handle *h, int32_t nx, int32_t ny, double alpha, const float *rhs, float *phi);

/* Poisson-flux start for B pairs (layout as uot_solve_batched): for each pair
 * M0 = -D* phi with D D* phi = c - mean(c), c = dst - src, which is the
 * least-squares flux carrying the mass difference; r0 = D M0 + c, so the
 * start satisfies the constraint; a0 = 0; the free prox arguments start at
 * src / dst.  Pass the state to uot_solve* with UOT_WARM_START.  Needs the
 * zero-flux boundary (bc = 0). */
uot_status uot_init_poisson(uot_handle *h, int32_t B, const int32_t *nx, const int32_t *ny,
                            const int64_t *offset, const float *src, const float *dst, uot_state *packed);

/* The same with row strides (layout as uot_solve_batched_pitched). */
uot_status uot_init_poisson_pitched(uot_handle *h, int32_t B, const int32_t *nx, const int32_t *ny,
                                    const int32_t *pitch, const int64_t *offset, const float *src,
                                    const float *dst, uot_state *packed);

/* Advances the state `in` by `iters` iterations of Algorithm 1 into `out`,
 * with no stopping rule and no checks: the fixed number of warm-started
 * prox passes an outer solver makes per outer iteration (Sec. IV, Algorithms
 * 2 and 3 call the prox that way).  One fused launch per up to T iterations
 * (the handle's kernel shape), alternating between `out` and the handle's
 * shadow copy so that the first launch reads `in` and the last writes `out`.
 * `in` is only read: it is validated like a warm start (a non-finite value
 * gives UOT_ERR_NONFINITE) and its structural boundary zeros are taken as
 * zero whatever it holds there.  No plane of `out` may be a plane of `in`
 * (UOT_ERR_ARG).  One grid (uot_params nx, ny, pitch); the steps are the
 * handle's (tau1, tau2, or the scaled default of the images; no residual
 * balancing).  iters = 0 copies `in` to `out`.  src/dst as for uot_solve.
 * Synchronous. */
uot_status uot_step(uot_handle *h, const float *src, const float *dst, const uot_state *in, uot_state *out,
                    int32_t iters);

/* Profiling aid: captures n (rounded up to even) back-to-back launches of
 * the fused iteration kernel on the handle's grid and stream into a graph,
 * replays it once untimed and once bracketed by HIP events, starting from
 * the caller's state *st (no checks, no zeroing; the state and images are
 * validated first).  A launch runs one iteration, or T for a temporally
 * blocked shape (T = tile_rows / 1000), so *st advances by 2 n T
 * iterations.  *ms_per_iter receives the average event-to-event time per
 * launch; *tile_rows (may be NULL) the kernel shape that ran.  src/dst as
 * for uot_solve. */
uot_status uot_time_iterations(uot_handle *h, const float *src, const float *dst, uot_state *st,
                               int32_t n, double *ms_per_iter, int32_t *tile_rows);

/* The same over a batch layout (as uot_solve_batched_pitched; pitch may be
 * NULL), every pair live: the launch the batched solve runs until its first
 * pair stops. */
uot_status uot_time_iterations_batched(uot_handle *h, int32_t B, const int32_t *nx, const int32_t *ny,
                                       const int32_t *pitch, const int64_t *offset, const float *src,
                                       const float *dst, uot_state *packed, int32_t n,
                                       double *ms_per_iter, int32_t *tile_rows);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): uot_solve
 * without a handle and without any allocation.  The workspace (the shadow
 * copy of the state, the c plane, tile lists, partial sums and per-pair
 * records) is carved from a fixed device array of UOT_NOALLOC_SCRATCH_BYTES
 * that the library holds on every GPU it runs on until the process ends; no
 * hipMalloc, hipHostMalloc, hipFree or graph instantiation is called.
 * Arguments as uot_create + uot_solve (prm: one grid of nx x ny, hip_stream:
 * a hipStream_t or NULL for the default stream), with these differences:
 *   - UOT_AUTOTUNE is rejected (UOT_ERR_ARG); kernels are launched directly
 *     (as with UOT_NO_GRAPH);
 *   - the balanced zero-flux DIST mode reports no certified bounds (primal,
 *     dual, rel_gap are NaN: they need the DCT Poisson solve's matrices);
 *   - UOT_ERR_TOO_LARGE when the workspace does not fit the scratch: at most
 *     UOT_NOALLOC_MAX_PIXELS pixels (pitch * (ny - 1) + nx) and
 *     UOT_NOALLOC_MAX_TILES tiles of the chosen kernel shape.
 * Every call on a GPU uses that GPU's one scratch array, which keeps the last
 * call's contents (everything a call reads from it, it has written first):
 * calls that overlap on one GPU (several host threads or streams) race and
 * must be serialised by the caller.  Synchronous with respect to the host. */
#define UOT_NOALLOC_SCRATCH_BYTES (32u << 20)
#define UOT_NOALLOC_MAX_PIXELS (1 << 20)
#define UOT_NOALLOC_MAX_TILES (1 << 14)
uot_status uot_solve_noalloc(const uot_params *prm, void *hip_stream, const float *src, const float *dst,
                             uot_state *st, uot_report *rep);

/* Releases the handle's workspace.  NULL is a no-op. */
void uot_destroy(uot_handle *h);

const char *uot_status_string(uot_status s);

#ifdef __cplusplus
}
#endif

#endif /* UOT_H */
