// Internal interface between the ADMM host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "uot_internal.hpp"

namespace uot {

// Element-wise parts of one UOT-DF ADMM iteration (Algorithm 2).
struct DfArgs {
  long n;                      // pixels
  const float *y, *phi;        // observation, diagonal of Phi (nullptr = identity)
  float *s, *x, *a, *b;        // ADMM planes
  float *p, *zo;               // prox centre s - b; z before the prox
  const float* z;              // the prox state's free argument (z)
  float rho, thr;              // ADMM penalty; l1 threshold lam / (2 rho)
  int record;                  // leave residual partials (last iteration of a window)
  double* partial;             // [blocks][3]: ||x-s||^2 + ||z-s||^2, ||x-x_prev||^2, ||z-z_prev||^2
};

// Element-wise parts of one RPCA+UOT-DF ADMM iteration (Algorithm 3).
// Frames are packed back to back (frame t at offset t * npx); the frame-pair
// planes (b, c, prox centres, the prox state's z and w) hold T - 1 frames.
constexpr int RP_MAX_FRAMES = 64;  // the Gram eigensolve keeps T x T in LDS
constexpr int RP_SLOTS = 5;        // residual partial slots per block
constexpr int RP_MAX_SWEEPS = 40;  // Jacobi sweeps per eigensolve
constexpr int RP_MAX_REFINE = 3;  // refinement passes of the warm start before the sweeps
struct RpArgs {
  long npx;                    // pixels per frame
  int T;                       // frames
  const float *y, *phi;        // observations, diagonal of Phi (nullptr = identity)
  float *S, *L, *X, *Tn, *A, *D;
  float *B, *C;                // multipliers of z (pair t) and w (pair t: frame t + 1)
  float *P0, *P1;              // prox centres s_t - b_t, s_{t+1} - c_{t+1}
  float *zo, *wo;              // z, w before the prox
  const float *Z, *W;          // the prox state's free arguments x0 (z_t), x1 (w_{t+1})
  float rho, lam;
  int record;
  double* partial;             // [RP_SLOTS][pstride]: 0 ||X-S-L||^2+||z-s||^2+||w-s||^2, 1 ||dX||^2,
                               // 2 ||L-Tn||^2, 3 ||dTn||^2, 4 ||dz||^2+||dw||^2
  const float* Wm;             // T x T matrix of the singular-value threshold (svt apply)
  int pstride;                 // partial slot j of block b at partial[j * pstride + b]
  float* Sm;                   // S- of the signed sparse part (nullptr: S >= 0, Algorithm 3)
  long mo;                     // offset of the - pairs in the pair planes (signed sparse part)
};

// Number of partials each residual slot holds after a recorded iteration.
struct RpCounts {
  int n[RP_SLOTS];
};

int df_blocks(long n);
hipError_t launch_rp_sx(const RpArgs& a, int bx, hipStream_t s);  // grid bx x T
hipError_t launch_rp_gram(const RpArgs& a, int blocks, double* gpart, hipStream_t s);
hipError_t launch_rp_gram_reduce(const double* gpart, int blocks, int T, double* G, hipStream_t s);
// Eigensolve of G warm-started from V (updated in place): refinement by
// matrix products, else Jacobi sweeps; then Wm.  lam holds 64 eigenvalues,
// sweeps the number of Jacobi sweeps run (0 after a refinement).
hipError_t launch_rp_eig(const double* G, int T, double thr, double* V, double* lam, float* Wm, int* sweeps,
                         hipStream_t s);
hipError_t launch_rp_svt_apply(const RpArgs& a, int blocks, hipStream_t s);
hipError_t launch_rp_dual(const RpArgs& a, int bx, hipStream_t s);  // grid bx x T
hipError_t launch_rp_reduce(const double* partial, int pstride, const RpCounts& cnt, double* out, hipStream_t s);
hipError_t launch_rp_dualsx(const RpArgs& a, int bx, hipStream_t s);  // rp_dual + the next rp_sx
hipError_t launch_rp_sub(long n, const float* a, const float* b, float* out, hipStream_t s);
hipError_t launch_rp_validate(long n, const float* y, const float* phi, double* partial, int blocks, hipStream_t s);
hipError_t launch_df_sx(const DfArgs& a, hipStream_t s);
hipError_t launch_df_ab(const DfArgs& a, hipStream_t s);
hipError_t launch_df_absx(const DfArgs& a, hipStream_t s);  // df_ab of one iteration + df_sx of the next
hipError_t launch_df_reduce(const double* partial, int nblocks, double* out, hipStream_t s);
hipError_t launch_df_validate(long n, const float* y, const float* phi, const float* s0, double* partial,
                              hipStream_t s);

}  // namespace uot
