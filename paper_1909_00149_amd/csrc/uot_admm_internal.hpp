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

int df_blocks(long n);
hipError_t launch_df_sx(const DfArgs& a, hipStream_t s);
hipError_t launch_df_ab(const DfArgs& a, hipStream_t s);
hipError_t launch_df_reduce(const double* partial, int nblocks, double* out, hipStream_t s);
hipError_t launch_df_validate(long n, const float* y, const float* phi, const float* s0, double* partial,
                              hipStream_t s);

}  // namespace uot
