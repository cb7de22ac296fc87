// HIP kernels (gfx950) of the ADMM solvers that call the UOT prox.
//
// UOT-DF (Sec. IV-A, Algorithm 2): the element-wise parts of one ADMM
// iteration around the prox launches of the fused Algorithm-1 kernel.
//   df_sx_kernel  s <- max(((x + a) + (z + b))/2 - lam/(2 rho), 0)
//                 x <- (phi y + rho (s - a)) / (phi^2 + rho)
//                 p <- s - b (the prox centre),  zo <- z (z before the prox)
//   df_ab_kernel  a <- a + x - s,  b <- b + z - s
// Both stream their planes once (HBM-bound, 9 and 7 planes of 4 bytes per
// pixel).  On the last iteration of a check window they also leave per-block
// FP64 partial sums of the residuals, which df_reduce_kernel adds up in a
// fixed order (no atomics, so the result does not depend on timing).
#include "uot_admm_internal.hpp"

namespace uot {

namespace {

constexpr int RB = 256;  // threads per block of the element-wise kernels

// Sums v over the block into *out (thread 0 writes).
__device__ __forceinline__ void block_sum(double v, double* out) {
  __shared__ double red[RB / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < RB / 64; ++i) t += red[i];
    *out = t;
  }
  __syncthreads();
}

}  // namespace

__global__ __launch_bounds__(RB) void df_sx_kernel(DfArgs A) {
  double dx2 = 0.0;
  const float rho = A.rho, thr = A.thr;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < A.n; i += (long)gridDim.x * RB) {
    const float x = A.x[i], a = A.a[i], b = A.b[i], z = A.z[i];
    const float ph = A.phi ? A.phi[i] : 1.f;
    const float s = fmaxf(0.5f * ((x + a) + (z + b)) - thr, 0.f);
    const float xn = (ph * A.y[i] + rho * (s - a)) / (ph * ph + rho);
    A.s[i] = s;
    A.x[i] = xn;
    A.p[i] = s - b;
    A.zo[i] = z;
    if (A.record) {
      const float d = xn - x;
      dx2 += (double)d * d;
    }
  }
  if (A.record) block_sum(dx2, A.partial + 3 * blockIdx.x + 1);
}

__global__ __launch_bounds__(RB) void df_ab_kernel(DfArgs A) {
  double rp2 = 0.0, dz2 = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < A.n; i += (long)gridDim.x * RB) {
    const float x = A.x[i], s = A.s[i], z = A.z[i];
    A.a[i] = A.a[i] + (x - s);
    A.b[i] = A.b[i] + (z - s);
    if (A.record) {
      const float e = x - s, f = z - s, g = z - A.zo[i];
      rp2 += (double)e * e + (double)f * f;
      dz2 += (double)g * g;
    }
  }
  if (A.record) {
    block_sum(rp2, A.partial + 3 * blockIdx.x);
    block_sum(dz2, A.partial + 3 * blockIdx.x + 2);
  }
}

// out[j] = sum over blocks of partial[3 b + j], j = 0..2 (one block).
__global__ __launch_bounds__(RB) void df_reduce_kernel(const double* partial, int nblocks, double* out) {
  for (int j = 0; j < 3; ++j) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RB) v += partial[3 * b + j];
    block_sum(v, out + j);
  }
}

// Input check: counts non-finite entries of y, phi, s0 and negative entries
// of s0 (out[0], out[1]).
__global__ __launch_bounds__(RB) void df_validate_kernel(long n, const float* y, const float* phi, const float* s0,
                                                          double* partial) {
  double bad = 0.0, neg = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
    const float v = y[i], w = s0[i], f = phi ? phi[i] : 1.f;
    bad += (isfinite(v) && isfinite(w) && isfinite(f)) ? 0.0 : 1.0;
    neg += w < 0.f ? 1.0 : 0.0;
  }
  block_sum(bad, partial + 3 * blockIdx.x);
  block_sum(neg, partial + 3 * blockIdx.x + 1);
  if (threadIdx.x == 0) partial[3 * blockIdx.x + 2] = 0.0;
}

int df_blocks(long n) { return (int)std::min<long>(1024, std::max<long>(1, (n + RB - 1) / RB)); }

hipError_t launch_df_sx(const DfArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(df_sx_kernel, dim3(df_blocks(a.n)), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_df_ab(const DfArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(df_ab_kernel, dim3(df_blocks(a.n)), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_df_reduce(const double* partial, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(df_reduce_kernel, dim3(1), dim3(RB), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_df_validate(long n, const float* y, const float* phi, const float* s0, double* partial,
                              hipStream_t s) {
  hipLaunchKernelGGL(df_validate_kernel, dim3(df_blocks(n)), dim3(RB), 0, s, n, y, phi, s0, partial);
  return hipGetLastError();
}

}  // namespace uot
