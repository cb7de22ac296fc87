// HIP kernels (gfx950) of the solver that are not instantiated per mode:
// input validation and set-up, the per-pair reduction with the stopping
// decision, the copy of live pairs and the dual (Poisson) kernel, plus the
// dispatch to the per-mode instantiations of the fused Algorithm-1 kernels
// and the check (uot_iter_mode.hip, compiled once per mode).
#include "uot_iter_impl.hpp"

namespace uot {

// Input validation, c = q - p, and state initialisation (K8).
__global__ __launch_bounds__(BLOCK) void setup_kernel(SetupArgs A) {
  const int lx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
    const Tile tl = A.tiles[t];
    const PairInfo P = A.pairs[tl.pair];
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    for (int ly = wv; ly < A.tile_rows; ly += 4) {
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const long o = P.off + (long)gy * pitch + gx;
      const float s = A.src[o], d = A.dst[o];
      acc[U_NONFIN_IN] += (isfinite(s) ? 0.0 : 1.0) + (isfinite(d) ? 0.0 : 1.0);
      acc[U_NEG] += (s < 0.f ? 1.0 : 0.0) + (d < 0.f ? 1.0 : 0.0);
      acc[U_SUMS] += s;
      acc[U_SUMD] += d;
      acc[U_SQS] += (double)s * s;
      acc[U_SQD] += (double)d * d;
      acc[U_MAXIN] = fmax(acc[U_MAXIN], (double)fmaxf(fabsf(s), fabsf(d)));
      if (A.mode == 0 && A.write_c) A.c[o] = d - s;
      const bool zx = (A.bc == 0 && gx == nx - 1), zy = (A.bc == 0 && gy == ny - 1);
      if (!A.warm) {
        if (A.write_state) {
          A.st.Mx[o] = 0.f;
          A.st.My[o] = 0.f;
          A.st.a[o] = 0.f;
          if (A.resid != R_BAL) A.st.r[o] = 0.f;
          if (A.mode == 1) A.st.x0[o] = 0.f;
          if (A.mode != 0) A.st.x1[o] = 0.f;
        }
      } else {
        const float mx = A.st.Mx[o], my = A.st.My[o], a = A.st.a[o];
        bool fin = isfinite(mx) && isfinite(my) && isfinite(a);
        if (A.resid != R_BAL) fin = fin && isfinite(A.st.r[o]);
        if (A.mode == 1) fin = fin && isfinite(A.st.x0[o]);
        if (A.mode != 0) fin = fin && isfinite(A.st.x1[o]);
        acc[U_NONFIN_ST] += fin ? 0.0 : 1.0;
        if (A.write_state) {
          if (zx) A.st.Mx[o] = 0.f;
          if (zy) A.st.My[o] = 0.f;
        }
      }
    }
    block_reduce_store(acc, kMaxSlotsSetup, A.partial + (long)t * NS);
  }
}

// Stopping decision for pair b after a window of W iterations (device side,
// so that captured windows need no host round trip).
// The pair's flag, iteration count, norm and adaptation factor come in
// preloaded (read at the start of the reduction, in flight with it).
struct DecidePre {
  int active, iters;
  double xnorm, alpha;
};

__device__ void decide_pair(const DecideArgs& A, int b, const double* S, const PairInfo& P0, const DecidePre& pre) {
  if (!pre.active) return;
  const int iters = pre.iters + A.W;
  A.iters[b] = iters;
  bool done = false;
  if (A.check && !A.keep_rel) {
    const double xn = A.mode == 0 ? pre.xnorm : sqrt(S[S_X0SQ]) + sqrt(S[S_X1SQ]);
    const double p = sqrt(S[S_PRES2]) / fmax(xn, 1e-30);
    const double d = sqrt(S[S_STAT2]) / fmax(sqrt(S[S_KA2]), 1e-30);
    const double rel = fmax(p, d);
    A.rel_res[b] = rel;
    if (S[S_NONFIN] > 0.0 || !isfinite(rel)) {
      A.status[b] = 2;
      done = true;
    } else if (A.tol > 0.0 && rel <= A.tol) {
      A.status[b] = 0;
      done = true;
    }
    if (!done && A.adaptive && !A.final_pass) {
      // residual balancing: keep tau1*tau2, move the ratio toward the side
      // whose relative residual lags
      PairInfo& P = A.pairs[b];
      const double al = pre.alpha;
      double t1 = P0.tau1, t2 = P0.tau2;
      bool ch = false;
      if (d > 1.5 * p) {
        t1 /= (1.0 - al);
        t2 *= (1.0 - al);
        ch = true;
      } else if (p > 1.5 * d) {
        t1 *= (1.0 - al);
        t2 /= (1.0 - al);
        ch = true;
      }
      if (ch) {
        A.alpha[b] = al * 0.95;
        P.tau1 = (float)t1;
        P.tau2 = (float)t2;
        P.theta = A.mode == 0 ? 0.f : (float)(t1 / (A.rho + t1));
        P.mutau = (float)(A.mu * t1);
        P.inv2mt = (float)(1.0 / (1.0 + 2.0 * A.mu * t1));
      }
    }
  }
  if (!done && (A.final_pass || iters >= A.max_iter)) {
    A.status[b] = 1;
    done = true;
  }
  if (done) A.active[b] = 0;
}

// Per-pair sums of tile partials in a fixed order (deterministic); with
// do_decide, thread 0 then takes the pair's stopping decision.
__global__ __launch_bounds__(BLOCK) void pair_reduce_kernel(const PairInfo* pairs, const double* partial,
                                                            uint32_t max_mask, double* sums, DecideArgs dec,
                                                            int do_decide) {
  const int b = blockIdx.x;
  const PairInfo P = pairs[b];
  // uniform: a stopped pair keeps its record; the final pass still sums it
  const int act = do_decide ? dec.active[b] : 0;
  if (do_decide && !act && !dec.final_pass) return;
  DecidePre pre{act, 0, 0.0, 0.0};
  if (do_decide && threadIdx.x == 0) {
    pre.iters = dec.iters[b];
    if (dec.mode == 0) pre.xnorm = dec.xnorm[b];
    if (dec.adaptive) pre.alpha = dec.alpha[b];
  }
  // thread (group g, slot s): slot s of the pair's tiles g, g + 16, ..., so a
  // wave reads four whole partial rows per step
  static_assert(NS == 16 && BLOCK == 256, "16 slots x 16 groups");
  __shared__ double red[16][NS + 1];
  __shared__ double fin[NS];
  const int s = threadIdx.x & 15, g = threadIdx.x >> 4;
  const bool mx = (max_mask >> s) & 1u;
  double v = 0.0;
  const double* row = partial + (long)P.tile_begin * NS + s;
  int t = g;
  // eight loads in flight per thread, combined in tile order
  for (; t + 16 * 7 < P.tile_count; t += 16 * 8) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = row[(long)(t + 16 * u) * NS];
#pragma unroll
    for (int u = 0; u < 8; ++u) v = mx ? fmax(v, w[u]) : v + w[u];
  }
  for (; t < P.tile_count; t += 16) {
    const double w = row[(long)t * NS];
    v = mx ? fmax(v, w) : v + w;
  }
  red[g][s] = v;
  __syncthreads();
  if (threadIdx.x < NS) {
    double u = red[0][s];
    for (int k = 1; k < 16; ++k) u = mx ? fmax(u, red[k][s]) : u + red[k][s];
    sums[(long)b * NS + s] = u;
    fin[s] = u;
  }
  __syncthreads();
  if (do_decide && threadIdx.x == 0) decide_pair(dec, b, fin, P, pre);
}

// Copies the current iterate from src to dst for pairs still active.
__global__ __launch_bounds__(BLOCK) void copy_active_kernel(Planes dst, Planes src, const PairInfo* pairs,
                                                            const Tile* tiles, int ntiles, int tile_rows,
                                                            const int32_t* active) {
  const int lx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    if (!active[tl.pair]) continue;
    const PairInfo P = pairs[tl.pair];
    for (int ly = wv; ly < tile_rows; ly += 4) {
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= P.nx || gy >= P.ny) continue;
      const long o = P.off + (long)gy * P.pitch + gx;
      dst.Mx[o] = src.Mx[o];
      dst.My[o] = src.My[o];
      dst.a[o] = src.a[o];
      if (dst.r && src.r) dst.r[o] = src.r[o];
      if (dst.x0 && src.x0) dst.x0[o] = src.x0[o];
      if (dst.x1 && src.x1) dst.x1[o] = src.x1[o];
    }
  }
}

// Zeroes the state of the pairs whose flag is set (a cold start for pairs
// whose warm state was rejected).
__global__ __launch_bounds__(BLOCK) void zero_pairs_kernel(Planes st, const PairInfo* pairs, const Tile* tiles,
                                                           int ntiles, int tile_rows, const int32_t* mask) {
  const int lx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    if (!mask[tl.pair]) continue;
    const PairInfo P = pairs[tl.pair];
    for (int ly = wv; ly < tile_rows; ly += 4) {
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= P.nx || gy >= P.ny) continue;
      const long o = P.off + (long)gy * P.pitch + gx;
      st.Mx[o] = 0.f;
      st.My[o] = 0.f;
      st.a[o] = 0.f;
      if (st.r) st.r[o] = 0.f;
      if (st.x0) st.x0[o] = 0.f;
      if (st.x1) st.x1[o] = 0.f;
    }
  }
}

// Dual value of the scaled multiplier a/s for the PROX modes: the infimum
// over x >= 0 of the Lagrangian's x terms has the closed-form minimisers
// max(p0 + rho a, 0) and max(p1 - rho a, 0).
__global__ __launch_bounds__(BLOCK) void dual_kernel(DualArgs A) {
  const int lx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
    const Tile tl = A.tiles[t];
    const PairInfo P = A.pairs[tl.pair];
    const double is = A.inv_s[tl.pair];
    const double rho = A.rho;
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    for (int ly = wv; ly < A.tile_rows; ly += 4) {
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= P.nx || gy >= P.ny) continue;
      const long o = P.off + (long)gy * P.pitch + gx;
      const double ah = (double)A.a[o] * is;
      double v = 0.0;
      const double p1 = A.x_dst[o];
      const double x1s = fmax(p1 - rho * ah, 0.0);
      v += (x1s - p1) * (x1s - p1) / (2.0 * rho) + ah * x1s;
      if (A.mode == 1) {
        const double p0 = A.x_src[o];
        const double x0s = fmax(p0 + rho * ah, 0.0);
        v += (x0s - p0) * (x0s - p0) / (2.0 * rho) - ah * x0s;
      } else {
        v -= ah * (double)A.x_src[o];
      }
      if (A.resid == R_P2) v -= ah * ah / (4.0 * (double)A.mu);
      acc[0] += v;
    }
    block_reduce_store(acc, 0u, A.partial + (long)t * NS);
  }
}



hipError_t launch_iter(int mode, int resid, int bc, int ty, int grid, const IterArgs& a, hipStream_t s) {
  switch (mode) {
    case 0: return launch_iter_mode0(resid, bc, ty, grid, a, s);
    case 1: return launch_iter_mode1(resid, bc, ty, grid, a, s);
    case 2: return launch_iter_mode2(resid, bc, ty, grid, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t iter_chk_occupancy(int mode, int resid, int bc, int ty, int* n) {
  switch (mode) {
    case 0: return iter_chk_occupancy_mode0(resid, bc, ty, n);
    case 1: return iter_chk_occupancy_mode1(resid, bc, ty, n);
    case 2: return iter_chk_occupancy_mode2(resid, bc, ty, n);
  }
  return hipErrorInvalidValue;
}

hipError_t iter_occupancy(int mode, int resid, int bc, int ty, int* n) {
  switch (mode) {
    case 0: return iter_occupancy_mode0(resid, bc, ty, n);
    case 1: return iter_occupancy_mode1(resid, bc, ty, n);
    case 2: return iter_occupancy_mode2(resid, bc, ty, n);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iter_chk(int mode, int resid, int bc, int ty, int grid, const IterArgs& a, hipStream_t s) {
  switch (mode) {
    case 0: return launch_iter_chk_mode0(resid, bc, ty, grid, a, s);
    case 1: return launch_iter_chk_mode1(resid, bc, ty, grid, a, s);
    case 2: return launch_iter_chk_mode2(resid, bc, ty, grid, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_check(int mode, int resid, int bc, int grid, const CheckArgs& a, hipStream_t s) {
  switch (mode) {
    case 0: return launch_check_mode0(resid, bc, grid, a, s);
    case 1: return launch_check_mode1(resid, bc, grid, a, s);
    case 2: return launch_check_mode2(resid, bc, grid, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_setup(int grid, const SetupArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(setup_kernel, dim3(grid), dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pair_reduce(const PairInfo* pairs, int B, const double* partial, uint32_t max_mask,
                              double* sums, hipStream_t s) {
  DecideArgs none{};
  hipLaunchKernelGGL(pair_reduce_kernel, dim3(B), dim3(BLOCK), 0, s, pairs, partial, max_mask, sums, none, 0);
  return hipGetLastError();
}

hipError_t launch_reduce_decide(const DecideArgs& a, const double* partial, hipStream_t s) {
  hipLaunchKernelGGL(pair_reduce_kernel, dim3(a.B), dim3(BLOCK), 0, s, a.pairs, partial, kMaxSlotsCheck,
                     a.sums, a, 1);
  return hipGetLastError();
}

hipError_t launch_copy_active(const Planes& dst, const Planes& src, const PairInfo* pairs, const Tile* tiles,
                              int ntiles, int tile_rows, const int32_t* active, int grid, hipStream_t s) {
  hipLaunchKernelGGL(copy_active_kernel, dim3(grid), dim3(BLOCK), 0, s, dst, src, pairs, tiles, ntiles,
                     tile_rows, active);
  return hipGetLastError();
}

hipError_t launch_zero_pairs(const Planes& st, const PairInfo* pairs, const Tile* tiles, int ntiles, int tile_rows,
                             const int32_t* mask, int grid, hipStream_t s) {
  hipLaunchKernelGGL(zero_pairs_kernel, dim3(grid), dim3(BLOCK), 0, s, st, pairs, tiles, ntiles, tile_rows, mask);
  return hipGetLastError();
}

hipError_t launch_dual(int grid, const DualArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dual_kernel, dim3(grid), dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

}  // namespace uot
