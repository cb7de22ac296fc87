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

// ---------------------------------------------------------------------------
// RPCA+UOT-DF (Sec. IV-B, Algorithm 3).  Frames are packed back to back; e
// indexes pixel i of frame t as t * npx + i.  wz_t = 1 for t < T - 1 and
// ww_t = 1 for t > 0 (0-based); pair t couples frames t and t + 1.

// Lines 5-9 of Algorithm 3 and the prox centres, per pixel and frame:
//   k = (x - l + a) + wz (z_t + b_t) + ww (w_t + c_t),  sig = 1 + wz + ww
//   s = max(k / sig - lam / (rho sig), 0)
//   l = max((Tn - D + x - s + a) / 2, 0)
//   x = (phi y + rho (s + l - a)) / (phi^2 + rho)
//   p0_t = s_t - b_t,  p1_{t-1} = s_t - c_{t-1}; z, w saved for the residual
__global__ __launch_bounds__(RB) void rp_sx_kernel(RpArgs A) {
  double dx2 = 0.0;
  const long npx = A.npx, n = npx * A.T;
  const float rho = A.rho, lam = A.lam;
  for (long e = blockIdx.x * (long)RB + threadIdx.x; e < n; e += (long)gridDim.x * RB) {
    const int t = (int)(e / npx);
    const long i = e - (long)t * npx;
    const float x = A.X[e], l = A.L[e], a = A.A[e];
    float k = x - l + a, sig = 1.f;
    const long pe = (long)t * npx + i, pw = (long)(t - 1) * npx + i;
    if (t < A.T - 1) {
      k += A.Z[pe] + A.B[pe];
      sig += 1.f;
    }
    if (t > 0) {
      k += A.W[pw] + A.C[pw];
      sig += 1.f;
    }
    const float s = fmaxf(k / sig - lam / (rho * sig), 0.f);
    const float ln = fmaxf(0.5f * (A.Tn[e] - A.D[e] + x - s + a), 0.f);
    const float ph = A.phi ? A.phi[e] : 1.f;
    const float xn = (ph * A.y[e] + rho * (s + ln - a)) / (ph * ph + rho);
    A.S[e] = s;
    A.L[e] = ln;
    A.X[e] = xn;
    if (A.record) {
      const float d = xn - x;
      dx2 += (double)d * d;
    }
    if (t < A.T - 1) {
      A.P0[pe] = s - A.B[pe];
      A.zo[pe] = A.Z[pe];
    }
    if (t > 0) {
      A.P1[pw] = s - A.C[pw];
      A.wo[pw] = A.W[pw];
    }
  }
  if (A.record) block_sum(dx2, A.partial + RP_SLOTS * blockIdx.x + 1);
}

// Gram matrix of M = L + D (columns = frames): per-block partial sums of
// G[p][q] = sum_i M[p][i] M[q][i] for p <= q (packed upper triangle), FP64.
// A block stages 64 pixels of every frame in LDS; thread (bp, bq) of the
// 16 x 16 grid of threads owns the 4 x 4 block of entries p in 4bp..4bp+3,
// q in 4bq..4bq+3 (blocks below the diagonal idle), so 8 LDS reads feed 16
// FP64 multiply-adds.
__global__ __launch_bounds__(RB) void rp_gram_kernel(RpArgs A, double* gpart) {
  constexpr int CH = 64;
  static_assert(RP_MAX_FRAMES == 64 && RB == 256, "16 x 16 threads of 4 x 4 entries");
  __shared__ float sm[RP_MAX_FRAMES][CH + 1];
  const int T = A.T, np = T * (T + 1) / 2;
  const long npx = A.npx;
  const int bp = threadIdx.x >> 4, bq = threadIdx.x & 15;
  const int p0 = 4 * bp, q0 = 4 * bq;
  const bool live = p0 < T && q0 < T && p0 <= q0 + 3;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (long c = blockIdx.x; c * CH < npx; c += gridDim.x) {
    __syncthreads();
    for (int e = threadIdx.x; e < RP_MAX_FRAMES * CH; e += RB) {
      const int t = e / CH, i = e - t * CH;
      const long g = c * CH + i;
      sm[t][i] = (t < T && g < npx) ? A.L[(long)t * npx + g] + A.D[(long)t * npx + g] : 0.f;
    }
    __syncthreads();
    if (live) {
      for (int i = 0; i < CH; ++i) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = (double)sm[p0 + u][i];
          b[u] = (double)sm[q0 + u][i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
      }
    }
  }
  if (live) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + u, q = q0 + v;
        if (p < T && q < T && p <= q) gpart[(long)blockIdx.x * np + (p * T - p * (p - 1) / 2 + (q - p))] = acc[u][v];
      }
  }
}

// G[j] = sum over blocks of gpart[b][j], in block order.
__global__ __launch_bounds__(RB) void rp_gram_reduce_kernel(const double* gpart, int blocks, int np, double* G) {
  for (int j = blockIdx.x * RB + threadIdx.x; j < np; j += gridDim.x * RB) {
    double v = 0.0;
#pragma unroll 8
    for (int b = 0; b < blocks; ++b) v += gpart[(long)b * np + j];
    G[j] = v;
  }
}

// Singular-value threshold of M from its Gram matrix G = M^T M = V Lam V^T:
// SVT_thr(M) = M V diag(f) V^T with f_j = max(1 - thr / sigma_j, 0),
// sigma_j = sqrt(lam_j).  The eigenvectors come from the cyclic Jacobi
// method with the parallel round-robin ordering (every round rotates T/2
// disjoint pairs at once), started from the previous call's eigenvectors V:
// the iteration moves little from one ADMM step to the next, so V^T G V is
// nearly diagonal and one or two sweeps finish it (often none).  One
// workgroup; G is staged into LDS, A and V live there in FP64.  Writes Wm = V diag(f) V^T (FP32), the new V, and the
// number of sweeps.
__global__ __launch_bounds__(RB) void rp_eig_kernel(const double* G, int T, double thr, double* Vg, float* Wm,
                                                     int* sweeps) {
  constexpr int MT = RP_MAX_FRAMES, LD = MT + 1;
  __shared__ double Am[MT * LD];
  __shared__ double Vm[MT * LD];
  __shared__ double cs[MT / 2][2];
  __shared__ int pq[MT / 2][2];
  __shared__ double fj[MT];
  __shared__ double red[2][RB / 64];
  const int tid = threadIdx.x;
  const int TT = T * T;
  auto g = [&](int i, int j) {
    const int p = i < j ? i : j, q = i < j ? j : i;
    return G[p * T - p * (p - 1) / 2 + (q - p)];
  };
  for (int e = tid; e < TT; e += RB) {
    const int i = e / T, j = e % T;
    Vm[i * LD + j] = Vg[e];
    Am[i * LD + j] = g(i, j);
  }
  __syncthreads();
  // A = V^T G V, in two products through registers
  constexpr int PER = (MT * MT + RB - 1) / RB;
  double tmp[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + RB * m;
    tmp[m] = 0.0;
    if (e < TT) {
      const int i = e / T, j = e % T;
      double v = 0.0;
      for (int k = 0; k < T; ++k) v += Am[i * LD + k] * Vm[k * LD + j];
      tmp[m] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + RB * m;
    if (e < TT) Am[(e / T) * LD + e % T] = tmp[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + RB * m;
    if (e < TT) {
      const int i = e / T, j = e % T;
      double v = 0.0;
      for (int k = 0; k < T; ++k) v += Vm[k * LD + i] * Am[k * LD + j];
      tmp[m] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + RB * m;
    if (e < TT) Am[(e / T) * LD + e % T] = tmp[m];
  }
  __syncthreads();

  const int Tp = T + (T & 1);  // even; index T is a dummy when T is odd
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < TT; e += RB) {
      const int i = e / T, j = e % T;
      const double v = Am[i * LD + j];
      tot += v * v;
      if (i != j) off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      tot += __shfl_down(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = tot;
    }
    __syncthreads();
    off = tot = 0.0;
    for (int w = 0; w < RB / 64; ++w) {
      off += red[0][w];
      tot += red[1][w];
    }
    __syncthreads();
    // off-diagonal norm below 1e-10 of the whole: eigenvalues to about 1e-20 relative,
    // eigenvectors to about 1e-10, far below the FP32 result
    if (!(off > 1e-20 * tot)) break;  // uniform: every thread holds the same sums
    for (int r = 0; r < Tp - 1; ++r) {
      if (tid < Tp / 2) {
        // round-robin pairing: player Tp - 1 fixed, the others rotate
        int p, q;
        if (tid == 0) {
          p = r;
          q = Tp - 1;
        } else {
          p = (r + tid) % (Tp - 1);
          q = (r - tid + (Tp - 1)) % (Tp - 1);
        }
        if (p > q) {
          const int u = p;
          p = q;
          q = u;
        }
        double c = 1.0, s = 0.0;
        if (q < T) {
          const double apq = Am[p * LD + q];
          if (apq != 0.0) {
            const double tau = (Am[q * LD + q] - Am[p * LD + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[tid][0] = c;
        cs[tid][1] = s;
        pq[tid][0] = p;
        pq[tid][1] = q;
      }
      __syncthreads();
      for (int e = tid; e < (Tp / 2) * T; e += RB) {  // rows p, q of A
        const int k = e / T, j = e % T, p = pq[k][0], q = pq[k][1];
        if (q >= T) continue;
        const double c = cs[k][0], s = cs[k][1];
        const double a = Am[p * LD + j], b = Am[q * LD + j];
        Am[p * LD + j] = c * a - s * b;
        Am[q * LD + j] = s * a + c * b;
      }
      __syncthreads();
      for (int e = tid; e < (Tp / 2) * T; e += RB) {  // columns p, q of A and V
        const int k = e / T, i = e % T, p = pq[k][0], q = pq[k][1];
        if (q >= T) continue;
        const double c = cs[k][0], s = cs[k][1];
        const double a = Am[i * LD + p], b = Am[i * LD + q];
        Am[i * LD + p] = c * a - s * b;
        Am[i * LD + q] = s * a + c * b;
        const double va = Vm[i * LD + p], vb = Vm[i * LD + q];
        Vm[i * LD + p] = c * va - s * vb;
        Vm[i * LD + q] = s * va + c * vb;
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < T; j += RB) {
    const double sig = sqrt(fmax(Am[j * LD + j], 0.0));
    fj[j] = sig > thr ? 1.0 - thr / sig : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < TT; e += RB) {
    const int i = e / T, j = e % T;
    double v = 0.0;
    for (int k = 0; k < T; ++k) v += Vm[i * LD + k] * fj[k] * Vm[j * LD + k];
    Wm[e] = (float)v;
    Vg[e] = Vm[i * LD + j];
  }
  if (tid == 0) *sweeps = sweep;
}

// Tn = (L + D) Wm per pixel (T x T product from LDS), then D += L - Tn.  Wm
// rows are padded to a multiple of 4 with zeros so that every LDS read
// fetches 4 outputs' weights at once (a broadcast: all lanes read one row).
__global__ __launch_bounds__(RB) void rp_svt_apply_kernel(RpArgs A) {
  constexpr int MP = RP_MAX_FRAMES;
  __shared__ __attribute__((aligned(16))) float w[RP_MAX_FRAMES * MP];
  const int T = A.T, TP = (T + 3) & ~3;
  for (int e = threadIdx.x; e < T * TP; e += RB) {
    const int s_ = e / TP, t = e - s_ * TP;
    w[s_ * MP + t] = t < T ? A.Wm[s_ * T + t] : 0.f;
  }
  __syncthreads();
  double lt2 = 0.0, dt2 = 0.0;
  const long npx = A.npx;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    float m[RP_MAX_FRAMES];
#pragma unroll
    for (int s_ = 0; s_ < RP_MAX_FRAMES; ++s_)
      m[s_] = s_ < T ? A.L[(long)s_ * npx + i] + A.D[(long)s_ * npx + i] : 0.f;
    for (int t4 = 0; t4 < TP; t4 += 4) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int s_ = 0; s_ < RP_MAX_FRAMES; ++s_) {
        if (s_ < T) {
          const float4 wv = *reinterpret_cast<const float4*>(&w[s_ * MP + t4]);
          acc.x += m[s_] * wv.x;
          acc.y += m[s_] * wv.y;
          acc.z += m[s_] * wv.z;
          acc.w += m[s_] * wv.w;
        }
      }
      const float av[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t4 + u;
        if (t >= T) break;
        const long e = (long)t * npx + i;
        const float l = A.L[e], told = A.Tn[e];
        A.Tn[e] = av[u];
        A.D[e] = A.D[e] + (l - av[u]);
        if (A.record) {
          const float d1 = l - av[u], d2 = av[u] - told;
          lt2 += (double)d1 * d1;
          dt2 += (double)d2 * d2;
        }
      }
    }
  }
  if (A.record) {
    block_sum(lt2, A.partial + RP_SLOTS * blockIdx.x + 2);
    block_sum(dt2, A.partial + RP_SLOTS * blockIdx.x + 3);
  }
}

// Lines 12-15: A += X - S - L, b_t += z_t - s_t, c_t += w_{t+1} - s_{t+1}.
__global__ __launch_bounds__(RB) void rp_dual_kernel(RpArgs A) {
  double rp2 = 0.0, dz2 = 0.0;
  const long npx = A.npx, n = npx * A.T;
  for (long e = blockIdx.x * (long)RB + threadIdx.x; e < n; e += (long)gridDim.x * RB) {
    const int t = (int)(e / npx);
    const long i = e - (long)t * npx;
    const float x = A.X[e], s = A.S[e], l = A.L[e];
    A.A[e] = A.A[e] + x - s - l;
    if (A.record) {
      const float u = x - s - l;
      rp2 += (double)u * u;
    }
    if (t < A.T - 1) {
      const long pe = (long)t * npx + i;
      const float z = A.Z[pe];
      A.B[pe] = A.B[pe] + (z - s);
      if (A.record) {
        const float u = z - s, v = z - A.zo[pe];
        rp2 += (double)u * u;
        dz2 += (double)v * v;
      }
    }
    if (t > 0) {
      const long pw = (long)(t - 1) * npx + i;
      const float w = A.W[pw];
      A.C[pw] = A.C[pw] + (w - s);
      if (A.record) {
        const float u = w - s, v = w - A.wo[pw];
        rp2 += (double)u * u;
        dz2 += (double)v * v;
      }
    }
  }
  if (A.record) {
    block_sum(rp2, A.partial + RP_SLOTS * blockIdx.x + 0);
    block_sum(dz2, A.partial + RP_SLOTS * blockIdx.x + 4);
  }
}

__global__ __launch_bounds__(RB) void rp_reduce_kernel(const double* partial, int nblocks, double* out) {
  for (int j = 0; j < RP_SLOTS; ++j) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RB) v += partial[RP_SLOTS * b + j];
    block_sum(v, out + j);
  }
}

__global__ __launch_bounds__(RB) void rp_validate_kernel(long n, const float* y, const float* phi, double* partial) {
  double bad = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
    const float v = y[i], f = phi ? phi[i] : 1.f;
    bad += (isfinite(v) && isfinite(f)) ? 0.0 : 1.0;
  }
  block_sum(bad, partial + RP_SLOTS * blockIdx.x);
  if (threadIdx.x == 0)
    for (int j = 1; j < RP_SLOTS; ++j) partial[RP_SLOTS * blockIdx.x + j] = 0.0;
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

hipError_t launch_rp_sx(const RpArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_sx_kernel, dim3(blocks), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_gram(const RpArgs& a, int blocks, double* gpart, hipStream_t s) {
  hipLaunchKernelGGL(rp_gram_kernel, dim3(blocks), dim3(RB), 0, s, a, gpart);
  return hipGetLastError();
}

hipError_t launch_rp_gram_reduce(const double* gpart, int blocks, int T, double* G, hipStream_t s) {
  const int np = T * (T + 1) / 2;
  hipLaunchKernelGGL(rp_gram_reduce_kernel, dim3((np + RB - 1) / RB), dim3(RB), 0, s, gpart, blocks, np, G);
  return hipGetLastError();
}

hipError_t launch_rp_eig(const double* G, int T, double thr, double* V, float* Wm, int* sweeps, hipStream_t s) {
  hipLaunchKernelGGL(rp_eig_kernel, dim3(1), dim3(RB), 0, s, G, T, thr, V, Wm, sweeps);
  return hipGetLastError();
}

hipError_t launch_rp_svt_apply(const RpArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_svt_apply_kernel, dim3(blocks), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_dual(const RpArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_dual_kernel, dim3(blocks), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_reduce(const double* partial, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(rp_reduce_kernel, dim3(1), dim3(RB), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_rp_validate(long n, const float* y, const float* phi, double* partial, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_validate_kernel, dim3(blocks), dim3(RB), 0, s, n, y, phi, partial);
  return hipGetLastError();
}

}  // namespace uot
