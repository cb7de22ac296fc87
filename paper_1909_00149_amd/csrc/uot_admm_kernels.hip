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
// indexes pixel i of frame t as t * npx + i.  Pair t couples frames t and
// t + 1; its planes (b, c, prox centres, z, w) are packed the same way.
// The frame-wise kernels run on a (pixel blocks, frames) grid, so the frame
// comes from blockIdx.y and no index is divided.  Residual partials go to
// partial[slot * pstride + block] (one block id per launch block).

// The s-, L- and x-steps and the prox centres, per pixel of frame t:
//   k = (x - l + a) + wz (z_t + b_t) + ww (w_{t-1} + c_{t-1}),  sig = 1 + wz + ww
//   s = max(k / sig - lam / (rho sig), 0)
//   l = max((Tn - D + x - s + a) / 2, 0)
//   x = (phi y + rho (s + l - a)) / (phi^2 + rho)
//   p0_t = s_t - b_t,  p1_{t-1} = s_t - c_{t-1}
// with wz = 1 unless t is the last frame and ww = 1 unless t is the first.
// z and w are saved (zo, wo) only where the residual is recorded.
__global__ __launch_bounds__(RB) void rp_sx_kernel(RpArgs A) {
  double dx2 = 0.0;
  const int t = blockIdx.y;
  const long npx = A.npx, fe = (long)t * npx, fw = (long)(t - 1) * npx;
  const bool hz = t < A.T - 1, hw = t > 0;
  const float rho = A.rho, lam = A.lam;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    const long e = fe + i;
    const float x = A.X[e], l = A.L[e], a = A.A[e];
    float k = x - l + a, sig = 1.f, z = 0.f, w = 0.f, bz = 0.f, cw = 0.f;
    if (hz) {
      z = A.Z[e];
      bz = A.B[e];
      k += z + bz;
      sig += 1.f;
    }
    if (hw) {
      w = A.W[fw + i];
      cw = A.C[fw + i];
      k += w + cw;
      sig += 1.f;
    }
    const float s = fmaxf(k / sig - lam / (rho * sig), 0.f);
    const float ln = fmaxf(0.5f * (A.Tn[e] - A.D[e] + x - s + a), 0.f);
    const float ph = A.phi ? A.phi[e] : 1.f;
    const float xn = (ph * A.y[e] + rho * (s + ln - a)) / (ph * ph + rho);
    A.S[e] = s;
    A.L[e] = ln;
    A.X[e] = xn;
    if (hz) A.P0[e] = s - bz;
    if (hw) A.P1[fw + i] = s - cw;
    if (A.record) {
      const float d = xn - x;
      dx2 += (double)d * d;
      if (hz) A.zo[e] = z;
      if (hw) A.wo[fw + i] = w;
    }
  }
  if (A.record) block_sum(dx2, A.partial + 1 * A.pstride + blockIdx.y * gridDim.x + blockIdx.x);
}

// Gram matrix of M = L + D (columns = frames): per-block partial sums of
// G[p][q] = sum_i M[p][i] M[q][i] for p <= q (packed upper triangle), FP64.
// A block stages 64 pixels of every frame in LDS (converted to FP64 once);
// its threads own the 4 x 4 tiles on and above the diagonal (136 tiles for
// T = 64, numbered row by row), so 8 LDS reads of two doubles feed 32 FP64
// multiply-adds.  The next chunk's loads are in flight while a chunk is
// multiplied.
__global__ __launch_bounds__(RB) void rp_gram_kernel(RpArgs A, double* gpart) {
  constexpr int CH = 64, LDC = CH + 2, PER = RP_MAX_FRAMES * CH / RB;
  static_assert(RP_MAX_FRAMES == 64 && RB == 256, "64 frames x 64 pixels staged by 256 threads");
  __shared__ __attribute__((aligned(16))) double sm[RP_MAX_FRAMES * LDC];
  const int T = A.T, nb = (T + 3) >> 2, np = T * (T + 1) / 2;
  const long npx = A.npx;
  int bp = 0, rem = threadIdx.x;
  while (bp < nb && rem >= nb - bp) {
    rem -= nb - bp;
    ++bp;
  }
  const bool live = bp < nb;
  const int p0 = 4 * bp, q0 = 4 * (bp + rem);
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  float pf[PER];
  auto fetch = [&](long c) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = threadIdx.x + RB * m, t = e >> 6, i = e & (CH - 1);
      const long g = c * CH + i;
      pf[m] = (t < T && g < npx) ? A.L[(long)t * npx + g] + A.D[(long)t * npx + g] : 0.f;
    }
  };
  long c = blockIdx.x;
  if (c * CH < npx) fetch(c);
  for (; c * CH < npx; c += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = threadIdx.x + RB * m;
      sm[(e >> 6) * LDC + (e & (CH - 1))] = (double)pf[m];
    }
    __syncthreads();
    if ((c + gridDim.x) * CH < npx) fetch(c + gridDim.x);
    if (live) {
      for (int i = 0; i < CH; i += 2) {
        double2 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = *reinterpret_cast<const double2*>(&sm[(p0 + u) * LDC + i]);
          b[u] = *reinterpret_cast<const double2*>(&sm[(q0 + u) * LDC + i]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u].y, b[v].y, fma(a[u].x, b[v].x, acc[u][v]));
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

// G[j] = sum over blocks of gpart[b][j]: a block adds 64 entries, its four
// waves take every fourth partial, and the four sums are combined in a
// fixed order (the result does not depend on timing).
__global__ __launch_bounds__(RB) void rp_gram_reduce_kernel(const double* gpart, int blocks, int np, double* G) {
  __shared__ double red[RB / 64][64];
  const int jl = threadIdx.x & 63, q = threadIdx.x >> 6, j = blockIdx.x * 64 + jl;
  double v = 0.0;
  if (j < np)
    for (int b = q; b < blocks; b += RB / 64) v += gpart[(long)b * np + j];
  red[q][jl] = v;
  __syncthreads();
  if (q == 0 && j < np) G[j] = (red[0][jl] + red[1][jl]) + (red[2][jl] + red[3][jl]);
}

// Singular-value threshold of M from its Gram matrix G = M^T M = V Lam V^T:
// SVT_thr(M) = M V diag(f) V^T with f_j = max(1 - thr / sigma_j, 0),
// sigma_j = sqrt(lam_j).  The eigenvectors come from the cyclic Jacobi
// method with the parallel round-robin ordering (every round rotates 32
// disjoint pairs at once), started from the previous call's eigenvectors V:
// the iteration moves little from one ADMM step to the next, so V^T G V is
// nearly diagonal and one sweep usually finishes it.  One workgroup; the
// matrix is padded to 64 x 64 (zero rows and columns of A, identity in V,
// which no rotation touches since their off-diagonal entries stay zero), so
// all index arithmetic is shifts.  A and V live in LDS in FP64.  A round:
// 32 threads form the rotations; then every 2 x 2 block (pair k1 rows, pair
// k2 columns) of A becomes R_k1^T A R_k2 and the two columns of V of every
// pair rotate, each block and column pair owned by one thread (no
// conflicting writes), diagonal blocks taking the exact diagonalisation.
// The products V^T G V and V diag(f) V^T keep a 4 x 4 block per thread.
// Writes Wm = V diag(f) V^T (FP32, T x T), the new V, and the number of
// sweeps.
__global__ __launch_bounds__(RB) void rp_eig_kernel(const double* G, int T, double thr, double* Vg, float* Wm,
                                                     int* sweeps) {
  constexpr int N = RP_MAX_FRAMES, LD = N + 1, NP = N / 2;
  static_assert(N == 64 && RB == 256, "64 x 64 matrices, 16 x 16 threads of 4 x 4 blocks");
  __shared__ double Am[N * LD];
  __shared__ double Vm[N * LD];
  __shared__ double rot[NP][3];  // c, s, t = s / c
  __shared__ int pq[NP][2];
  __shared__ double fj[N];
  __shared__ double red[2][RB / 64];
  const int tid = threadIdx.x;
  for (int e = tid; e < N * N; e += RB) {
    const int i = e >> 6, j = e & (N - 1);
    double gv = 0.0, vv = i == j ? 1.0 : 0.0;
    if (i < T && j < T) {
      const int p = i < j ? i : j, q = i < j ? j : i;
      gv = G[p * T - p * (p - 1) / 2 + (q - p)];
      vv = Vg[i * T + j];
    }
    Am[i * LD + j] = gv;
    Vm[i * LD + j] = vv;
  }
  __syncthreads();
  const int bi = tid >> 4, bj = tid & 15;
  double acc[4][4];
  // Am <- G V
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k = 0; k < N; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Am[(4 * bi + u) * LD + k];
      b[u] = Vm[k * LD + 4 * bj + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Am[(4 * bi + u) * LD + 4 * bj + v] = acc[u][v];
  __syncthreads();
  // Am <- V^T Am
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k = 0; k < N; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Vm[k * LD + 4 * bi + u];
      b[u] = Am[k * LD + 4 * bj + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Am[(4 * bi + u) * LD + 4 * bj + v] = acc[u][v];
  __syncthreads();

  const int k2 = tid & (NP - 1), r1 = tid >> 5;  // this thread's column pair; first row pair / V row
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < N * N; e += RB) {
      const int i = e >> 6, j = e & (N - 1);
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
    // off-diagonal norm below 1e-10 of the whole: eigenvalues to about 1e-20
    // relative, eigenvectors to about 1e-10, far below the FP32 result
    if (!(off > 1e-20 * tot)) break;  // uniform: every thread holds the same sums
    for (int r = 0; r < N - 1; ++r) {
      if (tid < NP) {
        // round-robin pairing: player N - 1 fixed, the others rotate
        int p = tid == 0 ? r : (r + tid) % (N - 1);
        int q = tid == 0 ? N - 1 : (r - tid + (N - 1)) % (N - 1);
        if (p > q) {
          const int u = p;
          p = q;
          q = u;
        }
        double c = 1.0, s = 0.0, t = 0.0;
        const double apq = Am[p * LD + q];
        if (apq != 0.0) {
          const double tau = (Am[q * LD + q] - Am[p * LD + p]) / (2.0 * apq);
          t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        rot[tid][0] = c;
        rot[tid][1] = s;
        rot[tid][2] = t;
        pq[tid][0] = p;
        pq[tid][1] = q;
      }
      __syncthreads();
      const int p2 = pq[k2][0], q2 = pq[k2][1];
      const double c2 = rot[k2][0], s2 = rot[k2][1];
#pragma unroll
      for (int m = 0; m < NP / 8; ++m) {
        const int k1 = r1 + 8 * m;
        const int p1 = pq[k1][0], q1 = pq[k1][1];
        const double a = Am[p1 * LD + p2], b = Am[p1 * LD + q2], cc = Am[q1 * LD + p2], d = Am[q1 * LD + q2];
        if (k1 == k2) {
          const double t1 = rot[k1][2];
          Am[p1 * LD + p1] = a - t1 * b;
          Am[q1 * LD + q1] = d + t1 * b;
          Am[p1 * LD + q1] = 0.0;
          Am[q1 * LD + p1] = 0.0;
        } else {
          const double c1 = rot[k1][0], s1 = rot[k1][1];
          const double rpp = c1 * a - s1 * cc, rpq = c1 * b - s1 * d;
          const double rqp = s1 * a + c1 * cc, rqq = s1 * b + c1 * d;
          Am[p1 * LD + p2] = c2 * rpp - s2 * rpq;
          Am[p1 * LD + q2] = s2 * rpp + c2 * rpq;
          Am[q1 * LD + p2] = c2 * rqp - s2 * rqq;
          Am[q1 * LD + q2] = s2 * rqp + c2 * rqq;
        }
      }
#pragma unroll
      for (int m = 0; m < N / 8; ++m) {
        const int i = r1 + 8 * m;
        const double va = Vm[i * LD + p2], vb = Vm[i * LD + q2];
        Vm[i * LD + p2] = c2 * va - s2 * vb;
        Vm[i * LD + q2] = s2 * va + c2 * vb;
      }
      __syncthreads();
    }
  }
  if (tid < N) {
    const double sig = sqrt(fmax(Am[tid * LD + tid], 0.0));
    fj[tid] = sig > thr ? 1.0 - thr / sig : 0.0;
  }
  __syncthreads();
  // Wm = V diag(f) V^T
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k = 0; k < N; ++k) {
    const double f = fj[k];
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Vm[(4 * bi + u) * LD + k] * f;
      b[u] = Vm[(4 * bj + u) * LD + k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * bi + u, j = 4 * bj + v;
      if (i < T && j < T) {
        Wm[i * T + j] = (float)acc[u][v];
        Vg[i * T + j] = Vm[i * LD + j];
      }
    }
  if (tid == 0) *sweeps = sweep;
}

// Tn = (L + D) Wm per pixel, then D <- (L + D) - Tn (= D + L - Tn).  A
// block takes 64 pixels at a time; its wave g computes the outputs of frames
// 16g .. 16g + 15 from float4 rows of Wm in LDS (every lane reads the same
// address) while it streams L + D of all frames; the four waves read the
// same pixels, so HBM sees them once.
__global__ __launch_bounds__(RB) void rp_svt_apply_kernel(RpArgs A) {
  constexpr int MP = RP_MAX_FRAMES;
  static_assert(RB == 4 * 64 && MP == 64, "four waves of 16 output frames");
  __shared__ __attribute__((aligned(16))) float w[MP * MP];
  const int T = A.T;
  for (int e = threadIdx.x; e < MP * MP; e += RB) {
    const int s_ = e >> 6, t = e & (MP - 1);
    w[e] = (s_ < T && t < T) ? A.Wm[s_ * T + t] : 0.f;
  }
  __syncthreads();
  double lt2 = 0.0, dt2 = 0.0;
  const long npx = A.npx;
  const int t0 = 16 * (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t0 < T) {
    for (long c = blockIdx.x; c * 64 < npx; c += gridDim.x) {
      const long i = c * 64 + lane;
      const bool valid = i < npx;
      float acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.f;
#pragma unroll 4
      for (int s_ = 0; s_ < T; ++s_) {
        const float m = valid ? A.L[(long)s_ * npx + i] + A.D[(long)s_ * npx + i] : 0.f;
        const float4* wr = reinterpret_cast<const float4*>(&w[s_ * MP + t0]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 wv = wr[j];
          acc[4 * j + 0] += m * wv.x;
          acc[4 * j + 1] += m * wv.y;
          acc[4 * j + 2] += m * wv.z;
          acc[4 * j + 3] += m * wv.w;
        }
      }
      if (!valid) continue;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int t = t0 + u;
        if (t < T) {
          const long e = (long)t * npx + i;
          const float l = A.L[e], m = l + A.D[e];
          if (A.record) {
            const float d1 = l - acc[u], d2 = acc[u] - A.Tn[e];
            lt2 += (double)d1 * d1;
            dt2 += (double)d2 * d2;
          }
          A.Tn[e] = acc[u];
          A.D[e] = m - acc[u];
        }
      }
    }
  }
  if (A.record) {
    block_sum(lt2, A.partial + 2 * A.pstride + blockIdx.x);
    block_sum(dt2, A.partial + 3 * A.pstride + blockIdx.x);
  }
}

// The multiplier steps, per pixel of frame t: A += X - S - L,
// b_t += z_t - s_t (t below the last frame), c_{t-1} += w_{t-1} - s_t
// (t above the first).
__global__ __launch_bounds__(RB) void rp_dual_kernel(RpArgs A) {
  double rp2 = 0.0, dz2 = 0.0;
  const int t = blockIdx.y;
  const long npx = A.npx, fe = (long)t * npx, fw = (long)(t - 1) * npx;
  const bool hz = t < A.T - 1, hw = t > 0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    const long e = fe + i;
    const float x = A.X[e], s = A.S[e], l = A.L[e];
    const float u0 = x - s - l;
    A.A[e] = A.A[e] + u0;
    if (A.record) rp2 += (double)u0 * u0;
    if (hz) {
      const float z = A.Z[e];
      A.B[e] = A.B[e] + (z - s);
      if (A.record) {
        const float u = z - s, v = z - A.zo[e];
        rp2 += (double)u * u;
        dz2 += (double)v * v;
      }
    }
    if (hw) {
      const long pw = fw + i;
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
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    block_sum(rp2, A.partial + 0 * A.pstride + b);
    block_sum(dz2, A.partial + 4 * A.pstride + b);
  }
}

// out[j] = sum of the first count[j] partials of slot j (one block, fixed order).
__global__ __launch_bounds__(RB) void rp_reduce_kernel(const double* partial, int pstride, RpCounts cnt, double* out) {
  for (int j = 0; j < RP_SLOTS; ++j) {
    double v = 0.0;
    for (int b = threadIdx.x; b < cnt.n[j]; b += RB) v += partial[(long)j * pstride + b];
    block_sum(v, out + j);
  }
}

// Input check: counts the non-finite entries of y and phi into slot 0.
__global__ __launch_bounds__(RB) void rp_validate_kernel(long n, const float* y, const float* phi, double* partial) {
  double bad = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
    const float v = y[i], f = phi ? phi[i] : 1.f;
    bad += (isfinite(v) && isfinite(f)) ? 0.0 : 1.0;
  }
  block_sum(bad, partial + blockIdx.x);
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

hipError_t launch_rp_sx(const RpArgs& a, int bx, hipStream_t s) {
  hipLaunchKernelGGL(rp_sx_kernel, dim3(bx, a.T), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_gram(const RpArgs& a, int blocks, double* gpart, hipStream_t s) {
  hipLaunchKernelGGL(rp_gram_kernel, dim3(blocks), dim3(RB), 0, s, a, gpart);
  return hipGetLastError();
}

hipError_t launch_rp_gram_reduce(const double* gpart, int blocks, int T, double* G, hipStream_t s) {
  const int np = T * (T + 1) / 2;
  hipLaunchKernelGGL(rp_gram_reduce_kernel, dim3((np + 63) / 64), dim3(RB), 0, s, gpart, blocks, np, G);
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

hipError_t launch_rp_dual(const RpArgs& a, int bx, hipStream_t s) {
  hipLaunchKernelGGL(rp_dual_kernel, dim3(bx, a.T), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_reduce(const double* partial, int pstride, const RpCounts& cnt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(rp_reduce_kernel, dim3(1), dim3(RB), 0, s, partial, pstride, cnt, out);
  return hipGetLastError();
}

hipError_t launch_rp_validate(long n, const float* y, const float* phi, double* partial, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_validate_kernel, dim3(blocks), dim3(RB), 0, s, n, y, phi, partial);
  return hipGetLastError();
}

}  // namespace uot
