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

// The multiplier steps of one iteration fused with the s- and x-steps of
// the next (within a check window): a <- a + x - s, b <- b + z - s, then
// s, x, the prox centre from the new a, b, with the expressions of
// df_ab_kernel and df_sx_kernel (so the iterates are the same bit for bit)
// and 12 planes streamed instead of 16.  record: the next iteration is the
// last of its window (leave ||x - x_prev||^2 and the copy of z).
__global__ __launch_bounds__(RB) void df_absx_kernel(DfArgs A) {
  double dx2 = 0.0;
  const float rho = A.rho, thr = A.thr;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < A.n; i += (long)gridDim.x * RB) {
    const float x = A.x[i], s = A.s[i], z = A.z[i];
    const float a = A.a[i] + (x - s);
    const float b = A.b[i] + (z - s);
    A.a[i] = a;
    A.b[i] = b;
    const float ph = A.phi ? A.phi[i] : 1.f;
    const float sn = fmaxf(0.5f * ((x + a) + (z + b)) - thr, 0.f);
    const float xn = (ph * A.y[i] + rho * (sn - a)) / (ph * ph + rho);
    A.s[i] = sn;
    A.x[i] = xn;
    A.p[i] = sn - b;
    if (A.record) {
      A.zo[i] = z;
      const float d = xn - x;
      dx2 += (double)d * d;
    }
  }
  if (A.record) block_sum(dx2, A.partial + 3 * blockIdx.x + 1);
}

// out[j] = sum over blocks of partial[3 b + j], j = 0..2 (block j, fixed order).
__global__ __launch_bounds__(RB) void df_reduce_kernel(const double* partial, int nblocks, double* out) {
  const int j = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RB) v += partial[3 * b + j];
  block_sum(v, out + j);
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
// With SGN (the sparse part S = S+ - S-, eq. RPCA_UOTDF_PN) S holds S+, Sm
// holds S-, the pair planes hold the + pairs then the - pairs (offset mo),
// and the blocks are minimised in the order S+, S-, L, X:
//   k+ = (x - l + s- + a) + (+ pairs),  k- = (l - x + s+ - a) + (- pairs)
//   l = max((Tn - D + x - s+ + s- + a) / 2, 0),  x = (phi y + rho (s+ - s- + l - a)) / (phi^2 + rho)
// z and w are saved (zo, wo) only where the residual is recorded.
template <bool SGN>
__global__ __launch_bounds__(RB) void rp_sx_kernel(RpArgs A) {
  double dx2 = 0.0;
  const int t = blockIdx.y;
  const long npx = A.npx, fe = (long)t * npx, fw = (long)(t - 1) * npx, mo = A.mo;
  const bool hz = t < A.T - 1, hw = t > 0;
  const float rho = A.rho, lam = A.lam;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    const long e = fe + i, ew = fw + i;
    const float x = A.X[e], l = A.L[e], a = A.A[e];
    float k = x - l + a, sig = 1.f, z = 0.f, w = 0.f, bz = 0.f, cw = 0.f;
    if (SGN) k += A.Sm[e];
    if (hz) {
      z = A.Z[e];
      bz = A.B[e];
      k += z + bz;
      sig += 1.f;
    }
    if (hw) {
      w = A.W[ew];
      cw = A.C[ew];
      k += w + cw;
      sig += 1.f;
    }
    const float s = fmaxf(k / sig - lam / (rho * sig), 0.f);
    float sm = 0.f, zm = 0.f, wm = 0.f, bm = 0.f, cm = 0.f;
    if (SGN) {
      float km = l - x + s - a;
      if (hz) {
        zm = A.Z[mo + e];
        bm = A.B[mo + e];
        km += zm + bm;
      }
      if (hw) {
        wm = A.W[mo + ew];
        cm = A.C[mo + ew];
        km += wm + cm;
      }
      sm = fmaxf(km / sig - lam / (rho * sig), 0.f);
    }
    const float ln = fmaxf(0.5f * (A.Tn[e] - A.D[e] + x - s + sm + a), 0.f);
    const float ph = A.phi ? A.phi[e] : 1.f;
    const float xn = (ph * A.y[e] + rho * (s - sm + ln - a)) / (ph * ph + rho);
    A.S[e] = s;
    if (SGN) A.Sm[e] = sm;
    A.L[e] = ln;
    A.X[e] = xn;
    if (hz) A.P0[e] = s - bz;
    if (hw) A.P1[ew] = s - cw;
    if (SGN) {
      if (hz) A.P0[mo + e] = sm - bm;
      if (hw) A.P1[mo + ew] = sm - cm;
    }
    if (A.record) {
      const float d = xn - x;
      dx2 += (double)d * d;
      if (hz) A.zo[e] = z;
      if (hw) A.wo[ew] = w;
      if (SGN) {
        if (hz) A.zo[mo + e] = zm;
        if (hw) A.wo[mo + ew] = wm;
      }
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
// waves take every fourth partial (32 loads in flight, added in block
// order), and the four sums are combined in a fixed order (the result does
// not depend on timing).
__global__ __launch_bounds__(RB) void rp_gram_reduce_kernel(const double* gpart, int blocks, int np, double* G) {
  __shared__ double red[RB / 64][64];
  constexpr int Q = RB / 64, U = 32;
  const int jl = threadIdx.x & 63, q = threadIdx.x >> 6, j = blockIdx.x * 64 + jl;
  double v = 0.0;
  if (j < np) {
    int b = q;
    for (; b + Q * (U - 1) < blocks; b += Q * U) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gpart[(long)(b + Q * u) * np + j];
#pragma unroll
      for (int u = 0; u < U; ++u) v += x[u];
    }
    for (; b < blocks; b += Q) v += gpart[(long)b * np + j];
  }
  red[q][jl] = v;
  __syncthreads();
  if (q == 0 && j < np) G[j] = (red[0][jl] + red[1][jl]) + (red[2][jl] + red[3][jl]);
}

// Singular-value threshold of M from its Gram matrix G = M^T M = V Lam V^T:
// SVT_thr(M) = M V diag(f) V^T with f_j = max(1 - thr / sigma_j, 0),
// sigma_j = sqrt(lam_j).  One kernel, one workgroup (rp_eig_kernel), from
// the previous call's eigenvectors V: the iteration moves little from one
// ADMM step to the next, so V^T G V is nearly diagonal.  V is refined by
// matrix products (below); where that does not apply, the cyclic Jacobi
// method with the parallel round-robin ordering (every round rotates 32
// disjoint pairs at once) diagonalises A = V^T G V and rotates V alongside.
// Either way the kernel leaves V, the eigenvalues and Wm = V diag(f) V^T.
// The matrices are padded to 64 x 64 (zero rows and columns of A, identity
// in V; no rotation touches the padding since its off-diagonal entries stay
// zero), so all index arithmetic is shifts.

// Round r of the round-robin: pair k of 32 is (p, q), p < q; player 63 is
// fixed, the others rotate.
__device__ __forceinline__ void rr_pair(int r, int k, int& p, int& q) {
  constexpr int N1 = RP_MAX_FRAMES - 1;
  int a = k == 0 ? r : (r + k) % N1;
  int b = k == 0 ? N1 : (r - k + N1) % N1;
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// acc = op(X) Y for 64 x 64 FP64 matrices in LDS (leading dimension 65),
// op(X) = X or X^T; thread (bi, bj) of 16 x 16 forms the 4 x 4 block at
// rows 4 bi, columns 4 bj.
template <bool TX>
__device__ __forceinline__ void mm64(const double* X, const double* Y, int bi, int bj, double (&acc)[4][4]) {
  constexpr int N = RP_MAX_FRAMES, LD = N + 1;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
  for (int k = 0; k < N; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = TX ? X[k * LD + 4 * bi + u] : X[(4 * bi + u) * LD + k];
      b[u] = Y[k * LD + 4 * bj + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
}

// The same products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  One
// instruction forms a 16 x 16 tile from a 16 x 4 slice of op(X) (lane l
// holds row l % 16, column l / 16) and a 4 x 16 slice of Y (row l / 16,
// column l % 16), and lane l accumulates rows l / 16 + 4 r (r < 4), column
// l % 16 of the tile.  Wave w forms the four tiles of rows 16 w .. 16 w + 15;
// c[t][r] is element (16 w + l / 16 + 4 r, 16 t + l % 16).  With two Y, the
// slices of op(X) are shared.
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <bool TX, int NY>
__device__ __forceinline__ void mm64_mfma(const double* X, const double* const (&Y)[NY], double (&c)[NY][4][4]) {
  constexpr int N = RP_MAX_FRAMES, LD = N + 1;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, m = l & 15, g = l >> 4;
  f64x4 acc[NY][4];
#pragma unroll
  for (int y = 0; y < NY; ++y)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[y][t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kc = 0; kc < N / 4; ++kc) {
    const int row = 16 * w + m, col = 4 * kc + g;
    const double a = TX ? X[col * LD + row] : X[row * LD + col];
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[y][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Y[y][col * LD + 16 * t + m], acc[y][t], 0, 0, 0);
  }
#pragma unroll
  for (int y = 0; y < NY; ++y)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) c[y][t][r] = acc[y][t][r];
}

// Two sums and a maximum over the block, the same in every thread (fixed
// order), through red[3][RB / 64].
__device__ __forceinline__ void block_sum2_max(double& s0, double& s1, double& m, double (*red)[RB / 64]) {
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_down(s0, o, 64);
    s1 += __shfl_down(s1, o, 64);
    m = fmax(m, __shfl_down(m, o, 64));
  }
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = s0;
    red[1][tid >> 6] = s1;
    red[2][tid >> 6] = m;
  }
  __syncthreads();
  s0 = red[0][0];
  s1 = red[1][0];
  m = red[2][0];
  for (int w = 1; w < RB / 64; ++w) {
    s0 += red[0][w];
    s1 += red[1][w];
    m = fmax(m, red[2][w]);
  }
  __syncthreads();
}

// Two sums and two maxima over the block, the same in every thread.
__device__ __forceinline__ void block_sum2_max2(double& s0, double& s1, double& m0, double& m1,
                                                double (*red)[RB / 64]) {
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_down(s0, o, 64);
    s1 += __shfl_down(s1, o, 64);
    m0 = fmax(m0, __shfl_down(m0, o, 64));
    m1 = fmax(m1, __shfl_down(m1, o, 64));
  }
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = s0;
    red[1][tid >> 6] = s1;
    red[2][tid >> 6] = m0;
    red[3][tid >> 6] = m1;
  }
  __syncthreads();
  s0 = red[0][0];
  s1 = red[1][0];
  m0 = red[2][0];
  m1 = red[3][0];
  for (int w = 1; w < RB / 64; ++w) {
    s0 += red[0][w];
    s1 += red[1][w];
    m0 = fmax(m0, red[2][w]);
    m1 = fmax(m1, red[3][w]);
  }
  __syncthreads();
}

// One workgroup.  A lives in LDS in FP64; after the start only its upper
// triangle (with the diagonal) is kept.  A round: 32 threads form the
// rotations (symmetric Schur, Golub and Van Loan); then every block of the
// upper triangle (pair k1 rows, pair k2 >= k1 columns) becomes
// R_k1^T A R_k2, each block owned by one thread, the diagonal blocks taking
// the exact diagonalisation.  V^T G V keeps a 4 x 4 block per thread.
//
// Before the sweeps, the warm start is refined by the iteration of Ogita and
// Aishima (2018) for symmetric eigenproblems, which needs only matrix
// products: with R = I - V^T V and S = V^T G V, the eigenvalue estimates are
// l_i = S_ii / (1 - R_ii), and V <- V + V E with E_ij = (S_ij + l_j R_ij) /
// (l_j - l_i) where |l_j - l_i| exceeds the cluster bound
// delta = 2 (||S - diag(l)|| + ||G|| ||R||) and E_ij = R_ij / 2 otherwise (and
// on the diagonal); the error falls quadratically.  The threshold needs only
// the matrix function Wm = V diag(f(l)) V^T, which does not depend on the
// basis inside the set of eigenvalues under the threshold (f = 0, most of
// them), so pairs inside that set are only re-orthogonalised (E = R / 2),
// never rotated, and the refinement stops when the first-order error of Wm,
// max over i != j of |S_ij| |f_i - f_j| / |l_i - l_j|, and ||R|| are both
// below 1e-9, provided a Gershgorin bound keeps every eigenvalue of the
// f = 0 block of S under thr^2.  It is abandoned (the original V and the
// sweeps take over) when S is far from diagonal (the first call, from the
// identity), when that bound fails, or after RP_MAX_REFINE passes, which is
// what happens when a cluster of close eigenvalues straddles the threshold.
__global__ __launch_bounds__(RB) void rp_eig_kernel(const double* G, int T, double thr, double* Vg, double* lam,
                                                     float* Wm, int* sweeps) {
  constexpr int N = RP_MAX_FRAMES, LD = N + 1, NP = N / 2;
  static_assert(N == 64 && RB == 256, "64 x 64 matrices, 16 x 16 threads of 4 x 4 blocks");
  __shared__ double Am[N * LD];
  __shared__ double Vm[N * LD];
  __shared__ double Gm[N * LD];
  __shared__ double Rm[N * LD];
  __shared__ double lt[N], ft[N];
  __shared__ double red3[3][RB / 64];
  __shared__ double red4[4][RB / 64];
  __shared__ double rot[NP][3];  // c, s, t = s / c
  __shared__ double red[2][RB / 64];
  __shared__ int prs[(N - 1) * NP];  // round r, pair k: p | q << 8
  const int tid = threadIdx.x;
  {
    // all loads in flight before the first store
    constexpr int PT = N * N / RB;
    double gv[PT], vv[PT];
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int e = tid + RB * m, i = e >> 6, j = e & (N - 1);
      gv[m] = 0.0;
      vv[m] = i == j ? 1.0 : 0.0;
      if (i < T && j < T) {
        const int p = i < j ? i : j, q = i < j ? j : i;
        gv[m] = G[p * T - p * (p - 1) / 2 + (q - p)];
        vv[m] = Vg[i * T + j];
      }
    }
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int e = tid + RB * m, i = e >> 6, j = e & (N - 1);
      Gm[i * LD + j] = gv[m];
      Vm[i * LD + j] = vv[m];
    }
  }
  __syncthreads();
  const int bi = tid >> 4, bj = tid & 15;
  double acc[4][4];

  // ---- refinement of the warm start ----
  double gn = 0.0, z0 = 0.0, z1 = 0.0;
  for (int e = tid; e < N * N; e += RB) {
    const double g = Gm[(e >> 6) * LD + (e & (N - 1))];
    gn += g * g;
  }
  block_sum2_max(gn, z0, z1, red3);
  gn = sqrt(gn);
  bool refined = false;
  // element (mi + 4 r, 16 t + mj) of a product is c[t][r] of this thread
  const int mi = 16 * (tid >> 6) + ((tid & 63) >> 4), mj = tid & 15;
  for (int it = 0; it < RP_MAX_REFINE; ++it) {
    {
      double c[1][4][4];
      const double* const y1[1] = {Vm};
      mm64_mfma<false, 1>(Gm, y1, c);  // G V
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) Am[(mi + 4 * r) * LD + 16 * t + mj] = c[0][t][r];
    }
    __syncthreads();
    {
      double c[2][4][4];
      const double* const y2[2] = {Am, Vm};
      mm64_mfma<true, 2>(Vm, y2, c);  // S = V^T G V, V^T V
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = mi + 4 * r, j = 16 * t + mj;
          Am[i * LD + j] = c[0][t][r];
          Rm[i * LD + j] = (i == j ? 1.0 : 0.0) - c[1][t][r];
        }
    }
    __syncthreads();
    if (tid < N) {
      const double l = Am[tid * LD + tid] / (1.0 - Rm[tid * LD + tid]);
      const double sg = sqrt(fmax(l, 0.0));
      lt[tid] = l;
      ft[tid] = (tid < T && sg > thr) ? 1.0 - thr / sg : 0.0;
    }
    __syncthreads();
    // off: S off the diagonal over the pairs with f > 0 on either side (the
    // basis inside the f = 0 set is never rotated); werr: the first-order
    // error of Wm; gm: Gershgorin bound on the eigenvalues of the f = 0 block
    // of S, which must stay under thr^2 for that block to hold no eigenvalue
    // with f > 0.  Thread 4 i + q takes row i, columns q, q + 4, ...; the
    // row's Gershgorin sum is combined from its four threads (consecutive
    // lanes).
    double off = 0.0, rn = 0.0, werr = 0.0, gm = -INFINITY;
    {
      const int i = tid >> 2, q = tid & 3;
      const bool zi = i < T && ft[i] == 0.0;
      double gs = 0.0;
      if (i < T) {
#pragma unroll 4
        for (int j = q; j < T; j += 4) {
          const double r = Rm[i * LD + j];
          rn += r * r;
          if (j != i) {
            const double sij = Am[i * LD + j];
            const double fj = ft[j];
            if (ft[i] > 0.0 || fj > 0.0) off += sij * sij;
            if (zi && fj == 0.0) gs += fabs(sij);
            const double dl = fabs(lt[i] - lt[j]), df = fabs(ft[i] - fj);
            if (df > 0.0) werr = fmax(werr, dl > 0.0 ? fabs(sij) * df / dl : INFINITY);
          }
        }
      }
      gs += __shfl_xor(gs, 1, 4);
      gs += __shfl_xor(gs, 2, 4);
      if (zi) gm = lt[i] + gs;
    }
    block_sum2_max2(off, rn, werr, gm, red4);  // uniform over the block
    off = sqrt(off);
    rn = sqrt(rn);
    const bool zero_block_ok = gm <= thr * thr;
    if (werr <= 1e-9 && rn <= 1e-9 && zero_block_ok) {
      refined = true;
      break;
    }
    if (!(off <= 1e-2 * gn) || !zero_block_ok || it + 1 == RP_MAX_REFINE) break;  // the sweeps take over
    const double delta = 2.0 * (off + gn * rn);
    for (int e = tid; e < N * N; e += RB) {  // E in place of R
      const int i = e >> 6, j = e & (N - 1);
      const double r = Rm[i * LD + j], dl = lt[j] - lt[i];
      const bool rot = i != j && (ft[i] > 0.0 || ft[j] > 0.0) && fabs(dl) > delta;
      Rm[i * LD + j] = rot ? (Am[i * LD + j] + lt[j] * r) / dl : 0.5 * r;
    }
    __syncthreads();
    {
      double c[1][4][4];
      const double* const y1[1] = {Rm};
      mm64_mfma<false, 1>(Vm, y1, c);  // V E
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) Vm[(mi + 4 * r) * LD + 16 * t + mj] += c[0][t][r];
    }
    __syncthreads();
  }
  // The result: the eigenvalues, V, and Wm = V diag(f) V^T (Rm <- diag(f)
  // V^T, then V Rm on the matrix cores); ft must hold f.
  auto finish = [&](int nsweeps) {
    for (int e = tid; e < T * T; e += RB) Vg[e] = Vm[(e / T) * LD + e % T];
    for (int e = tid; e < N * N; e += RB) {
      const int k = e >> 6, j = e & (N - 1);
      Rm[k * LD + j] = ft[k] * Vm[j * LD + k];
    }
    __syncthreads();
    double c[1][4][4];
    const double* const y1[1] = {Rm};
    mm64_mfma<false, 1>(Vm, y1, c);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mi + 4 * r, j = 16 * t + mj;
        if (i < T && j < T) Wm[i * T + j] = (float)c[0][t][r];
      }
    if (tid == 0) *sweeps = nsweeps;
  };
  if (refined) {
    if (tid < N) lam[tid] = lt[tid];
    finish(0);
    return;  // uniform
  }
  // the sweeps start again from the caller's V
  for (int e = tid; e < N * N; e += RB) {
    const int i = e >> 6, j = e & (N - 1);
    Vm[i * LD + j] = (i < T && j < T) ? Vg[i * T + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();

  // Am <- G V
  mm64<false>(Gm, Vm, bi, bj, acc);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Am[(4 * bi + u) * LD + 4 * bj + v] = acc[u][v];
  __syncthreads();
  // Am <- V^T Am
  mm64<true>(Vm, Am, bi, bj, acc);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Am[(4 * bi + u) * LD + 4 * bj + v] = acc[u][v];
  __syncthreads();

  for (int e = tid; e < (N - 1) * NP; e += RB) {  // the round-robin pairs (read after the next barrier)
    int p, q;
    rr_pair(e / NP, e % NP, p, q);
    prs[e] = p | q << 8;
  }
  auto up = [](int i, int j) { return i < j ? i * LD + j : j * LD + i; };  // upper-triangle slot
  int sweep = 0;
  for (; sweep < RP_MAX_SWEEPS; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < N * N; e += RB) {
      const int i = e >> 6, j = e & (N - 1);
      if (i <= j) {
        const double v = Am[i * LD + j];
        const double w2 = i == j ? v * v : 2.0 * v * v;
        tot += w2;
        if (i != j) off += w2;
      }
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
        const int pqv = prs[r * NP + tid], p = pqv & 255, q = pqv >> 8;
        // symmetric Schur: t = tan of the angle that zeroes A[p][q]
        const double apq = Am[p * LD + q], d = Am[q * LD + q] - Am[p * LD + p];
        double c = 1.0, s_ = 0.0, t = 0.0;
        if (apq != 0.0) {
          t = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) / (fabs(d) + sqrt(d * d + 4.0 * apq * apq));
          c = rsqrt(1.0 + t * t);
          s_ = t * c;
        }
        rot[tid][0] = c;
        rot[tid][1] = s_;
        rot[tid][2] = t;
      }
      __syncthreads();
      // V <- V J: row i, pair k: (V_ip, V_iq) <- (c V_ip - s V_iq, s V_ip + c V_iq)
#pragma unroll
      for (int m = 0; m < N * NP / RB; ++m) {
        const int e = tid + RB * m, i = e >> 5, k = e & (NP - 1);
        const int pq = prs[r * NP + k], p = pq & 255, q = pq >> 8;
        const double c = rot[k][0], sn = rot[k][1];
        const double vp = Vm[i * LD + p], vq = Vm[i * LD + q];
        Vm[i * LD + p] = c * vp - sn * vq;
        Vm[i * LD + q] = sn * vp + c * vq;
      }
      // every upper-triangle block of this round, branch-free: a diagonal
      // block (k1 = k2) writes its first off-diagonal slot twice, both zero
      const int k2 = tid & (NP - 1), pq2 = prs[r * NP + k2], p2 = pq2 & 255, q2 = pq2 >> 8;
      const double c2 = rot[k2][0], s2 = rot[k2][1];
      int ix[NP / 8][4];
      double nv[NP / 8][4];
#pragma unroll
      for (int m = 0; m < NP / 8; ++m) {
        const int k1 = (tid >> 5) + 8 * m;
        const int pq1 = prs[r * NP + k1], p1 = pq1 & 255, q1 = pq1 >> 8;
        ix[m][0] = up(p1, p2);
        ix[m][1] = up(p1, q2);
        ix[m][2] = up(q1, p2);
        ix[m][3] = up(q1, q2);
        const double a = Am[ix[m][0]], b = Am[ix[m][1]], cc = Am[ix[m][2]], d = Am[ix[m][3]];
        const double c1 = rot[k1][0], s1 = rot[k1][1], t1 = rot[k1][2];
        const double rpp = c1 * a - s1 * cc, rpq = c1 * b - s1 * d;
        const double rqp = s1 * a + c1 * cc, rqq = s1 * b + c1 * d;
        const bool dg = k1 == k2;
        nv[m][0] = dg ? a - t1 * b : c2 * rpp - s2 * rpq;
        nv[m][1] = dg ? 0.0 : s2 * rpp + c2 * rpq;
        nv[m][2] = dg ? 0.0 : c2 * rqp - s2 * rqq;
        nv[m][3] = dg ? d + t1 * b : s2 * rqp + c2 * rqq;
      }
#pragma unroll
      for (int m = 0; m < NP / 8; ++m) {
        if ((tid >> 5) + 8 * m <= k2) {
#pragma unroll
          for (int u = 0; u < 4; ++u) Am[ix[m][u]] = nv[m][u];
        }
      }
      __syncthreads();
    }
  }
  if (tid < N) {
    const double l = Am[tid * LD + tid], sg = sqrt(fmax(l, 0.0));
    lam[tid] = l;
    ft[tid] = (tid < T && sg > thr) ? 1.0 - thr / sg : 0.0;
  }
  __syncthreads();
  finish(sweep);
}

// Tn = (L + D) Wm per pixel, then D <- (L + D) - Tn (= D + L - Tn): for 32
// pixels at a time, Tn^T = Wm^T (L + D)^T is two 32 x 32 output tiles of
// v_mfma_f32_32x32x2f32 over K = 64 frames.  Lane l supplies A[l%32][l/32]
// and B[l/32][l%32] and holds D rows 8(r/4) + 4(l/32) + r%4, column l%32,
// in register r.  The K order is free, so step kk gives lane half h frame
// 8(kk/4) + 4h + kk%4: the frames a lane loads for B are then exactly the
// output frames it holds, and D - Tn needs no exchange.  Wm^T stays in
// registers; (L + D) is streamed once.
__device__ __forceinline__ int svt_frame(int kk, int h) { return 8 * (kk >> 2) + 4 * h + (kk & 3); }

__global__ __launch_bounds__(RB) void rp_svt_apply_kernel(RpArgs A) {
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  const int T = A.T;
  const long npx = A.npx;
  const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
  const long wave = (long)blockIdx.x * (RB / 64) + (threadIdx.x >> 6), nw = (long)gridDim.x * (RB / 64);
  float wa[2][32];
#pragma unroll
  for (int tau = 0; tau < 2; ++tau)
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
      const int s_ = svt_frame(kk, h), t = 32 * tau + j;
      wa[tau][kk] = (s_ < T && t < T) ? A.Wm[s_ * T + t] : 0.f;
    }
  double lt2 = 0.0, dt2 = 0.0;
  for (long g = wave; g * 32 < npx; g += nw) {
    const long i = g * 32 + j;
    const bool valid = i < npx;
    float m[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
      const int s_ = svt_frame(kk, h);
      m[kk] = (valid && s_ < T) ? A.L[(long)s_ * npx + i] + A.D[(long)s_ * npx + i] : 0.f;
    }
    f32x16 c0 = {}, c1 = {};
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[0][kk], m[kk], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[1][kk], m[kk], c1, 0, 0, 0);
    }
    if (!valid) continue;
#pragma unroll
    for (int tau = 0; tau < 2; ++tau)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int t = svt_frame(16 * tau + r, h);
        if (t < T) {
          const float tn = tau == 0 ? c0[r] : c1[r];
          const long e = (long)t * npx + i;
          if (A.record) {
            const float d1 = A.L[e] - tn, d2 = tn - A.Tn[e];
            lt2 += (double)d1 * d1;
            dt2 += (double)d2 * d2;
          }
          A.Tn[e] = tn;
          A.D[e] = m[16 * tau + r] - tn;
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
// (t above the first); with SGN, A += X - S+ + S- - L and the - pairs'
// multipliers follow S- the same way.
template <bool SGN>
__global__ __launch_bounds__(RB) void rp_dual_kernel(RpArgs A) {
  double rp2 = 0.0, dz2 = 0.0;
  const int t = blockIdx.y;
  const long npx = A.npx, fe = (long)t * npx, fw = (long)(t - 1) * npx, mo = A.mo;
  const bool hz = t < A.T - 1, hw = t > 0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    const long e = fe + i, ew = fw + i;
    const float x = A.X[e], s = A.S[e], l = A.L[e];
    const float sm = SGN ? A.Sm[e] : 0.f;
    const float u0 = SGN ? x - s + sm - l : x - s - l;
    A.A[e] = A.A[e] + u0;
    if (A.record) rp2 += (double)u0 * u0;
#pragma unroll
    for (int g = 0; g < (SGN ? 2 : 1); ++g) {
      const long o = g ? mo : 0;
      const float sv = g ? sm : s;
      if (hz) {
        const float z = A.Z[o + e];
        A.B[o + e] = A.B[o + e] + (z - sv);
        if (A.record) {
          const float u = z - sv, v = z - A.zo[o + e];
          rp2 += (double)u * u;
          dz2 += (double)v * v;
        }
      }
      if (hw) {
        const float w = A.W[o + ew];
        A.C[o + ew] = A.C[o + ew] + (w - sv);
        if (A.record) {
          const float u = w - sv, v = w - A.wo[o + ew];
          rp2 += (double)u * u;
          dz2 += (double)v * v;
        }
      }
    }
  }
  if (A.record) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    block_sum(rp2, A.partial + 0 * A.pstride + b);
    block_sum(dz2, A.partial + 4 * A.pstride + b);
  }
}

// The multiplier steps of one iteration fused with the S-, L- and X-steps
// of the next (within a check window): A, b, c (and the - pairs' b, c)
// updated as in rp_dual_kernel, then the next iteration's steps as in
// rp_sx_kernel from the updated multipliers, with the same expressions (the
// iterates are the same bit for bit) and each plane streamed once.
// record: the next iteration is the last of its window.
template <bool SGN>
__global__ __launch_bounds__(RB) void rp_dualsx_kernel(RpArgs A) {
  double dx2 = 0.0;
  const int t = blockIdx.y;
  const long npx = A.npx, fe = (long)t * npx, fw = (long)(t - 1) * npx, mo = A.mo;
  const bool hz = t < A.T - 1, hw = t > 0;
  const float rho = A.rho, lam = A.lam;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < npx; i += (long)gridDim.x * RB) {
    const long e = fe + i, ew = fw + i;
    const float x = A.X[e], so = A.S[e], l = A.L[e];
    const float smo = SGN ? A.Sm[e] : 0.f;
    // multiplier steps of the finished iteration
    const float a = A.A[e] + (SGN ? x - so + smo - l : x - so - l);
    A.A[e] = a;
    float z = 0.f, w = 0.f, bz = 0.f, cw = 0.f, zm = 0.f, wm = 0.f, bm = 0.f, cm = 0.f;
    if (hz) {
      z = A.Z[e];
      bz = A.B[e] + (z - so);
      A.B[e] = bz;
      if (SGN) {
        zm = A.Z[mo + e];
        bm = A.B[mo + e] + (zm - smo);
        A.B[mo + e] = bm;
      }
    }
    if (hw) {
      w = A.W[ew];
      cw = A.C[ew] + (w - so);
      A.C[ew] = cw;
      if (SGN) {
        wm = A.W[mo + ew];
        cm = A.C[mo + ew] + (wm - smo);
        A.C[mo + ew] = cm;
      }
    }
    // S-, L-, X-steps of the next iteration
    float k = x - l + a, sig = 1.f;
    if (SGN) k += smo;
    if (hz) {
      k += z + bz;
      sig += 1.f;
    }
    if (hw) {
      k += w + cw;
      sig += 1.f;
    }
    const float s = fmaxf(k / sig - lam / (rho * sig), 0.f);
    float sm = 0.f;
    if (SGN) {
      float km = l - x + s - a;
      if (hz) km += zm + bm;
      if (hw) km += wm + cm;
      sm = fmaxf(km / sig - lam / (rho * sig), 0.f);
    }
    const float ln = fmaxf(0.5f * (A.Tn[e] - A.D[e] + x - s + sm + a), 0.f);
    const float ph = A.phi ? A.phi[e] : 1.f;
    const float xn = (ph * A.y[e] + rho * (s - sm + ln - a)) / (ph * ph + rho);
    A.S[e] = s;
    if (SGN) A.Sm[e] = sm;
    A.L[e] = ln;
    A.X[e] = xn;
    if (hz) A.P0[e] = s - bz;
    if (hw) A.P1[ew] = s - cw;
    if (SGN) {
      if (hz) A.P0[mo + e] = sm - bm;
      if (hw) A.P1[mo + ew] = sm - cm;
    }
    if (A.record) {
      const float d = xn - x;
      dx2 += (double)d * d;
      if (hz) A.zo[e] = z;
      if (hw) A.wo[ew] = w;
      if (SGN) {
        if (hz) A.zo[mo + e] = zm;
        if (hw) A.wo[mo + ew] = wm;
      }
    }
  }
  if (A.record) block_sum(dx2, A.partial + 1 * A.pstride + blockIdx.y * gridDim.x + blockIdx.x);
}

// out = a - b (the signed sparse part S+ - S-).
__global__ __launch_bounds__(RB) void rp_sub_kernel(long n, const float* a, const float* b, float* out) {
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) out[i] = a[i] - b[i];
}

// out[j] = sum of the first count[j] partials of slot j: block j, fixed order.
__global__ __launch_bounds__(RB) void rp_reduce_kernel(const double* partial, int pstride, RpCounts cnt, double* out) {
  const int j = blockIdx.x;
  const int n = cnt.n[j];
  const double* p = partial + (long)j * pstride;
  double v = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * RB < n; b += 8 * RB) {  // eight loads in flight, added in order
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = p[b + u * RB];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += w[u];
  }
  for (; b < n; b += RB) v += p[b];
  block_sum(v, out + j);
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

hipError_t launch_df_absx(const DfArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(df_absx_kernel, dim3(df_blocks(a.n)), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_df_reduce(const double* partial, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(df_reduce_kernel, dim3(3), dim3(RB), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_df_validate(long n, const float* y, const float* phi, const float* s0, double* partial,
                              hipStream_t s) {
  hipLaunchKernelGGL(df_validate_kernel, dim3(df_blocks(n)), dim3(RB), 0, s, n, y, phi, s0, partial);
  return hipGetLastError();
}

hipError_t launch_rp_sx(const RpArgs& a, int bx, hipStream_t s) {
  if (a.Sm) hipLaunchKernelGGL(rp_sx_kernel<true>, dim3(bx, a.T), dim3(RB), 0, s, a);
  else hipLaunchKernelGGL(rp_sx_kernel<false>, dim3(bx, a.T), dim3(RB), 0, s, a);
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

hipError_t launch_rp_eig(const double* G, int T, double thr, double* V, double* lam, float* Wm, int* sweeps,
                         hipStream_t s) {
  hipLaunchKernelGGL(rp_eig_kernel, dim3(1), dim3(RB), 0, s, G, T, thr, V, lam, Wm, sweeps);
  return hipGetLastError();
}

hipError_t launch_rp_svt_apply(const RpArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_svt_apply_kernel, dim3(blocks), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_dual(const RpArgs& a, int bx, hipStream_t s) {
  if (a.Sm) hipLaunchKernelGGL(rp_dual_kernel<true>, dim3(bx, a.T), dim3(RB), 0, s, a);
  else hipLaunchKernelGGL(rp_dual_kernel<false>, dim3(bx, a.T), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_dualsx(const RpArgs& a, int bx, hipStream_t s) {
  if (a.Sm) hipLaunchKernelGGL(rp_dualsx_kernel<true>, dim3(bx, a.T), dim3(RB), 0, s, a);
  else hipLaunchKernelGGL(rp_dualsx_kernel<false>, dim3(bx, a.T), dim3(RB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rp_sub(long n, const float* a, const float* b, float* out, hipStream_t s) {
  hipLaunchKernelGGL(rp_sub_kernel, dim3(df_blocks(n)), dim3(RB), 0, s, n, a, b, out);
  return hipGetLastError();
}

hipError_t launch_rp_reduce(const double* partial, int pstride, const RpCounts& cnt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(rp_reduce_kernel, dim3(RP_SLOTS), dim3(RB), 0, s, partial, pstride, cnt, out);
  return hipGetLastError();
}

hipError_t launch_rp_validate(long n, const float* y, const float* phi, double* partial, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(rp_validate_kernel, dim3(blocks), dim3(RB), 0, s, n, y, phi, partial);
  return hipGetLastError();
}

}  // namespace uot
