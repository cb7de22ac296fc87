// Neumann-Poisson solve (alpha I + D D*) phi = c on one grid, for the
// zero-flux boundary, where D D* is the grid Laplacian with Neumann ends and
// the orthonormal DCT-II diagonalises it with eigenvalues
//     4 sin^2(pi kx / (2 nx)) + 4 sin^2(pi ky / (2 ny)).
// The 2-D transform is separable: T = Cy c Cx^T, divide by the eigenvalues,
// phi = Cy^T T Cx, i.e. four dense products with the DCT matrices, done on
// the FP32 matrix cores (v_mfma_f32_32x32x2f32).  Also the kernels that use
// phi: the Poisson-flux warm start and the feasibility repair of the
// balanced certificate.
#include "uot_internal.hpp"

#include <algorithm>

namespace uot {

namespace {
constexpr int GT = 32;   // output tile of one workgroup
constexpr int GK = 32;   // K slab of one wave
}  // namespace

// C[M x N] = op(A) op(B), row-major FP32.  op(A) is M x K: A[m*lda+k], or
// A[k*lda+m] when TA.  op(B) is K x N: B[k*ldb+n], or B[n*ldb+k] when TB.
// On v_mfma_f32_32x32x2f32: a workgroup of four waves owns a 32 x 32 output
// tile, wave w takes the K slabs w, w + 4, ... (32 wide), stages each slab
// of op(A) and op(B) in its own LDS buffers with global reads along the
// contiguous dimension, and the four partial tiles are added in a fixed
// order at the end.  Lane l supplies A[l%32][l/32] and B[l/32][l%32] of
// each K = 2 step and holds C rows 8(r/4) + 4(l/32) + r%4, column l%32, in
// accumulator register r.
//
// With SPEC the product is the forward transform T = Cy (c Cx^T) (M = ny,
// N = nx), and each output element is divided by its eigenvalue
// alpha + 4 sin^2(pi n / (2 N)) + 4 sin^2(pi m / (2 M)) on the way out (the
// constant mode dropped when that is zero), in place of a separate pass.
template <bool TA, bool TB, bool SPEC = false>
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                    const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                    int ldc, float alpha = 0.f) {
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  constexpr int LT = GT + 1;
  __shared__ float As[4][GK][LT];  // [wave][k][m]
  __shared__ float Bs[4][GK][LT];  // [wave][k][n]
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  f32x16 acc = {};
  // slab loads: 32 x 32 of op(A) and of op(B) as 256 quads each, four per
  // lane, along the contiguous dimension; whole quads are read with one
  // 16-byte load where the leading dimension allows it
  const bool qa = (lda & 3) == 0 && ((uintptr_t)A & 15) == 0;
  const bool qb = (ldb & 3) == 0 && ((uintptr_t)B & 15) == 0;
  float ra[4][4], rb[4][4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = l + 64 * q, major = idx >> 3, c = 4 * (idx & 7);
      // op(A): !TA rows m = m0 + major, k = k0 + c..c+3; TA rows k = k0 + major, m = m0 + c..c+3
      {
        const int r0 = TA ? k0 + major : m0 + major, c0 = TA ? m0 + c : k0 + c;
        const int rl = TA ? K : M, cl = TA ? M : K;
        const float* src = A + (long)r0 * lda + c0;
        if (qa && r0 < rl && c0 + 3 < cl) {
          const float4 v = *reinterpret_cast<const float4*>(src);
          ra[q][0] = v.x, ra[q][1] = v.y, ra[q][2] = v.z, ra[q][3] = v.w;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) ra[q][t] = (r0 < rl && c0 + t < cl) ? src[t] : 0.f;
        }
      }
      // op(B): !TB rows k = k0 + major, n = n0 + c..c+3; TB rows n = n0 + major, k = k0 + c..c+3
      {
        const int r0 = TB ? n0 + major : k0 + major, c0 = TB ? k0 + c : n0 + c;
        const int rl = TB ? N : K, cl = TB ? K : N;
        const float* src = B + (long)r0 * ldb + c0;
        if (qb && r0 < rl && c0 + 3 < cl) {
          const float4 v = *reinterpret_cast<const float4*>(src);
          rb[q][0] = v.x, rb[q][1] = v.y, rb[q][2] = v.z, rb[q][3] = v.w;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) rb[q][t] = (r0 < rl && c0 + t < cl) ? src[t] : 0.f;
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = l + 64 * q, major = idx >> 3, c = 4 * (idx & 7);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (TA) As[wv][major][c + t] = ra[q][t];
        else As[wv][c + t][major] = ra[q][t];
        if (TB) Bs[wv][c + t][major] = rb[q][t];
        else Bs[wv][major][c + t] = rb[q][t];
      }
    }
  };
  load(wv * GK);
  for (int kb = 0; kb < K; kb += 4 * GK) {  // the same trip count for every wave
    store();
    __syncthreads();
    if (kb + 4 * GK < K) load(kb + 4 * GK + wv * GK);  // next slab in flight during the products
#pragma unroll
    for (int s2 = 0; s2 < GK / 2; ++s2) {
      const int k = 2 * s2 + (l >> 5);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[wv][k][l & 31], Bs[wv][k][l & 31], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // the four partial tiles, added in wave order
  float* part = &As[0][0][0];  // 4 x 32 x 33 floats, free after the loop
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), col = l & 31;
    part[(wv * GT + row) * LT + col] = acc[r];
  }
  __syncthreads();
  // a thread's output column is the same for every q (256 is a multiple of 32)
  const double sx = SPEC ? sin(3.14159265358979323846 * (n0 + (threadIdx.x & 31)) / (2.0 * N)) : 0.0;
#pragma unroll
  for (int q = 0; q < GT * GT / 256; ++q) {
    const int idx = threadIdx.x + 256 * q, row = idx >> 5, col = idx & 31;
    const float v = ((part[(0 * GT + row) * LT + col] + part[(1 * GT + row) * LT + col]) +
                     part[(2 * GT + row) * LT + col]) + part[(3 * GT + row) * LT + col];
    const int m = m0 + row, n = n0 + col;
    if (m < M && n < N) {
      if (SPEC) {
        const double sy = sin(3.14159265358979323846 * m / (2.0 * M));
        const double lam = (double)alpha + 4.0 * sx * sx + 4.0 * sy * sy;
        C[(long)m * ldc + n] = lam > 0.0 ? (float)(v / lam) : 0.f;
      } else {
        C[(long)m * ldc + n] = v;
      }
    }
  }
}

// Poisson-flux start on one grid: M0 = -D* phi (zero-flux edges), r0 = D M0 +
// c so that K z0 = 0, a0 = 0; the free arguments start at their prox centres.
// phi is contiguous; images and state have row stride pitch.
__global__ void poisson_start_kernel(const float* phi, const float* src, const float* dst, Planes st, int nx,
                                     int ny, int pitch, int mode, int balanced) {
  const long n = (long)nx * ny;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    auto mx_at = [&](int ii, int jj) -> float {
      if (ii < 0 || ii >= nx - 1) return 0.f;
      const long o = (long)jj * nx + ii;
      return -(phi[o] - phi[o + 1]);
    };
    auto my_at = [&](int ii, int jj) -> float {
      if (jj < 0 || jj >= ny - 1) return 0.f;
      const long o = (long)jj * nx + ii;
      return -(phi[o] - phi[o + nx]);
    };
    const long g = (long)j * pitch + i;
    const float mx = mx_at(i, j), my = my_at(i, j);
    st.Mx[g] = mx;
    st.My[g] = my;
    st.a[g] = 0.f;
    const float dm = mx - mx_at(i - 1, j) + my - my_at(i, j - 1);
    const float c = dst[g] - src[g];
    if (!balanced) st.r[g] = dm + c;
    if (mode == 1) st.x0[g] = src[g];
    if (mode != 0) st.x1[g] = dst[g];
  }
}

// e = D M + c of a state (the infeasibility the balanced repair removes);
// Mx = My = nullptr stands for the zero flux.  e is contiguous.
__global__ void infeasibility_kernel(const float* Mx, const float* My, const float* src, const float* dst,
                                     float* e_out, int nx, int ny, int pitch) {
  const long n = (long)nx * ny;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    const long g = (long)j * pitch + i;
    float dm = 0.f;
    if (Mx) {
      const float mx = i < nx - 1 ? Mx[g] : 0.f;
      const float my = j < ny - 1 ? My[g] : 0.f;
      const float mxl = i > 0 ? Mx[g - 1] : 0.f;
      const float myd = j > 0 ? My[g - pitch] : 0.f;
      dm = (mx - mxl) + (my - myd);
    }
    e_out[e] = dm + (dst[g] - src[g]);
  }
}

// Partial sums of ||(M - D* phi)_i||: the flux norm of the repaired flux
// (phi contiguous, M with row stride pitch); aniso: |.|_1 per pixel.
__global__ __launch_bounds__(256) void repaired_norm_kernel(const float* Mx, const float* My, const float* phi,
                                                            int nx, int ny, int pitch, int aniso, double* partial) {
  __shared__ double red[256];
  const long n = (long)nx * ny;
  double acc = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    const long g = (long)j * pitch + i;
    const float gx = i < nx - 1 ? phi[e] - phi[e + 1] : 0.f;
    const float gy = j < ny - 1 ? phi[e] - phi[e + nx] : 0.f;
    const float mx = (i < nx - 1 ? Mx[g] : 0.f) - gx;
    const float my = (j < ny - 1 ? My[g] : 0.f) - gy;
    acc += aniso ? fabsf(mx) + fabsf(my) : sqrtf(mx * mx + my * my);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_sgemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                        float* C, int ldc, hipStream_t s) {
  const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  if (!ta && !tb) hipLaunchKernelGGL((sgemm_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else if (!ta && tb) hipLaunchKernelGGL((sgemm_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else if (ta && !tb) hipLaunchKernelGGL((sgemm_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else hipLaunchKernelGGL((sgemm_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

static int elem_grid(long n) { return (int)std::min<long>(4096, std::max<long>(1, (n + 255) / 256)); }

hipError_t poisson_solve(const float* Cx, const float* Cy, int nx, int ny, float alpha, const float* rhs, float* phi,
                         float* t1, float* t2, hipStream_t s) {
  hipError_t e;
  // T1 = rhs Cx^T (transform along x)
  if ((e = launch_sgemm(false, true, ny, nx, nx, rhs, nx, Cx, nx, t1, nx, s)) != hipSuccess) return e;
  // T2 = Cy T1 (along y), divided by the spectrum in the product's epilogue
  hipLaunchKernelGGL((sgemm_kernel<false, false, true>), dim3((nx + GT - 1) / GT, (ny + GT - 1) / GT), dim3(256), 0,
                     s, ny, nx, ny, Cy, ny, t1, nx, t2, nx, alpha);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // T1 = Cy^T T2, phi = T1 Cx
  if ((e = launch_sgemm(true, false, ny, nx, ny, Cy, ny, t2, nx, t1, nx, s)) != hipSuccess) return e;
  return launch_sgemm(false, false, ny, nx, nx, t1, nx, Cx, nx, phi, nx, s);
}

hipError_t launch_poisson_start(const float* phi, const float* src, const float* dst, const Planes& st, int nx,
                                int ny, int pitch, int mode, int balanced, hipStream_t s) {
  hipLaunchKernelGGL(poisson_start_kernel, dim3(elem_grid((long)nx * ny)), dim3(256), 0, s, phi, src, dst, st, nx,
                     ny, pitch, mode, balanced);
  return hipGetLastError();
}

hipError_t launch_infeasibility(const float* Mx, const float* My, const float* src, const float* dst, float* e,
                                int nx, int ny, int pitch, hipStream_t s) {
  hipLaunchKernelGGL(infeasibility_kernel, dim3(elem_grid((long)nx * ny)), dim3(256), 0, s, Mx, My, src, dst, e,
                     nx, ny, pitch);
  return hipGetLastError();
}

int repaired_norm_blocks(int nx, int ny) { return std::min(1024, elem_grid((long)nx * ny)); }

hipError_t launch_repaired_norm(const float* Mx, const float* My, const float* phi, int nx, int ny, int pitch,
                                int aniso, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(repaired_norm_kernel, dim3(repaired_norm_blocks(nx, ny)), dim3(256), 0, s, Mx, My, phi, nx,
                     ny, pitch, aniso, partial);
  return hipGetLastError();
}

}  // namespace uot
