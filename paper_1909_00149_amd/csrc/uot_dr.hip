// HIP kernels (gfx950) of the Douglas-Rachford splitting of the UOT
// problems, the projection-based alternative to Algorithm 1:
//   z = prox_{gamma G}(w), u = 2 z - w,
//   e = K u - b                            (dr_prox_rhs_kernel)
//   (n I + D D*) phi = e                   (the DCT Poisson solve)
//   y = u - K^T phi,  w <- w + y - z       (dr_update_kernel)
// G holds the separable terms: the flux norm (group or component shrink),
// the residual penalty mu ||r||_1 or mu ||r||^2, and in the prox modes the
// quadratic ||x - p||^2 / (2 rho) with x >= 0.  K z = D M - x0 + x1 - r
// (the terms present in the mode); one grid, contiguous rows, zero-flux
// boundary (Mx of the last column and My of the last row are structurally
// zero and stay so: D* phi vanishes there).  Element-wise kernels, each
// plane read and written once per iteration.
#include "uot_internal.hpp"

namespace uot {

namespace {

constexpr int DB = 256;

__device__ __forceinline__ float dr_shrink1(float v, float s) {
  const float m = fabsf(v) - s;
  return m > 0.f ? copysignf(m, v) : 0.f;
}

__device__ __forceinline__ double dr_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < DB / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

}  // namespace

// Prox of gamma times the flux norm at one pixel (group or component shrink).
__device__ __forceinline__ void dr_flux_prox(float wx, float wy, float g, int aniso, float& zx, float& zy) {
  if (aniso) {
    zx = dr_shrink1(wx, g);
    zy = dr_shrink1(wy, g);
  } else {
    const float n2 = wx * wx + wy * wy;
    const float s = n2 > g * g ? 1.f - g * rsqrtf(n2) : 0.f;
    zx = s * wx;
    zy = s * wy;
  }
}

// z = prox(w), u = 2 z - w, and e = K u - b in one pass: D M_u needs u's
// flux at the left and lower neighbours, which is recomputed from w there
// (the flux prox is per pixel), so u is not read back.
__global__ __launch_bounds__(DB) void dr_prox_rhs_kernel(DrArgs A, float* out) {
  const int nx = A.nx, ny = A.ny;
  const long n = (long)nx * ny;
  const float g = A.gamma;
  for (long e = blockIdx.x * (long)DB + threadIdx.x; e < n; e += (long)gridDim.x * DB) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    const float wx = A.w.Mx[e], wy = A.w.My[e];
    float zx, zy;
    dr_flux_prox(wx, wy, g, A.aniso, zx, zy);
    const float ux = 2.f * zx - wx, uy = 2.f * zy - wy;
    A.z.Mx[e] = zx;
    A.z.My[e] = zy;
    A.u.Mx[e] = ux;
    A.u.My[e] = uy;
    float uxl = 0.f, uyd = 0.f;
    if (i > 0) {
      const float lx = A.w.Mx[e - 1], ly = A.w.My[e - 1];
      float qx, qy;
      dr_flux_prox(lx, ly, g, A.aniso, qx, qy);
      uxl = 2.f * qx - lx;
    }
    if (j > 0) {
      const float dx = A.w.Mx[e - nx], dy = A.w.My[e - nx];
      float qx, qy;
      dr_flux_prox(dx, dy, g, A.aniso, qx, qy);
      uyd = 2.f * qy - dy;
    }
    float v = (ux - uxl) + (uy - uyd);
    if (A.z.r) {
      const float wr = A.w.r[e];
      const float zr = A.resid == R_P1 ? dr_shrink1(wr, g * A.mu) : wr / (1.f + 2.f * g * A.mu);
      const float ur = 2.f * zr - wr;
      A.z.r[e] = zr;
      A.u.r[e] = ur;
      v -= ur;
    }
    if (A.z.x0) {
      const float wv = A.w.x0[e];
      const float zv = fmaxf((g * A.src[e] + A.rho * wv) / (A.rho + g), 0.f);
      const float uv = 2.f * zv - wv;
      A.z.x0[e] = zv;
      A.u.x0[e] = uv;
      v -= uv;
    }
    if (A.z.x1) {
      const float wv = A.w.x1[e];
      const float zv = fmaxf((g * A.dst[e] + A.rho * wv) / (A.rho + g), 0.f);
      const float uv = 2.f * zv - wv;
      A.z.x1[e] = zv;
      A.u.x1[e] = uv;
      v += uv;
    }
    if (A.mode == 0) v += A.dst[e] - A.src[e];
    if (A.mode == 2) v -= A.src[e];
    out[e] = v;
  }
}

// e = K u - b: D M_u - x0_u + x1_u - r_u, minus b (DIST: b = p - q, so
// + (q - p); PROX_FIXED: b = s).  With ka set the same for z, summed as
// ||K z - b||^2 into partial[block] (the feasibility of the output).
__global__ __launch_bounds__(DB) void dr_rhs_kernel(DrArgs A, int of_z, float* out, double* partial) {
  __shared__ double red[DB / 64];
  const Planes& V = of_z ? A.z : A.u;
  const int nx = A.nx, ny = A.ny;
  const long n = (long)nx * ny;
  double acc = 0.0;
  for (long e = blockIdx.x * (long)DB + threadIdx.x; e < n; e += (long)gridDim.x * DB) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    float v = (V.Mx[e] - (i > 0 ? V.Mx[e - 1] : 0.f)) + (V.My[e] - (j > 0 ? V.My[e - nx] : 0.f));
    if (V.r) v -= V.r[e];
    if (V.x0) v -= V.x0[e];
    if (V.x1) v += V.x1[e];
    if (A.mode == 0) v += A.dst[e] - A.src[e];
    if (A.mode == 2) v -= A.src[e];
    if (out) out[e] = v;
    acc += (double)v * v;
  }
  if (partial) {
    const double t = dr_block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// y = u - K^T phi, w <- w + (y - z); on record, partial[3 block + 0..1] =
// ||y - z||^2, ||z||^2.
__global__ __launch_bounds__(DB) void dr_update_kernel(DrArgs A, const float* phi, int record, double* partial) {
  __shared__ double red[DB / 64];
  const int nx = A.nx, ny = A.ny;
  const long n = (long)nx * ny;
  double d2 = 0.0, z2 = 0.0;
  for (long e = blockIdx.x * (long)DB + threadIdx.x; e < n; e += (long)gridDim.x * DB) {
    const int j = (int)(e / nx), i = (int)(e - (long)j * nx);
    const float ph = phi[e];
    const float gx = i < nx - 1 ? ph - phi[e + 1] : 0.f;  // (D* phi), zero on the zero-flux edges
    const float gy = j < ny - 1 ? ph - phi[e + nx] : 0.f;
    auto step = [&](float y, float z, float* w) {
      const float st = y - z;
      w[e] = w[e] + st;
      if (record) {
        d2 += (double)st * st;
        z2 += (double)z * z;
      }
    };
    step(A.u.Mx[e] - gx, A.z.Mx[e], A.w.Mx);
    step(A.u.My[e] - gy, A.z.My[e], A.w.My);
    if (A.z.r) step(A.u.r[e] + ph, A.z.r[e], A.w.r);
    if (A.z.x0) step(A.u.x0[e] + ph, A.z.x0[e], A.w.x0);
    if (A.z.x1) step(A.u.x1[e] - ph, A.z.x1[e], A.w.x1);
  }
  if (record) {
    const double a = dr_block_sum(d2, red);
    const double b = dr_block_sum(z2, red);
    if (threadIdx.x == 0) {
      partial[2 * blockIdx.x] = a;
      partial[2 * blockIdx.x + 1] = b;
    }
  }
}

// partial[3 block + 0..2] = flux norm, residual penalty, quadratic of z.
__global__ __launch_bounds__(DB) void dr_objective_kernel(DrArgs A, double* partial) {
  __shared__ double red[DB / 64];
  const long n = (long)A.nx * A.ny;
  double fm = 0.0, pen = 0.0, quad = 0.0;
  for (long e = blockIdx.x * (long)DB + threadIdx.x; e < n; e += (long)gridDim.x * DB) {
    const float mx = A.z.Mx[e], my = A.z.My[e];
    fm += A.aniso ? fabsf(mx) + fabsf(my) : sqrtf(mx * mx + my * my);
    if (A.z.r) {
      const float r = A.z.r[e];
      pen += A.resid == R_P1 ? fabsf(r) : (double)r * r;
    }
    if (A.z.x0) {
      const float d = A.z.x0[e] - A.src[e];
      quad += (double)d * d;
    }
    if (A.z.x1) {
      const float d = A.z.x1[e] - A.dst[e];
      quad += (double)d * d;
    }
  }
  const double a = dr_block_sum(fm, red);
  const double b = dr_block_sum(pen, red);
  const double c = dr_block_sum(quad, red);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = a;
    partial[3 * blockIdx.x + 1] = b;
    partial[3 * blockIdx.x + 2] = c;
  }
}

int dr_blocks(long n) { return (int)std::min<long>(DR_MAX_BLOCKS, std::max<long>(1, (n + DB - 1) / DB)); }

hipError_t launch_dr_prox_rhs(const DrArgs& a, float* out, hipStream_t s) {
  hipLaunchKernelGGL(dr_prox_rhs_kernel, dim3(dr_blocks((long)a.nx * a.ny)), dim3(DB), 0, s, a, out);
  return hipGetLastError();
}

hipError_t launch_dr_rhs(const DrArgs& a, int of_z, float* out, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(dr_rhs_kernel, dim3(dr_blocks((long)a.nx * a.ny)), dim3(DB), 0, s, a, of_z, out, partial);
  return hipGetLastError();
}

hipError_t launch_dr_update(const DrArgs& a, const float* phi, int record, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(dr_update_kernel, dim3(dr_blocks((long)a.nx * a.ny)), dim3(DB), 0, s, a, phi, record,
                     partial);
  return hipGetLastError();
}

hipError_t launch_dr_objective(const DrArgs& a, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(dr_objective_kernel, dim3(dr_blocks((long)a.nx * a.ny)), dim3(DB), 0, s, a, partial);
  return hipGetLastError();
}

}  // namespace uot
