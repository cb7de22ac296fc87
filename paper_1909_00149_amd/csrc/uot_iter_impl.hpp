// HIP kernels (gfx950) of the unbalanced Beckmann OT prox solver.
//
// cp_iter: one fused pass of Algorithm 1 (Sec. III-B) per launch:
//   M  <- group-shrink_{tau1}(M - tau1 D* a)          (eq. Prox_UOT_M_prox;
//         component shrink for the anisotropic l1,1 flux norm)
//   x  <- max(theta p + (1-theta)(x - tau1 A^T a), 0)   (PROX modes)
//   r  <- shrink_{mu tau1}(r + tau1 a)  |  (r + tau1 a)/(1 + 2 mu tau1)
//   a  <- a + tau2 (2 K(z_new) - K(z_old)),   K(z) = D M - x0 + x1 - r
// A workgroup owns a 64 x TY tile.  a^k is staged in LDS with a one-pixel
// halo on every side, the old flux with a halo on the low sides; the new
// flux is computed for the tile plus its low-side halo (so D M_new needs no
// second launch), then each pixel forms K_old, K_new and the dual step.
// Input and output states are different buffers (ping-pong), so no pixel
// reads a value another workgroup may already have overwritten.
//
// The tile list is walked by a fixed grid; blocks are mapped so that each
// of the 8 XCDs (which own separate L2 caches and receive workgroups
// round-robin) walks one contiguous eighth of the list, keeping vertically
// neighbouring tiles, which share halo rows, in one L2.
#pragma once

#include "uot_internal.hpp"

#include <cmath>
#include <type_traits>

namespace uot {

namespace {

// Soft threshold sign(v) max(|v| - s, 0), s >= 0, as v minus its clamp to
// [-s, s]: the same rounding (v - s, v + s or exactly 0), two instructions.
__device__ __forceinline__ float shrink1f(float v, float s) {
  return v - __builtin_amdgcn_fmed3f(v, -s, s);
}

// Prox of tau1 times the flux norm at v = (vx, vy) of one pixel: the group
// shrink of the l2,1 norm (the paper's), or with bit 1 of the boundary code
// set, the component shrink of the anisotropic l1,1 norm.
template <int BC>
__device__ __forceinline__ void flux_shrink(float vx, float vy, float tau1, float& ox, float& oy) {
  if (BC & 2) {
    ox = shrink1f(vx, tau1);
    oy = shrink1f(vy, tau1);
  } else {
    // max(1 - tau1 / ||v||, 0) v; at v = 0 the reciprocal square root is
    // +inf and the factor is 0.  The hardware reciprocal square root
    // without the rescaling of subnormal arguments: it gives the same bits
    // for every normal ||v||^2, and for a subnormal one (||v|| < 1.1e-19,
    // far below any step tau1) the factor is 0 either way.
    const float n2 = vx * vx + vy * vy;
    const float s = fmaxf(1.f - tau1 * __builtin_amdgcn_rsqf(n2), 0.f);
    ox = s * vx;
    oy = s * vy;
  }
}

template <int MODE>
__device__ __forceinline__ constexpr int n_id_blocks(int resid) {
  return (MODE == 0 ? 1 : (MODE == 1 ? 3 : 2)) - (resid == R_BAL ? 1 : 0);
}

// Chunked, XCD-aware walk of the tile list: returns the range of list
// indices this block visits as (first, stride, end).
__device__ __forceinline__ void xcd_chunk(int ntiles, long& first, long& stride, long& end) {
  const int G = gridDim.x;              // multiple of 8
  const int xcd = blockIdx.x & 7;
  const int slot = blockIdx.x >> 3;
  const int per = (G - xcd + 7) >> 3;  // blocks on this XCD
  const long cb = (long)ntiles * xcd / 8;
  end = (long)ntiles * (xcd + 1) / 8;
  first = cb + slot;
  stride = per;
}

}  // namespace

template <int MODE, int RES, int BC, int TY>
__global__ __launch_bounds__(BLOCK) void cp_iter_kernel(IterArgs A) {
  constexpr int PPT = TY / 4;
  __shared__ float sa[TY + 2][TX + 2];
  __shared__ float smx[TY + 1][TX + 1];
  __shared__ float smy[TY + 1][TX + 1];
  __shared__ float snx[TY + 1][TX + 1];
  __shared__ float sny[TY + 1][TX + 1];

  const int tid = threadIdx.x;
  const int lx = tid & 63;
  const int wv = tid >> 6;
  long t, stride, tend;
  xcd_chunk(*A.ntiles, t, stride, tend);

  for (; t < tend; t += stride) {
    const Tile tl = A.tiles[t];
    if (!A.active[tl.pair]) continue;  // uniform over the block
    const PairInfo P = A.pairs[tl.pair];
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const int gx0 = tl.x0, gy0 = tl.y0;
    const long off = P.off;
    const float tau1 = P.tau1, tau2 = P.tau2;

    __syncthreads();  // LDS of the previous tile is no longer read

    // ---- stage a^k (rows -1..TY, cols -1..TX) and old M (low halo) ----
    const float* __restrict__ a_in = A.in.a + off;
    for (int idx = tid; idx < (TY + 2) * (TX + 2); idx += BLOCK) {
      const int ry = idx / (TX + 2), rx = idx - ry * (TX + 2);
      const int gx = gx0 - 1 + rx, gy = gy0 - 1 + ry;
      float v = 0.f;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) v = a_in[(long)gy * pitch + gx];
      sa[ry][rx] = v;
    }
    const float* __restrict__ mx_in = A.in.Mx + off;
    const float* __restrict__ my_in = A.in.My + off;
    for (int idx = tid; idx < (TY + 1) * (TX + 1); idx += BLOCK) {
      const int ry = idx / (TX + 1), rx = idx - ry * (TX + 1);
      const int gx = gx0 - 1 + rx, gy = gy0 - 1 + ry;
      float vx = 0.f, vy = 0.f;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        const long o = (long)gy * pitch + gx;
        vx = mx_in[o];
        vy = my_in[o];
        if ((BC & 1) == 0) {
          if (gx == nx - 1) vx = 0.f;
          if (gy == ny - 1) vy = 0.f;
        }
      }
      smx[ry][rx] = vx;
      smy[ry][rx] = vy;
    }
    // own pixels: element-wise planes straight to registers
    float r_o[PPT], c0[PPT], c1[PPT], x0_o[PPT], x1_o[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int gx = gx0 + lx, gy = gy0 + wv + 4 * k;
      r_o[k] = c0[k] = c1[k] = x0_o[k] = x1_o[k] = 0.f;
      if (gx < nx && gy < ny) {
        const long o = off + (long)gy * pitch + gx;
        if (RES != R_BAL) r_o[k] = A.in.r[o];
        if (MODE == 0) {
          c0[k] = A.c[o];
        } else {
          c0[k] = A.src[o];
          c1[k] = A.dst[o];
          if (MODE == 1) x0_o[k] = A.in.x0[o];
          x1_o[k] = A.in.x1[o];
        }
      }
    }
    __syncthreads();

    // ---- new flux over the tile and its low-side halo ----
    for (int idx = tid; idx < (TY + 1) * (TX + 1); idx += BLOCK) {
      const int ry = idx / (TX + 1), rx = idx - ry * (TX + 1);
      const int gx = gx0 - 1 + rx, gy = gy0 - 1 + ry;
      float nxv = 0.f, nyv = 0.f;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        const float ac = sa[ry][rx];
        float gxx = ac - sa[ry][rx + 1];
        float gyy = ac - sa[ry + 1][rx];
        if ((BC & 1) == 0) {
          if (gx == nx - 1) gxx = 0.f;
          if (gy == ny - 1) gyy = 0.f;
        }
        const float vx = smx[ry][rx] - tau1 * gxx;
        const float vy = smy[ry][rx] - tau1 * gyy;
        flux_shrink<BC>(vx, vy, tau1, nxv, nyv);
      }
      snx[ry][rx] = nxv;
      sny[ry][rx] = nyv;
    }
    __syncthreads();

    // ---- element-wise steps and the dual update ----
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int ly = wv + 4 * k;
      const int gx = gx0 + lx, gy = gy0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const int ry = ly + 1, rx = lx + 1;
      const float dmn = snx[ry][rx] - snx[ry][rx - 1] + sny[ry][rx] - sny[ry - 1][rx];
      const float dmo = smx[ry][rx] - smx[ry][rx - 1] + smy[ry][rx] - smy[ry - 1][rx];
      const float a = sa[ry][rx];
      float kold, knew;
      float x0n = 0.f, x1n = 0.f, rn = 0.f;
      if (RES == R_P1) rn = shrink1f(r_o[k] + tau1 * a, P.mutau);
      if (RES == R_P2) rn = (r_o[k] + tau1 * a) * P.inv2mt;
      if (MODE == 0) {
        kold = dmo + c0[k];
        knew = dmn + c0[k];
      } else if (MODE == 1) {
        const float th = P.theta;
        x0n = fmaxf(th * c0[k] + (1.f - th) * (x0_o[k] + tau1 * a), 0.f);
        x1n = fmaxf(th * c1[k] + (1.f - th) * (x1_o[k] - tau1 * a), 0.f);
        kold = dmo - x0_o[k] + x1_o[k];
        knew = dmn - x0n + x1n;
      } else {
        const float th = P.theta;
        x1n = fmaxf(th * c1[k] + (1.f - th) * (x1_o[k] - tau1 * a), 0.f);
        kold = dmo - c0[k] + x1_o[k];
        knew = dmn - c0[k] + x1n;
      }
      if (RES != R_BAL) {
        kold -= r_o[k];
        knew -= rn;
      }
      const float an = a + tau2 * (2.f * knew - kold);
      const long o = off + (long)gy * pitch + gx;
      A.out.Mx[o] = snx[ry][rx];
      A.out.My[o] = sny[ry][rx];
      A.out.a[o] = an;
      if (RES != R_BAL) A.out.r[o] = rn;
      if (MODE == 1) A.out.x0[o] = x0n;
      if (MODE != 0) A.out.x1[o] = x1n;
    }
  }
}

// Vectorised form of cp_iter_kernel: 16 threads per row, each owning 4
// consecutive pixels (a quad), so every global access of the tile body is
// one 16-byte load or store.  Rows need not start on a 16-byte boundary:
// the accesses only need 4-byte alignment, which the memory system serves
// at full width.  A quad that runs past the end of its row (nx not a
// multiple of 4) is read and written pixel by pixel, so nothing outside the
// pair's rows is touched.  LDS rows keep the tile body 16-byte aligned at
// column 4 (x = 0) with the left halo at column 3 (x = -1) and, for a, the
// right halo at column 68 (x = 64).  The arithmetic per pixel is that of
// cp_iter_kernel.
//
// NT: the outputs are written with non-temporal stores, which pays once the
// state no longer fits the Infinity Cache (measured: about +5% at 4096^2 and
// 8192^2, -15% at 2048^2).  Issuing the next tile's loads before computing
// the current one was measured too and brought nothing.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

// Quad load: n = number of the 4 pixels inside the row (>= 4: all); pixels
// past the row end read as 0 and are never dereferenced.
__device__ __forceinline__ float4 ld4(const float* p, int n) {
  if (n >= 4) {
    const f32x4u v = *reinterpret_cast<const f32x4u*>(p);
    return make_float4(v.x, v.y, v.z, v.w);
  }
  float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
  if (n > 0) r.x = p[0];
  if (n > 1) r.y = p[1];
  if (n > 2) r.z = p[2];
  return r;
}

// Sets component j (0..3) of v to zero; no-op for other j.
__device__ __forceinline__ void zero_at(float4& v, int j) {
  if (j == 0) v.x = 0.f;
  if (j == 1) v.y = 0.f;
  if (j == 2) v.z = 0.f;
  if (j == 3) v.w = 0.f;
}

template <int MODE, int RES, int BC, int TY>
struct VecStage {
  static constexpr int NA = (TY + 2 + 15) / 16, NM = (TY + 1 + 15) / 16, PR = TY / 16;
  float4 a[NA], mx[NM], my[NM];
  float ha, hmx, hmy;
  float4 r[PR], c0[PR], c1[PR], x0[PR], x1[PR];
};

template <int MODE, int RES, int BC, int TY>
__device__ __forceinline__ void vec_fetch(const IterArgs& A, const PairInfo& P, const Tile& tl,
                                          VecStage<MODE, RES, BC, TY>& S) {
  using St = VecStage<MODE, RES, BC, TY>;
  const int tid = threadIdx.x, q = tid & 15, rr = tid >> 4;
  const int nx = P.nx, ny = P.ny, pitch = P.pitch, gx0 = tl.x0, gy0 = tl.y0;
  const long off = P.off;
  const int gxq = gx0 + 4 * q;
  const int nin = nx - gxq;  // pixels of this quad inside the row (>= 4: all)
  const bool quad_in = nin > 0;
  const float* __restrict__ a_in = A.in.a + off;
  const float* __restrict__ mx_in = A.in.Mx + off;
  const float* __restrict__ my_in = A.in.My + off;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int i = 0; i < St::NA; ++i) {
    const int ry = rr + 16 * i, gy = gy0 - 1 + ry;
    S.a[i] = z;
    if (ry < TY + 2 && gy >= 0 && gy < ny && quad_in) S.a[i] = ld4(a_in + (long)gy * pitch + gxq, nin);
  }
#pragma unroll
  for (int i = 0; i < St::NM; ++i) {
    const int ry = rr + 16 * i, gy = gy0 - 1 + ry;
    S.mx[i] = S.my[i] = z;
    if (ry < TY + 1 && gy >= 0 && gy < ny && quad_in) {
      const long o = (long)gy * pitch + gxq;
      S.mx[i] = ld4(mx_in + o, nin);
      S.my[i] = ld4(my_in + o, nin);
      if ((BC & 1) == 0) {
        zero_at(S.mx[i], nx - 1 - gxq);
        if (gy == ny - 1) S.my[i] = z;
      }
    }
  }
  S.ha = S.hmx = S.hmy = 0.f;
  if (tid < 2 * (TY + 2)) {  // halo columns of a: x = -1 and x = 64
    const int ry = tid >> 1, side = tid & 1;
    const int gx = side ? gx0 + 64 : gx0 - 1, gy = gy0 - 1 + ry;
    if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) S.ha = a_in[(long)gy * pitch + gx];
  } else if (tid >= 128 && tid < 128 + TY + 1) {  // halo column of M: x = -1
    const int ry = tid - 128, gx = gx0 - 1, gy = gy0 - 1 + ry;
    if (gx >= 0 && gy >= 0 && gy < ny) {
      const long o = (long)gy * pitch + gx;
      S.hmx = mx_in[o];  // gx < nx - 1 here: never the structurally zero column
      S.hmy = ((BC & 1) == 0 && gy == ny - 1) ? 0.f : my_in[o];
    }
  }
#pragma unroll
  for (int k = 0; k < St::PR; ++k) {
    const int gy = gy0 + rr + 16 * k;
    S.r[k] = S.c0[k] = S.c1[k] = S.x0[k] = S.x1[k] = z;
    if (quad_in && gy < ny) {
      const long o = off + (long)gy * pitch + gxq;
      if (RES != R_BAL) S.r[k] = ld4(A.in.r + o, nin);
      if (MODE == 0) {
        S.c0[k] = ld4(A.c + o, nin);
      } else {
        S.c0[k] = ld4(A.src + o, nin);
        S.c1[k] = ld4(A.dst + o, nin);
        if (MODE == 1) S.x0[k] = ld4(A.in.x0 + o, nin);
        S.x1[k] = ld4(A.in.x1 + o, nin);
      }
    }
  }
}

// Quad store of the first n (>= 4: all) pixels of v.
template <bool NT>
__device__ __forceinline__ void st4(float* p, float4 v, int n) {
  if (n >= 4) {
    const f32x4u w = {v.x, v.y, v.z, v.w};
    if (NT)
      __builtin_nontemporal_store(w, reinterpret_cast<f32x4u*>(p));
    else
      *reinterpret_cast<f32x4u*>(p) = w;
    return;
  }
  if (n > 0) p[0] = v.x;
  if (n > 1) p[1] = v.y;
  if (n > 2) p[2] = v.z;
}

template <int MODE, int RES, int BC, int TY, bool NT>
__global__ __launch_bounds__(BLOCK) void cp_iter_vec_kernel(IterArgs A) {
  static_assert(TY % 16 == 0, "16 rows per pass");
  using St = VecStage<MODE, RES, BC, TY>;
  constexpr int LA = 72, LM = 68, PR = St::PR;
  __shared__ __attribute__((aligned(16))) float sa[TY + 2][LA];
  __shared__ __attribute__((aligned(16))) float smx[TY + 1][LM];
  __shared__ __attribute__((aligned(16))) float smy[TY + 1][LM];
  __shared__ __attribute__((aligned(16))) float snx[TY + 1][LM];
  __shared__ __attribute__((aligned(16))) float sny[TY + 1][LM];
  const int tid = threadIdx.x;
  const int q = tid & 15, rr = tid >> 4;
  long t, stride, tend;
  xcd_chunk(*A.ntiles, t, stride, tend);

  St cur;
  for (; t < tend; t += stride) {
    const Tile tl = A.tiles[t];
    if (!A.active[tl.pair]) continue;  // uniform over the block
    const PairInfo P = A.pairs[tl.pair];
    vec_fetch<MODE, RES, BC, TY>(A, P, tl, cur);
    {
      const int nx = P.nx, ny = P.ny, pitch = P.pitch;
      const int gx0 = tl.x0, gy0 = tl.y0;
      const long off = P.off;
      const float tau1 = P.tau1, tau2 = P.tau2;
      const int gxq = gx0 + 4 * q;
      const int nin = nx - gxq;
      const bool quad_in = nin > 0;

      __syncthreads();  // LDS of the previous tile is no longer read
#pragma unroll
      for (int i = 0; i < St::NA; ++i)
        if (rr + 16 * i < TY + 2) *reinterpret_cast<float4*>(&sa[rr + 16 * i][4 + 4 * q]) = cur.a[i];
#pragma unroll
      for (int i = 0; i < St::NM; ++i)
        if (rr + 16 * i < TY + 1) {
          *reinterpret_cast<float4*>(&smx[rr + 16 * i][4 + 4 * q]) = cur.mx[i];
          *reinterpret_cast<float4*>(&smy[rr + 16 * i][4 + 4 * q]) = cur.my[i];
        }
      if (tid < 2 * (TY + 2)) {
        sa[tid >> 1][(tid & 1) ? 68 : 3] = cur.ha;
      } else if (tid >= 128 && tid < 128 + TY + 1) {
        smx[tid - 128][3] = cur.hmx;
        smy[tid - 128][3] = cur.hmy;
      }
      __syncthreads();

      // ---- new flux over the tile and its low-side halo ----
      auto shrink = [&](float ac, float ar, float au, float mx, float my, int gx, int gy, float& ox, float& oy) {
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) {
          ox = oy = 0.f;
          return;
        }
        float gxx = ac - ar, gyy = ac - au;
        if ((BC & 1) == 0) {
          if (gx == nx - 1) gxx = 0.f;
          if (gy == ny - 1) gyy = 0.f;
        }
        const float vx = mx - tau1 * gxx;
        const float vy = my - tau1 * gyy;
        flux_shrink<BC>(vx, vy, tau1, ox, oy);
      };
      for (int ry = rr; ry < TY + 1; ry += 16) {
        const int gy = gy0 - 1 + ry;
        const int c = 4 + 4 * q;
        const float4 ac = *reinterpret_cast<const float4*>(&sa[ry][c]);
        const float4 au = *reinterpret_cast<const float4*>(&sa[ry + 1][c]);
        const float ar4 = sa[ry][c + 4];
        const float4 mx = *reinterpret_cast<const float4*>(&smx[ry][c]);
        const float4 my = *reinterpret_cast<const float4*>(&smy[ry][c]);
        float4 ox, oy;
        shrink(ac.x, ac.y, au.x, mx.x, my.x, gxq + 0, gy, ox.x, oy.x);
        shrink(ac.y, ac.z, au.y, mx.y, my.y, gxq + 1, gy, ox.y, oy.y);
        shrink(ac.z, ac.w, au.z, mx.z, my.z, gxq + 2, gy, ox.z, oy.z);
        shrink(ac.w, ar4, au.w, mx.w, my.w, gxq + 3, gy, ox.w, oy.w);
        *reinterpret_cast<float4*>(&snx[ry][c]) = ox;
        *reinterpret_cast<float4*>(&sny[ry][c]) = oy;
      }
      if (tid < TY + 1) {  // halo column x = -1
        const int ry = tid;
        float ox, oy;
        shrink(sa[ry][3], sa[ry][4], sa[ry + 1][3], smx[ry][3], smy[ry][3], gx0 - 1, gy0 - 1 + ry, ox, oy);
        snx[ry][3] = ox;
        sny[ry][3] = oy;
      }
      __syncthreads();

      // ---- element-wise steps and the dual update, 4 pixels per thread ----
#pragma unroll
      for (int k = 0; k < PR; ++k) {
        const int ly = rr + 16 * k;
        const int gy = gy0 + ly;
        if (!quad_in || gy >= ny) continue;
        const int ry = ly + 1, c = 4 + 4 * q;
        const float4 nxc = *reinterpret_cast<const float4*>(&snx[ry][c]);
        const float nxl = snx[ry][c - 1];
        const float4 nyc = *reinterpret_cast<const float4*>(&sny[ry][c]);
        const float4 nyd = *reinterpret_cast<const float4*>(&sny[ry - 1][c]);
        const float4 mxc = *reinterpret_cast<const float4*>(&smx[ry][c]);
        const float mxl = smx[ry][c - 1];
        const float4 myc = *reinterpret_cast<const float4*>(&smy[ry][c]);
        const float4 myd = *reinterpret_cast<const float4*>(&smy[ry - 1][c]);
        const float4 a4 = *reinterpret_cast<const float4*>(&sa[ry][c]);
        const float nxv[5] = {nxl, nxc.x, nxc.y, nxc.z, nxc.w};
        const float mxv[5] = {mxl, mxc.x, mxc.y, mxc.z, mxc.w};
        const float nyv[4] = {nyc.x, nyc.y, nyc.z, nyc.w}, nydv[4] = {nyd.x, nyd.y, nyd.z, nyd.w};
        const float myv[4] = {myc.x, myc.y, myc.z, myc.w}, mydv[4] = {myd.x, myd.y, myd.z, myd.w};
        const float av[4] = {a4.x, a4.y, a4.z, a4.w};
        const float rv[4] = {cur.r[k].x, cur.r[k].y, cur.r[k].z, cur.r[k].w};
        const float c0v[4] = {cur.c0[k].x, cur.c0[k].y, cur.c0[k].z, cur.c0[k].w};
        const float c1v[4] = {cur.c1[k].x, cur.c1[k].y, cur.c1[k].z, cur.c1[k].w};
        const float x0v[4] = {cur.x0[k].x, cur.x0[k].y, cur.x0[k].z, cur.x0[k].w};
        const float x1v[4] = {cur.x1[k].x, cur.x1[k].y, cur.x1[k].z, cur.x1[k].w};
        float an[4], rn[4], x0n[4], x1n[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dmn = nxv[e + 1] - nxv[e] + nyv[e] - nydv[e];
          const float dmo = mxv[e + 1] - mxv[e] + myv[e] - mydv[e];
          const float a = av[e];
          float kold, knew;
          x0n[e] = x1n[e] = rn[e] = 0.f;
          if (RES == R_P1) rn[e] = shrink1f(rv[e] + tau1 * a, P.mutau);
          if (RES == R_P2) rn[e] = (rv[e] + tau1 * a) * P.inv2mt;
          if (MODE == 0) {
            kold = dmo + c0v[e];
            knew = dmn + c0v[e];
          } else if (MODE == 1) {
            const float th = P.theta;
            x0n[e] = fmaxf(th * c0v[e] + (1.f - th) * (x0v[e] + tau1 * a), 0.f);
            x1n[e] = fmaxf(th * c1v[e] + (1.f - th) * (x1v[e] - tau1 * a), 0.f);
            kold = dmo - x0v[e] + x1v[e];
            knew = dmn - x0n[e] + x1n[e];
          } else {
            const float th = P.theta;
            x1n[e] = fmaxf(th * c1v[e] + (1.f - th) * (x1v[e] - tau1 * a), 0.f);
            kold = dmo - c0v[e] + x1v[e];
            knew = dmn - c0v[e] + x1n[e];
          }
          if (RES != R_BAL) {
            kold -= rv[e];
            knew -= rn[e];
          }
          an[e] = a + tau2 * (2.f * knew - kold);
        }
        const long o = off + (long)gy * pitch + gxq;
        st4<NT>(A.out.Mx + o, nxc, nin);
        st4<NT>(A.out.My + o, nyc, nin);
        st4<NT>(A.out.a + o, make_float4(an[0], an[1], an[2], an[3]), nin);
        if (RES != R_BAL) st4<NT>(A.out.r + o, make_float4(rn[0], rn[1], rn[2], rn[3]), nin);
        if (MODE == 1) st4<NT>(A.out.x0 + o, make_float4(x0n[0], x0n[1], x0n[2], x0n[3]), nin);
        if (MODE != 0) st4<NT>(A.out.x1 + o, make_float4(x1n[0], x1n[1], x1n[2], x1n[3]), nin);
      }
    }
  }
}

// Temporally blocked form: one launch runs `steps` (<= T) iterations with
// the per-pixel arithmetic of the kernels above.  A workgroup loads its
// 64 x TH tile with a halo of T pixels on every side (a, Mx, My into LDS, the
// element-wise planes into registers) and repeats the flux phase and the
// dual phase over the whole region.  One iteration couples a pixel only to
// pixels at distance one (D* a looks one pixel up and right, D M one pixel
// down and left, so a^{k+1} depends on a^k within distance one), so after s
// steps every value is exact except within s pixels of the region's edge,
// and a halo of T keeps the owned tile exact for up to T steps.  Pixels
// outside the grid hold zero and are never updated, as in the single-step
// kernels.  K(z^k) of each pixel is carried in a register from one step to
// the next (it is the K(z^{k+1}) of the step before), so the old flux is not
// needed again and the flux is updated in place.  The last iteration before
// a convergence check runs as one step with a halo of two that also
// evaluates the check: the iterate it read is kept in registers, the one it
// wrote is in LDS, and both iterates stay in the ping-pong buffers for the
// final evaluation of a solve.
// ---------------------------------------------------------------------------
// Block reduction of NS double slots into one partial row (and, if fin is
// given, into that LDS row too, visible to the whole block on return),
// through the LDS buffer buf of NS x BLOCK doubles.  Every thread stores its
// NS values; then thread 16 s + g combines values g, g + 16, ... of slot s
// (a pairwise tree; the 16 lanes of a load hit distinct banks), and the 16
// lanes of a slot, consecutive lanes of one wave, combine by an xor
// butterfly.  The order is fixed, so the result does not depend on timing.
// Slots in max_mask are max-reduced, the others summed.
__device__ __forceinline__ void block_reduce_lds(double (&acc)[NS], uint32_t max_mask, double* dst, double* buf,
                                                 double* fin = nullptr) {
  static_assert(NS == 16 && BLOCK == 256, "16 slots x 16 lanes x 16 values");
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < NS; ++s) buf[s * BLOCK + tid] = acc[s];
  __syncthreads();
  const int s = tid >> 4, g = tid & 15;
  const bool mx = (max_mask >> s) & 1u;
  double w[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) w[k] = buf[s * BLOCK + g + 16 * k];
#pragma unroll
  for (int h = 8; h > 0; h >>= 1)
#pragma unroll
    for (int k = 0; k < h; ++k) w[k] = mx ? fmax(w[k], w[k + h]) : w[k] + w[k + h];
  double v = w[0];
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    const double u = __shfl_xor(v, o, 16);
    v = mx ? fmax(v, u) : v + u;
  }
  if (g == 0) {
    dst[s] = v;
    if (fin) fin[s] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ void block_reduce_store(double (&acc)[NS], uint32_t max_mask, double* dst,
                                                   double* fin = nullptr) {
  __shared__ double buf[NS * BLOCK];
  block_reduce_lds(acc, max_mask, dst, buf, fin);
}

// Cell idx (0 <= idx < NC * BLOCK) of a workgroup's region, in region
// coordinates (rx, ry), region cell (0, 0) being grid pixel (x0 - H, y0 - H):
// the owned 64 x TH tile first, row by row, so that each thread's first
// TH / 4 cells are owned and every wave reads and writes whole tile rows;
// then the ring around the tile: the H rows below and the H rows above it
// (full region width), then the H columns left and right of its rows.
// Slots past the region come back with ry = RH and rx numbering them.
template <int TH, int H>
__device__ __forceinline__ void region_cell(int idx, int& rx, int& ry) {
  constexpr int RW = TX + 2 * H;
  constexpr int OWN = TX * TH, BAND = H * RW, SIDE = H * TH;
  if (idx < OWN) {
    ry = H + idx / TX;
    rx = H + idx % TX;
    return;
  }
  int j = idx - OWN;
  if (j < 2 * BAND) {
    const int b = j >= BAND;  // 0 below the tile, 1 above
    j -= b * BAND;
    ry = j / RW + b * (H + TH);
    rx = j % RW;
    return;
  }
  j -= 2 * BAND;
  if (j < 2 * SIDE) {
    const int b = j >= SIDE;  // 0 left of the tile, 1 right
    j -= b * SIDE;
    ry = H + j / H;
    rx = j % H + b * (H + TX);
    return;
  }
  ry = TH + 2 * H;
  rx = j - 2 * SIDE;
}

// A plane's pixels as seen from a tile: `base` is the plane's address of
// region cell (0, 0), uniform over the workgroup, formed in integer
// arithmetic since it may lie before the pair (the region reaches past the
// grid); cells are read and written at 32-bit byte offsets from it, so the
// per-cell address arithmetic stays 32-bit.
struct RegionPlane {
  using gbyte = __attribute__((address_space(1))) char;  // global memory
  gbyte* base;
  __device__ __forceinline__ RegionPlane(const float* p, long rbase)
      : base((gbyte*)((uintptr_t)p + (uintptr_t)(rbase * (long)sizeof(float)))) {}
  __device__ __forceinline__ float ld(unsigned bo) const {
    return *(const __attribute__((address_space(1))) float*)(base + bo);
  }
  __device__ __forceinline__ void st(unsigned bo, float v) const {
    *(__attribute__((address_space(1))) float*)(base + bo) = v;
  }
  // a direct load into LDS: lane i of the wave writes lds[i], lds being
  // the same for the whole wave
  __device__ __forceinline__ void to_lds(unsigned bo, float* lds) const {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(base + bo),
                                     (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
  }
};

// H: the halo, so up to H steps per launch keep the owned tile exact.  CHK:
// the launch also evaluates the convergence check of the iterate pair of its
// last step (steps <= H - 1, so that the new dual is exact one cell beyond
// the tile, where the check reads its right and upper neighbours).  The
// stationarity residual splits into a part of the step's input and output
// values, formed during the last step and kept in registers for the owned
// cells, and the gradient of the new dual, added after it; the feasibility
// residual is the last step's K(z) itself.
template <int MODE, int RES, int BC, int TH, int H, bool CHK>
__device__ __forceinline__ void cp_iter_tb_body(const IterArgs& A) {
  constexpr int RW = TX + 2 * H, RH = TH + 2 * H, NCELL = RW * RH;
  constexpr int NC = (NCELL + BLOCK - 1) / BLOCK;
  constexpr int NOWN = TX * TH / BLOCK;  // owned cells per thread: the first NOWN
  // PERCELL: each phase of a step reads, computes and writes one cell at a
  // time (fewer live registers, so more workgroups per CU: the tall tiles
  // of large grids and batches).  With 4- and 8-row tiles, whose grids are
  // too small to fill more workgroups per CU, every cell's inputs are read
  // first: more loads in flight.  The arithmetic is the same either way.
  constexpr bool PERCELL = TH >= 16;
  static_assert(TX * TH % BLOCK == 0, "whole tile rows per thread");
  static_assert(!CHK || H >= 2, "the check needs one exact cell beyond the tile");
  // LDS: the region's RH rows of RW cells back to back, so that the
  // region in row-major order is one run of LDS words (cell (rx, ry) at
  // (ry + 1) RW + rx + 1), between a zero row below and a zero row above;
  // the slots past the region follow the upper zero row (always zero, read
  // only by themselves).  A cell at the region's left or right edge reads
  // the neighbouring row's end as its neighbour: such cells are never
  // exact, and the owned tile does not depend on them.
  constexpr int PAD = NC * BLOCK - NCELL;
  constexpr int LW = RW;
  constexpr int NCHUNK = (NCELL + 63) / 64;  // 64-cell runs of the region, one per direct load
  constexpr int F_IN = 1, F_ZX = 2, F_ZY = 4, F_PAD = 8;  // per-cell flags
  // a, Mx, My planes of the region
  constexpr int PLANE = (RH + 4) * RW + PAD + 2;
  __shared__ double pool[(3 * PLANE + 1) / 2];
  // CHK: each thread's running sums of the stopping rule's summed terms
  // over its block's run of tiles of one pair, one LDS word per thread and
  // term (slots kSumSlot[0..NSUM)): held in registers across the steps they
  // cost the check variant about 40 VGPRs and a workgroup per CU
  constexpr int NSUM = 3 + (MODE == 1) + (MODE != 0);
  __shared__ double runsum[CHK ? NSUM * BLOCK : 1];
  __shared__ double wsum[CHK ? 4 * (NSUM + 1) : 1];  // per wave: the run's sums and non-finite count
  float* const sa = reinterpret_cast<float*>(pool);
  float* const smx = sa + PLANE;
  float* const smy = sa + 2 * PLANE;
  const int tid = threadIdx.x;
  for (int i = tid; i < PLANE; i += BLOCK) sa[i] = smx[i] = smy[i] = 0.f;
  const int steps = A.steps;
  long t, stride, tend;
  xcd_chunk(*A.ntiles, t, stride, tend);
  // the LDS index of each cell does not depend on the tile
  int l_[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    int rx, ry;
    region_cell<TH, H>(tid + k * BLOCK, rx, ry);
    l_[k] = ry < RH ? (ry + 1) * RW + rx + 1 : (RH + 2) * RW + 1 + rx;
  }
  // CHK: per-thread check sums over the block's run of tiles of one pair
  // (runsum, and the non-finite count), reduced once per run into the row
  // of its first tile (the run's other rows are zeroed, so the per-pair sum
  // of the rows is unchanged).  Only the terms of the stopping rule are
  // accumulated: the report's objective and bounds come from the final
  // evaluation of a solve.
  constexpr int kSumSlot[5] = {S_PRES2, S_STAT2, S_KA2, MODE == 1 ? S_X0SQ : S_X1SQ, S_X1SQ};
  int nonfin = 0;
  int run_pair = -1, run_row = 0;
  // the run's sums reduced over the block into the row of partials of its
  // first tile, and set back to zero: an xor butterfly within each wave
  // (every lane ends with the same bits), then the four waves' values in a
  // fixed order; the slots the check does not sum are written as zero.
  // Runs are short on batches of small pairs (a workgroup's consecutive
  // tiles lie a grid's width apart in the tile list), so the reduction
  // leaves the region planes alone and costs one barrier.
  auto flush_run = [&]() {
    double v[NSUM + 1];
#pragma unroll
    for (int q = 0; q < NSUM; ++q) {
      v[q] = runsum[q * BLOCK + tid];
      runsum[q * BLOCK + tid] = 0.0;
    }
    v[NSUM] = (double)nonfin;
    nonfin = 0;
#pragma unroll
    for (int q = 0; q <= NSUM; ++q)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if ((tid & 63) == 0) {
#pragma unroll
      for (int q = 0; q <= NSUM; ++q) wsum[(tid >> 6) * (NSUM + 1) + q] = v[q];
    }
    __syncthreads();
    if (tid < NS) {
      int q = tid == S_NONFIN ? NSUM : -1;
#pragma unroll
      for (int j = 0; j < NSUM; ++j)
        if (kSumSlot[j] == tid) q = j;
      double sum = 0.0;
      if (q >= 0)
        sum = (wsum[q] + wsum[(NSUM + 1) + q]) + (wsum[2 * (NSUM + 1) + q] + wsum[3 * (NSUM + 1) + q]);
      A.chk[(long)run_row * NS + tid] = sum;
    }
  };
  if (CHK) {
#pragma unroll
    for (int q = 0; q < NSUM; ++q) runsum[q * BLOCK + tid] = 0.0;
  }

  // the next tile's record is loaded while this one computes; its flag and
  // pair record are then loaded together
  Tile tl_n{};
  if (t < tend) tl_n = A.tiles[t];
  for (; t < tend; t += stride) {
    const Tile tl = tl_n;
    const int act = A.active[tl.pair];
    const PairInfo P = A.pairs[tl.pair];
    if (t + stride < tend) tl_n = A.tiles[t + stride];
    if (!act) continue;  // uniform over the block
    if (CHK) {
      if (tl.pair != run_pair) {
        if (run_pair >= 0) flush_run();
        run_pair = tl.pair;
        run_row = tl.pad;
      } else if (tid < NS) {
        A.chk[(long)tl.pad * NS + tid] = 0.0;
      }
    }
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const long off = P.off;
    const float tau1 = P.tau1, tau2 = P.tau2;
    const float it1 = 1.f / tau1;
    const int bx = tl.x0 - H, by = tl.y0 - H;  // grid position of region cell (0, 0)
    int f_[NC];                                // flags of each cell
    float r_[NC], c0_[NC], c1_[NC], x0_[NC], x1_[NC], kp_[NC];
    // CHK: the parts of the stationarity residual that the last step forms
    // from its input and output values, per owned cell: flux (x, y), r, x0,
    // x1; the new dual's gradient (and the new dual) complete them
    float kpx_[NOWN], kpy_[NOWN], kpr_[NOWN], kp0_[NOWN], kp1_[NOWN];

    // the planes from region cell (0, 0); byte offsets of region cells are
    // below 4 GiB because the host runs blocked shapes only for pitches
    // that keep (RH + 1) rows under it
    const long rbase = off + (long)by * pitch + bx;
    const RegionPlane pa(A.in.a, rbase), pmx(A.in.Mx, rbase), pmy(A.in.My, rbase), pr(A.in.r, rbase);
    const RegionPlane pc(MODE == 0 ? A.c : A.src, rbase), pd(A.dst, rbase), px0(A.in.x0, rbase),
        px1(A.in.x1, rbase);

    __syncthreads();  // LDS of the previous tile is no longer read
    // ---- stage the region.  The a, Mx and My planes go to LDS by direct
    // loads, each wave instruction filling a run of 64 region cells; the
    // element-wise planes go to registers.  Every load is issued before any
    // value is used.  A cell outside the grid loads the nearest pixel of
    // the pair (always valid) and is set to zero afterwards. ----
    {
      const int lane = tid & 63;
      for (int j = tid >> 6; j < NCHUNK; j += BLOCK / 64) {
        const int f = j * 64 + lane;
        if (f < NCELL) {
          const int ry = f / RW, rx = f - ry * RW;
          const int cx = min(max(bx + rx, 0), nx - 1), cy = min(max(by + ry, 0), ny - 1);
          const unsigned bo = ((unsigned)(cy - by) * (unsigned)pitch + (unsigned)(cx - bx)) * 4u;
          const int l0 = RW + 1 + j * 64;  // the run's first LDS word (uniform over the wave)
          pa.to_lds(bo, sa + l0);
          pmx.to_lds(bo, smx + l0);
          pmy.to_lds(bo, smy + l0);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      int rx, ry;
      region_cell<TH, H>(tid + k * BLOCK, rx, ry);
      const int gx = bx + rx, gy = by + ry;
      const bool in = ry < RH && (unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny;
      f_[k] = (in ? F_IN : 0) | ((BC & 1) == 0 && gx == nx - 1 ? F_ZX : 0) |
              ((BC & 1) == 0 && gy == ny - 1 ? F_ZY : 0) | (ry >= RH ? F_PAD : 0);
      const int cx = min(max(gx, 0), nx - 1), cy = min(max(gy, 0), ny - 1);
      const unsigned bo = ((unsigned)(cy - by) * (unsigned)pitch + (unsigned)(cx - bx)) * 4u;
      r_[k] = RES != R_BAL ? pr.ld(bo) : 0.f;
      if (MODE == 0) {
        c0_[k] = pc.ld(bo);
        c1_[k] = x0_[k] = x1_[k] = 0.f;
      } else {
        c0_[k] = pc.ld(bo);
        c1_[k] = pd.ld(bo);
        x0_[k] = MODE == 1 ? px0.ld(bo) : 0.f;
        x1_[k] = px1.ld(bo);
      }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (!(f_[k] & F_IN)) r_[k] = c0_[k] = c1_[k] = x0_[k] = x1_[k] = 0.f;
      if (f_[k] & F_PAD) {  // slots past the region: no direct load writes them
        const int l = l_[k];
        sa[l] = smx[l] = smy[l] = 0.f;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's direct loads have reached LDS
    __syncthreads();
    // a region reaching past the grid or holding zero-flux cells: the cells
    // outside the grid are zero, and so is the flux through those edges
    const bool interior = bx >= 0 && by >= 0 && bx + RW <= nx - 1 && by + RH <= ny - 1;
    if (!interior) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int l = l_[k];
        const int fl = f_[k];
        if (!(fl & F_IN)) {
          sa[l] = smx[l] = smy[l] = 0.f;
        } else {
          if (fl & F_ZX) smx[l] = 0.f;
          if (fl & F_ZY) smy[l] = 0.f;
        }
      }
      __syncthreads();
    }

    // ---- K(z^k) of every cell ----
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int l = l_[k];
      const float dmo = smx[l] - smx[l - 1] + smy[l] - smy[l - LW];
      float kold;
      if (MODE == 0) kold = dmo + c0_[k];
      else if (MODE == 1) kold = dmo - x0_[k] + x1_[k];
      else kold = dmo - c0_[k] + x1_[k];
      if (RES != R_BAL) kold -= r_[k];
      kp_[k] = kold;
    }
    __syncthreads();  // the flux phase overwrites M, which the neighbours read above

    // one step over the region; KEEPSTEP: the step whose input iterate the
    // check compares with (the last), which keeps the owned cells' inputs
    // MASK: the region reaches past the grid or holds zero-flux cells, so
    // the cells outside the grid are held at zero and the flux through the
    // zero-flux edges at zero; without it (a region wholly inside the grid,
    // away from those edges) the selects are no-ops and are left out
    auto one_step = [&](auto keep_tag, auto mask_tag) {
      constexpr bool KEEPSTEP = decltype(keep_tag)::value;
      constexpr bool MASK = decltype(mask_tag)::value;
      if constexpr (PERCELL) {
        // ---- new flux.  A cell reads the dual at itself and its right and
        // upper neighbours and its own flux, and writes only its own flux,
        // which no other cell reads in this phase: each cell is read,
        // computed and written in turn ----
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int l = l_[k];
          const float ac = sa[l], ar = sa[l + 1], au = sa[l + LW], mx = smx[l], my = smy[l];
          float gxx = ac - ar;
          float gyy = ac - au;
          if ((BC & 1) == 0 && MASK) {
            if (f_[k] & F_ZX) gxx = 0.f;
            if (f_[k] & F_ZY) gyy = 0.f;
          }
          const float vx = mx - tau1 * gxx;
          const float vy = my - tau1 * gyy;
          float ox, oy;
          flux_shrink<BC>(vx, vy, tau1, ox, oy);
          if (KEEPSTEP && k < NOWN) {
            kpx_[k] = (mx - ox) * it1 - gxx;
            kpy_[k] = (my - oy) * it1 - gyy;
          }
          const bool in = !MASK || (f_[k] & F_IN);
          smx[l] = in ? ox : 0.f;
          smy[l] = in ? oy : 0.f;
        }
        __syncthreads();
        // ---- element-wise steps and the dual update.  A cell reads the new
        // flux at itself and its left and lower neighbours and its own dual,
        // and writes only its own dual ----
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int l = l_[k];
          const float dmn = smx[l] - smx[l - 1] + smy[l] - smy[l - LW];
          const float a = sa[l];
          float knew, x0n = 0.f, x1n = 0.f, rn = 0.f;
          if (RES == R_P1) rn = shrink1f(r_[k] + tau1 * a, P.mutau);
          if (RES == R_P2) rn = (r_[k] + tau1 * a) * P.inv2mt;
          if (MODE == 0) {
            knew = dmn + c0_[k];
          } else if (MODE == 1) {
            const float th = P.theta;
            x0n = fmaxf(th * c0_[k] + (1.f - th) * (x0_[k] + tau1 * a), 0.f);
            x1n = fmaxf(th * c1_[k] + (1.f - th) * (x1_[k] - tau1 * a), 0.f);
            knew = dmn - x0n + x1n;
          } else {
            const float th = P.theta;
            x1n = fmaxf(th * c1_[k] + (1.f - th) * (x1_[k] - tau1 * a), 0.f);
            knew = dmn - c0_[k] + x1n;
          }
          if (RES != R_BAL) knew -= rn;
          if (KEEPSTEP && k < NOWN) {
            if (RES != R_BAL) kpr_[k] = (r_[k] - rn) * it1 + a;
            if (MODE == 1) kp0_[k] = (x0_[k] - x0n) * it1 + a;
            if (MODE != 0) kp1_[k] = (x1_[k] - x1n) * it1 - a;
          }
          const bool in = !MASK || (f_[k] & F_IN);
          sa[l] = in ? a + tau2 * (2.f * knew - kp_[k]) : 0.f;
          kp_[k] = knew;
          r_[k] = rn;
          x0_[k] = x0n;
          x1_[k] = x1n;
        }
      } else {
        // ---- new flux: read every cell's inputs, then compute and write ----
        float ac_[NC], ar_[NC], au_[NC], mx_[NC], my_[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int l = l_[k];
          ac_[k] = sa[l];
          ar_[k] = sa[l + 1];
          au_[k] = sa[l + LW];
          mx_[k] = smx[l];
          my_[k] = smy[l];
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          float gxx = ac_[k] - ar_[k];
          float gyy = ac_[k] - au_[k];
          if ((BC & 1) == 0 && MASK) {
            if (f_[k] & F_ZX) gxx = 0.f;
            if (f_[k] & F_ZY) gyy = 0.f;
          }
          const float vx = mx_[k] - tau1 * gxx;
          const float vy = my_[k] - tau1 * gyy;
          float ox, oy;
          flux_shrink<BC>(vx, vy, tau1, ox, oy);
          if (KEEPSTEP && k < NOWN) {
            kpx_[k] = (mx_[k] - ox) * it1 - gxx;
            kpy_[k] = (my_[k] - oy) * it1 - gyy;
          }
          const bool in = !MASK || (f_[k] & F_IN);
          smx[l_[k]] = in ? ox : 0.f;
          smy[l_[k]] = in ? oy : 0.f;
        }
        __syncthreads();
        // ---- element-wise steps and the dual update ----
        float nc_[NC], nl_[NC], yc_[NC], yd_[NC], a_[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int l = l_[k];
          nc_[k] = smx[l];
          nl_[k] = smx[l - 1];
          yc_[k] = smy[l];
          yd_[k] = smy[l - LW];
          a_[k] = sa[l];
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const float dmn = nc_[k] - nl_[k] + yc_[k] - yd_[k];
          const float a = a_[k];
          float knew, x0n = 0.f, x1n = 0.f, rn = 0.f;
          if (RES == R_P1) rn = shrink1f(r_[k] + tau1 * a, P.mutau);
          if (RES == R_P2) rn = (r_[k] + tau1 * a) * P.inv2mt;
          if (MODE == 0) {
            knew = dmn + c0_[k];
          } else if (MODE == 1) {
            const float th = P.theta;
            x0n = fmaxf(th * c0_[k] + (1.f - th) * (x0_[k] + tau1 * a), 0.f);
            x1n = fmaxf(th * c1_[k] + (1.f - th) * (x1_[k] - tau1 * a), 0.f);
            knew = dmn - x0n + x1n;
          } else {
            const float th = P.theta;
            x1n = fmaxf(th * c1_[k] + (1.f - th) * (x1_[k] - tau1 * a), 0.f);
            knew = dmn - c0_[k] + x1n;
          }
          if (RES != R_BAL) knew -= rn;
          if (KEEPSTEP && k < NOWN) {
            if (RES != R_BAL) kpr_[k] = (r_[k] - rn) * it1 + a;
            if (MODE == 1) kp0_[k] = (x0_[k] - x0n) * it1 + a;
            if (MODE != 0) kp1_[k] = (x1_[k] - x1n) * it1 - a;
          }
          const bool in = !MASK || (f_[k] & F_IN);
          sa[l_[k]] = in ? a + tau2 * (2.f * knew - kp_[k]) : 0.f;
          kp_[k] = knew;
          r_[k] = rn;
          x0_[k] = x0n;
          x1_[k] = x1n;
        }
      }
      __syncthreads();
    };
    auto run = [&](auto mask_tag) {
      if (CHK) {
        // the host launches the check variant with 1 <= steps <= H - 1
        for (int st = 0; st + 1 < steps; ++st) one_step(std::false_type{}, mask_tag);
        one_step(std::true_type{}, mask_tag);
      } else {
        for (int st = 0; st < steps; ++st) one_step(std::false_type{}, mask_tag);
      }
    };
    // a region inside the grid and away from its right and top edges needs
    // no mask (the slots past the region read and write only zeros); the
    // check variant always masks (a second copy of its steps would cost it
    // registers and occupancy)
    if constexpr (!CHK) {
      if (interior) run(std::false_type{});
      else run(std::true_type{});
    } else {
      run(std::true_type{});
    }

    if (CHK) {
      // the stopping rule's terms for the iterate pair of the last step, per
      // owned cell, with the expressions of check_kernel: the new dual is
      // exact one cell beyond the tile, where its gradient reads the right
      // and upper neighbours; K(z) of the new iterate is the last step's
      constexpr float nid = (MODE == 0 ? 1 : (MODE == 1 ? 3 : 2)) - (RES == R_BAL ? 1 : 0);
      double ts_[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // this tile's sums, in the order of kSumSlot
#pragma unroll
      for (int k = 0; k < NOWN; ++k) {
        if (!(f_[k] & F_IN)) continue;
        const int l = l_[k];
        const float a = sa[l], aR = sa[l + 1], aU = sa[l + LW];
        const bool zx = (BC & 1) == 0 && (f_[k] & F_ZX), zy = (BC & 1) == 0 && (f_[k] & F_ZY);
        const float gxx = zx ? 0.f : a - aR, gyy = zy ? 0.f : a - aU;
        const float sx = kpx_[k] + gxx, sy = kpy_[k] + gyy;
        float st2 = sx * sx + sy * sy;
        float r = 0.f, x0 = 0.f, x1 = 0.f;
        if (RES != R_BAL) {
          r = r_[k];
          const float sr = kpr_[k] - a;
          st2 += sr * sr;
        }
        if (MODE == 1) {
          x0 = x0_[k];
          const float s0 = kp0_[k] - a;
          st2 += s0 * s0;
        }
        if (MODE != 0) {
          x1 = x1_[k];
          const float s1 = kp1_[k] + a;
          st2 += s1 * s1;
        }
        const float kz = kp_[k];
        const float g2 = gxx * gxx + gyy * gyy;
        ts_[0] += kz * kz;
        ts_[1] += st2;
        ts_[2] += g2 + nid * a * a;
        if (MODE == 1) ts_[3] += x0 * x0;
        if (MODE != 0) ts_[NSUM - 1] += x1 * x1;
        const bool fin = isfinite(a) && isfinite(smx[l]) && isfinite(smy[l]) && isfinite(r) && isfinite(x0) &&
                         isfinite(x1);
        nonfin += fin ? 0 : 1;
      }
#pragma unroll
      for (int q = 0; q < NSUM; ++q) runsum[q * BLOCK + tid] += ts_[q];
    }

    // ---- write the owned tile ----
    const RegionPlane qa(A.out.a, rbase), qmx(A.out.Mx, rbase), qmy(A.out.My, rbase), qr(A.out.r, rbase),
        qx0(A.out.x0, rbase), qx1(A.out.x1, rbase);
#pragma unroll
    for (int k = 0; k < NOWN; ++k) {
      if (!(f_[k] & F_IN)) continue;
      const int l = l_[k];
      const int idx = tid + k * BLOCK;  // an owned cell: row idx / 64 of the tile
      const unsigned bo = ((unsigned)(H + idx / TX) * (unsigned)pitch + (unsigned)(H + idx % TX)) * 4u;
      qmx.st(bo, smx[l]);
      qmy.st(bo, smy[l]);
      qa.st(bo, sa[l]);
      if (RES != R_BAL) qr.st(bo, r_[k]);
      if (MODE == 1) qx0.st(bo, x0_[k]);
      if (MODE != 0) qx1.st(bo, x1_[k]);
    }
  }
  if (CHK && run_pair >= 0) flush_run();
}

template <int MODE, int RES, int BC, int TH, int T>
__global__ __launch_bounds__(BLOCK) void cp_iter_tb_kernel(IterArgs A) {
  cp_iter_tb_body<MODE, RES, BC, TH, T, false>(A);
}

// The last launch of a check window on a blocked shape: up to H - 1 steps
// of the blocked kernel with a halo of H that also leave the stopping rule's
// partial rows of the iterate pair of its last step (so the window needs
// neither a single-step launch nor a separate check).  Occupancy targets
// that the variants meet without spilling: on tiles of up to 16 rows DIST
// (flux, r and a per cell) fits 128 VGPRs, so a CU takes four workgroups,
// and the modes with x0 and x1 take three; 32-row tiles take two.
template <int MODE, int RES, int BC, int TH, int H>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(TH >= 32 ? 2 : (MODE == 0 ? 4 : 3)))) void
cp_iter_tb_check_kernel(IterArgs A) {
  cp_iter_tb_body<MODE, RES, BC, TH, H, true>(A);
}

// Residuals and certificate terms of the current iterate (K2).  Direct
// global loads; neighbours come from the L2.  Per-pixel terms in FP32,
// sums over pixels in FP64.  Runs once per check window.
template <int MODE, int RES, int BC>
__global__ __launch_bounds__(BLOCK) void check_kernel(CheckArgs A) {
  const int lx = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr float nid = (MODE == 0 ? 1 : (MODE == 1 ? 3 : 2)) - (RES == R_BAL ? 1 : 0);
  for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
    const Tile tl = A.tiles[t];
    const bool act = A.active[tl.pair] != 0;
    if (!act && !A.all_pairs) continue;  // uniform
    const PairInfo P = A.pairs[tl.pair];
    const bool swap = A.swap_active && act;
    const Planes C = swap ? A.B : A.A;
    const Planes Q = swap ? A.A : A.B;  // previous iterate
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const float it1 = 1.f / P.tau1;
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    for (int ly = wv; ly < A.tile_rows; ly += 4) {
      const int gx = tl.x0 + lx, gy = tl.y0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const long o = P.off + (long)gy * pitch + gx;
      const bool hasR = gx + 1 < nx, hasU = gy + 1 < ny;
      const bool hasL = gx > 0, hasD = gy > 0;
      const float a = C.a[o], ap = Q.a[o];
      const float aR = hasR ? C.a[o + 1] : 0.f, apR = hasR ? Q.a[o + 1] : 0.f;
      const float aU = hasU ? C.a[o + pitch] : 0.f, apU = hasU ? Q.a[o + pitch] : 0.f;
      // the gradients of the dual and of the previous dual
      float gxx = a - aR, gyy = a - aU;
      float gxo = ap - apR, gyo = ap - apU;
      const bool zx = ((BC & 1) == 0 && gx == nx - 1), zy = ((BC & 1) == 0 && gy == ny - 1);
      if (zx) gxx = gxo = 0.f;
      if (zy) gyy = gyo = 0.f;
      const float mx = zx ? 0.f : C.Mx[o], my = zy ? 0.f : C.My[o];
      const float mxp = zx ? 0.f : Q.Mx[o], myp = zy ? 0.f : Q.My[o];
      const float mxl = hasL ? C.Mx[o - 1] : 0.f;
      const float myd = hasD ? C.My[o - pitch] : 0.f;
      const float dm = mx - mxl + my - myd;  // the steps' order of the terms
      float x0 = 0.f, x1 = 0.f, e;
      if (MODE == 0) {
        e = dm + A.c[o];
      } else if (MODE == 1) {
        x0 = C.x0[o];
        x1 = C.x1[o];
        e = dm - x0 + x1;
      } else {
        x1 = C.x1[o];
        e = dm - A.src[o] + x1;
      }
      float r = 0.f, rp = 0.f;
      if (RES != R_BAL) {
        r = C.r[o];
        rp = Q.r[o];
      }
      const float kz = e - r;
      // the stationarity residual (z^{k-1} - z^k)/tau1 - K*(a^{k-1} - a^k),
      // grouped as the blocked kernels form it: the previous dual's part
      // with the step's values, then the dual's
      const float sx = ((mxp - mx) * it1 - gxo) + gxx, sy = ((myp - my) * it1 - gyo) + gyy;
      float st2 = sx * sx + sy * sy;
      if (RES != R_BAL) {
        const float sr = ((rp - r) * it1 + ap) - a;
        st2 += sr * sr;
      }
      if (MODE == 1) {
        const float s0 = ((Q.x0[o] - x0) * it1 + ap) - a;
        st2 += s0 * s0;
      }
      if (MODE != 0) {
        const float s1 = ((Q.x1[o] - x1) * it1 - ap) + a;
        st2 += s1 * s1;
      }
      const float g2 = gxx * gxx + gyy * gyy;
      acc[S_PRES2] += kz * kz;
      acc[S_STAT2] += st2;
      acc[S_KA2] += g2 + nid * a * a;
      acc[S_X0SQ] += x0 * x0;
      acc[S_X1SQ] += x1 * x1;
      acc[S_MNORM] += (BC & 2) ? fabsf(mx) + fabsf(my) : sqrtf(mx * mx + my * my);
      if (RES == R_P1) {
        acc[S_RPEN] += fabsf(r);
        acc[S_EPEN] += fabsf(e);
      } else if (RES == R_P2) {
        acc[S_RPEN] += r * r;
        acc[S_EPEN] += e * e;
      }
      if (MODE == 0) acc[S_LIN] += a * A.c[o];
      if (MODE == 2) acc[S_LIN] -= a * A.src[o];
      if (MODE == 1) {
        const float d0 = x0 - A.src[o], d1 = x1 - A.dst[o];
        acc[S_QUAD] += d0 * d0 + d1 * d1;
      }
      if (MODE == 2) {
        const float d1 = x1 - A.dst[o];
        acc[S_QUAD] += d1 * d1;
      }
      acc[S_MAXG] = fmax(acc[S_MAXG], (double)((BC & 2) ? fmaxf(fabsf(gxx), fabsf(gyy)) : sqrtf(g2)));
      acc[S_MAXA] = fmax(acc[S_MAXA], (double)fabsf(a));
      const bool fin = isfinite(a) && isfinite(mx) && isfinite(my) && isfinite(r) && isfinite(x0) &&
                       isfinite(x1);
      acc[S_NONFIN] += fin ? 0.0 : 1.0;
      acc[S_A2] += a * a;
      acc[S_SUMA] += a;
    }
    block_reduce_store(acc, kMaxSlotsCheck, A.partial + (long)t * NS);
  }
}

// ---------------------------------------------------------------------------
// Launchers

namespace {
template <int MODE, int RES, int BC>
hipError_t iter_by_ty(int ty, int grid, const IterArgs& a, hipStream_t s) {
  switch (ty) {
    case 4: hipLaunchKernelGGL((cp_iter_kernel<MODE, RES, BC, 4>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 8: hipLaunchKernelGGL((cp_iter_kernel<MODE, RES, BC, 8>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 16: hipLaunchKernelGGL((cp_iter_kernel<MODE, RES, BC, 16>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 32: hipLaunchKernelGGL((cp_iter_kernel<MODE, RES, BC, 32>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 116: hipLaunchKernelGGL((cp_iter_vec_kernel<MODE, RES, BC, 16, false>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 132: hipLaunchKernelGGL((cp_iter_vec_kernel<MODE, RES, BC, 32, false>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 316: hipLaunchKernelGGL((cp_iter_vec_kernel<MODE, RES, BC, 16, true>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 332: hipLaunchKernelGGL((cp_iter_vec_kernel<MODE, RES, BC, 32, true>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 4008: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 8, 4>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 4004: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 4, 4>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 2016: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 16, 2>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 8016: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 16, 8>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 4016: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 16, 4>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 4032: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 32, 4>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 8032: hipLaunchKernelGGL((cp_iter_tb_kernel<MODE, RES, BC, 32, 8>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

using IterKernel = void (*)(IterArgs);

// The check variant of a blocked shape: its tile rows with a halo of one
// more than the steps it runs (the check reads one cell beyond the tile);
// chk_steps() gives those steps per shape.
template <int MODE, int RES, int BC>
IterKernel chk_kernel_ty(int ty) {
  switch (ty) {
    case 4004: return cp_iter_tb_check_kernel<MODE, RES, BC, 4, 5>;
    case 4008: return cp_iter_tb_check_kernel<MODE, RES, BC, 8, 5>;
    case 2016: return cp_iter_tb_check_kernel<MODE, RES, BC, 16, 3>;
    case 4016:
    case 8016: return cp_iter_tb_check_kernel<MODE, RES, BC, 16, 5>;
    case 4032:
    case 8032: return cp_iter_tb_check_kernel<MODE, RES, BC, 32, 3>;
  }
  return nullptr;
}
template <int MODE, int RES>
IterKernel chk_kernel_bc(int bcn, int ty) {
  switch (bcn) {
    case 0: return chk_kernel_ty<MODE, RES, 0>(ty);
    case 1: return chk_kernel_ty<MODE, RES, 1>(ty);
    case 2: return chk_kernel_ty<MODE, RES, 2>(ty);
    case 3: return chk_kernel_ty<MODE, RES, 3>(ty);
  }
  return nullptr;
}
template <int MODE>
IterKernel chk_kernel(int res, int bcn, int ty) {
  switch (res) {
    case R_BAL: return chk_kernel_bc<MODE, R_BAL>(bcn, ty);
    case R_P1: return chk_kernel_bc<MODE, R_P1>(bcn, ty);
    case R_P2: return chk_kernel_bc<MODE, R_P2>(bcn, ty);
  }
  return nullptr;
}

template <int MODE, int RES, int BC>
hipError_t occ_by_ty(int ty, int* n) {
  switch (ty) {
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_kernel<MODE, RES, BC, 4>, BLOCK, 0);
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_kernel<MODE, RES, BC, 8>, BLOCK, 0);
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_kernel<MODE, RES, BC, 16>, BLOCK, 0);
    case 32: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_kernel<MODE, RES, BC, 32>, BLOCK, 0);
    case 116: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_vec_kernel<MODE, RES, BC, 16, false>, BLOCK, 0);
    case 132: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_vec_kernel<MODE, RES, BC, 32, false>, BLOCK, 0);
    case 316: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_vec_kernel<MODE, RES, BC, 16, true>, BLOCK, 0);
    case 332: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_vec_kernel<MODE, RES, BC, 32, true>, BLOCK, 0);
    case 4008: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 8, 4>, BLOCK, 0);
    case 4004: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 4, 4>, BLOCK, 0);
    case 2016: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 16, 2>, BLOCK, 0);
    case 8016: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 16, 8>, BLOCK, 0);
    case 4016: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 16, 4>, BLOCK, 0);
    case 4032: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 32, 4>, BLOCK, 0);
    case 8032: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, cp_iter_tb_kernel<MODE, RES, BC, 32, 8>, BLOCK, 0);
    default: return hipErrorInvalidValue;
  }
}

// bcn: bit 0 the boundary reading (bc), bit 1 the anisotropic flux norm
template <int MODE, int RES>
hipError_t iter_bc(int bcn, int ty, int grid, const IterArgs& a, hipStream_t s) {
  switch (bcn) {
    case 0: return iter_by_ty<MODE, RES, 0>(ty, grid, a, s);
    case 1: return iter_by_ty<MODE, RES, 1>(ty, grid, a, s);
    case 2: return iter_by_ty<MODE, RES, 2>(ty, grid, a, s);
    case 3: return iter_by_ty<MODE, RES, 3>(ty, grid, a, s);
  }
  return hipErrorInvalidValue;
}
template <int MODE>
hipError_t iter_res(int res, int bc, int ty, int grid, const IterArgs& a, hipStream_t s) {
  switch (res) {
    case R_BAL: return iter_bc<MODE, R_BAL>(bc, ty, grid, a, s);
    case R_P1: return iter_bc<MODE, R_P1>(bc, ty, grid, a, s);
    case R_P2: return iter_bc<MODE, R_P2>(bc, ty, grid, a, s);
  }
  return hipErrorInvalidValue;
}

template <int MODE, int RES>
hipError_t occ_bc(int bcn, int ty, int* n) {
  switch (bcn) {
    case 0: return occ_by_ty<MODE, RES, 0>(ty, n);
    case 1: return occ_by_ty<MODE, RES, 1>(ty, n);
    case 2: return occ_by_ty<MODE, RES, 2>(ty, n);
    case 3: return occ_by_ty<MODE, RES, 3>(ty, n);
  }
  return hipErrorInvalidValue;
}
template <int MODE>
hipError_t occ_res(int res, int bc, int ty, int* n) {
  switch (res) {
    case R_BAL: return occ_bc<MODE, R_BAL>(bc, ty, n);
    case R_P1: return occ_bc<MODE, R_P1>(bc, ty, n);
    case R_P2: return occ_bc<MODE, R_P2>(bc, ty, n);
  }
  return hipErrorInvalidValue;
}

template <int MODE, int RES>
hipError_t check_bc(int bcn, int grid, const CheckArgs& a, hipStream_t s) {
  switch (bcn) {
    case 0: hipLaunchKernelGGL((check_kernel<MODE, RES, 0>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 1: hipLaunchKernelGGL((check_kernel<MODE, RES, 1>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 2: hipLaunchKernelGGL((check_kernel<MODE, RES, 2>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    case 3: hipLaunchKernelGGL((check_kernel<MODE, RES, 3>), dim3(grid), dim3(BLOCK), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <int MODE>
hipError_t check_res(int res, int bc, int grid, const CheckArgs& a, hipStream_t s) {
  switch (res) {
    case R_BAL: return check_bc<MODE, R_BAL>(bc, grid, a, s);
    case R_P1: return check_bc<MODE, R_P1>(bc, grid, a, s);
    case R_P2: return check_bc<MODE, R_P2>(bc, grid, a, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace

}  // namespace uot
