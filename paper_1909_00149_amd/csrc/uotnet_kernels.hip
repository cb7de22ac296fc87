// Kernels of the learned warm-start network (gfx950): BF16 activations and
// weights, FP32 accumulation on the matrix cores.
//
// A 3x3 convolution (stride 1, zero padding 1) over NHWC tensors is an
// implicit GEMM.  Forward: M = pixels, N = output channels, K = 9 * Cin with
// k = tap * Cin + ci (tap = 3 dy + dx); A is gathered from the input with
// its halo, B is the weight tensor stored [Cout][9][Cin].  The input
// gradient is the same product with the weights flipped and transposed
// ([Cin][9][Cout], tap 8 - t).  The weight gradient is a product over
// pixels: M = Cout, N = 9 * Cin, K = pixels, split over pixel ranges.
//
// One 256-thread workgroup computes an output tile: 128 pixels x 64 (or
// 32) channels for the convolution (convw_kernel), 64 x 64 for the weight
// gradient, whose four wavefronts own 32 x 32 quarters as 2 x 2 blocks of
// the 16x16x32 BF16 MFMA.  Operand tiles are staged in LDS with k contiguous (rows padded to
// 40 elements so the 16-byte fragment reads of the 16 rows land in distinct
// banks).  Lane l of a wavefront reads A row l%16 and B column l%16, k
// elements 8*(l/16)..+7; it receives D rows 4*(l/16)+i, column l%16.
#include "uotnet_internal.hpp"

namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void mma_tile(const uint16_t (*As)[LDK], const uint16_t (*Bs)[LDK], f32x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  bf16x8 a[2], b[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    a[t] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + t * 16 + r][kq]);
    b[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + t * 16 + r][kq]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
}

// y = conv(x) (+ bias) (relu); optional mask multiplies the result by
// (mask > 0) (the ReLU derivative of the layer that produced the input of
// the forward conv, when this launch computes an input gradient).
// A workgroup computes 64 MI pixels x 16 NB output channels: each
// wavefront owns 16 MI pixels x all NB blocks of 16 channels, so a k chunk
// of 32 is MI NB MFMAs per wavefront, and the next chunk's operands are
// loaded into registers while the current one multiplies.  For every output
// element the MFMAs take the k chunks in increasing order.
template <int MI, int NB>
__global__ __launch_bounds__(256) void convw_kernel(ConvArgs A) {
  constexpr int BMm = 64 * MI, BNn = 16 * NB;
  __shared__ __attribute__((aligned(16))) uint16_t As[BMm][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BNn][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long M = (long)A.N * A.H * A.W;
  const int K = 9 * A.Cin;
  const long m0 = (long)blockIdx.y * BMm;
  const int n0 = blockIdx.x * BNn;
  f32x4 acc[MI][NB];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this thread's A rows (pixels row + 64 h, h < MI) and, for the threads
  // with row < 16 NB, its B row (output channel)
  const int row = tid >> 2, kc = (tid & 3) * 8;
  long pn[MI];
  int py[MI], px[MI];
  bool mv[MI];
#pragma unroll
  for (int h = 0; h < MI; ++h) {
    const long m = m0 + row + 64 * h;
    mv[h] = m < M;
    pn[h] = 0;
    py[h] = px[h] = 0;
    if (mv[h]) {
      pn[h] = m / ((long)A.H * A.W);
      const long rem = m - pn[h] * A.H * A.W;
      py[h] = (int)(rem / A.W);
      px[h] = (int)(rem - (long)py[h] * A.W);
    }
  }
  const int co = n0 + row;
  const bool brow = row < BNn && co < A.Cout;
  u16x8 va[MI], vb;
  auto load = [&](int k0) {
    const int k = k0 + kc;
    const bool kin = k < K;
    const int tap = kin ? k / A.Cin : 0, ci = k - tap * A.Cin;
#pragma unroll
    for (int h = 0; h < MI; ++h) {
      va[h] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      const int iy = py[h] + tap / 3 - 1, ix = px[h] + tap % 3 - 1;
      if (mv[h] && kin && iy >= 0 && iy < A.H && ix >= 0 && ix < A.W)
        va[h] = *reinterpret_cast<const u16x8*>(A.X + (((pn[h] * A.H + iy) * A.W + ix) * A.Cin + ci));
    }
    vb = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (brow && kin) vb = *reinterpret_cast<const u16x8*>(A.Wt + ((long)co * K + k));
  };
  load(0);
  const int r = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int h = 0; h < MI; ++h) *reinterpret_cast<u16x8*>(&As[row + 64 * h][kc]) = va[h];
    if (row < BNn) *reinterpret_cast<u16x8*>(&Bs[row][kc]) = vb;
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);  // in flight during the MFMAs
    bf16x8 a[MI], b[NB];
#pragma unroll
    for (int t = 0; t < MI; ++t) a[t] = *reinterpret_cast<const bf16x8*>(&As[wv * 16 * MI + t * 16 + r][kq]);
#pragma unroll
    for (int t = 0; t < NB; ++t) b[t] = *reinterpret_cast<const bf16x8*>(&Bs[t * 16 + r][kq]);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + j * 16 + (lane & 15);
      if (n >= A.Cout) continue;
      const float bias = A.bias ? A.bias[n] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long mm = m0 + wv * 16 * MI + i * 16 + (lane >> 4) * 4 + e;
        if (mm >= M) continue;
        float v = acc[i][j][e] + bias;
        if (A.relu) v = fmaxf(v, 0.f);
        const long o = mm * A.Cout + n;
        if (A.mask && !(bf2f(A.mask[o]) > 0.f)) v = 0.f;
        if (A.Yf) A.Yf[o] = v;
        if (A.Y) A.Y[o] = f2bf(v);
      }
    }
}

// Partial weight gradient over one pixel range (grid.z):
//   part[z][co][tap*Cin + ci] = sum_p gy[p][co] x[p shifted by tap][ci]
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs A) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDK];
  const int tid = threadIdx.x;
  const long P = (long)A.N * A.H * A.W;
  const int K9 = 9 * A.Cin;
  const int c0 = blockIdx.y * BM;   // output channels
  const int n0 = blockIdx.x * BN;   // tap * Cin + ci
  const long per = ((P + gridDim.z - 1) / gridDim.z + BK - 1) / BK * BK;
  const long pbeg = (long)blockIdx.z * per;
  const long pend = pbeg + per < P ? pbeg + per : P;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int pl = tid >> 3, ch = (tid & 7) * 8;  // pixel within the chunk, channel chunk
  for (long p0 = pbeg; p0 < pend; p0 += BK) {
    const long p = p0 + pl;
    u16x8 va = {0, 0, 0, 0, 0, 0, 0, 0}, vb = {0, 0, 0, 0, 0, 0, 0, 0};
    if (p < pend) {
      if (c0 + ch < A.Cout) va = *reinterpret_cast<const u16x8*>(A.GY + (p * A.Cout + c0 + ch));
      const int k9 = n0 + ch;
      if (k9 < K9) {
        const int tap = k9 / A.Cin, ci = k9 - tap * A.Cin;
        const long pn = p / ((long)A.H * A.W);
        const long rem = p - pn * A.H * A.W;
        const int y = (int)(rem / A.W), x = (int)(rem - (long)y * A.W);
        const int iy = y + tap / 3 - 1, ix = x + tap % 3 - 1;
        if (iy >= 0 && iy < A.H && ix >= 0 && ix < A.W)
          vb = *reinterpret_cast<const u16x8*>(A.X + (((pn * A.H + iy) * A.W + ix) * A.Cin + ci));
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[ch + e][pl] = va[e];
      Bs[ch + e][pl] = vb[e];
    }
    __syncthreads();
    mma_tile(As, Bs, acc);
    __syncthreads();
  }
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  float* out = A.part + (long)blockIdx.z * A.Cout * K9;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      if (n >= K9) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = c0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
        if (c < A.Cout) out[(long)c * K9 + n] = acc[i][j][e];
      }
    }
}

// dst[i] (=|+=) sum_z part[z][i]
__global__ void sum_splits_kernel(const float* part, int splits, long n, float* dst, int accumulate) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(long)z * n + i];
    dst[i] = accumulate ? dst[i] + s : s;
  }
}

// Bias gradient partials: part[block][c] = sum over the block's pixels of gy[p][c].
__global__ __launch_bounds__(256) void bias_grad_kernel(const uint16_t* gy, long P, int C, float* part) {
  const int c = threadIdx.x & 63, lane_group = threadIdx.x >> 6;
  for (int cb = 0; cb < C; cb += 64) {
    float s = 0.f;
    if (cb + c < C)
      for (long p = blockIdx.x * 4 + lane_group; p < P; p += (long)gridDim.x * 4) s += bf2f(gy[p * C + cb + c]);
    __shared__ float red[4][64];
    red[lane_group][c] = s;
    __syncthreads();
    if (lane_group == 0 && cb + c < C) part[(long)blockIdx.x * C + cb + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    __syncthreads();
  }
}

// Network input: channel 0 = src * scale, channel 1 = dst * scale, the
// rest of the Cpad channels zero.  src/dst are B packed planes of H*W.
__global__ void pack_input_kernel(const float* src, const float* dst, float scale, long P, int Cpad, uint16_t* X) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    v[0] = f2bf(src[p] * scale);
    v[1] = f2bf(dst[p] * scale);
    *reinterpret_cast<u16x8*>(X + p * Cpad) = v;
    for (int c = 8; c < Cpad; c += 8) *reinterpret_cast<u16x8*>(X + p * Cpad + c) = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }
}

// 2x2 average pooling, NHWC.
__global__ void pool2_kernel(const uint16_t* x, int N, int H, int W, int C, uint16_t* y) {
  const int Ho = H / 2, Wo = W / 2;
  const long n = (long)N * Ho * Wo * C;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    long r = e / C;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const long b = r / Ho;
    const long base = ((b * H + 2 * yo) * W + 2 * xo) * C + c;
    const float s = bf2f(x[base]) + bf2f(x[base + C]) + bf2f(x[base + (long)W * C]) + bf2f(x[base + (long)W * C + C]);
    y[e] = f2bf(0.25f * s);
  }
}

// The same, 8 channels (16 bytes) per thread with 32-bit pixel indices
// (C a multiple of 8, 16-byte aligned tensors, N H W < 2^31): the same sum
// per element in the same order.
__global__ void pool2_v8_kernel(const uint16_t* x, int N, int H, int W, int C, uint16_t* y) {
  const int Ho = H / 2, Wo = W / 2, G = C / 8;
  const long n = (long)N * Ho * Wo * G;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const unsigned q = (unsigned)(e / G);  // output pixel
    const int c = (int)(e - (long)q * G) * 8;
    const unsigned xo = q % Wo, r = q / Wo, yo = r % Ho, b = r / Ho;
    const long base = ((long)(b * H + 2 * yo) * W + 2 * xo) * C + c;
    const u16x8 v0 = *reinterpret_cast<const u16x8*>(x + base);
    const u16x8 v1 = *reinterpret_cast<const u16x8*>(x + base + C);
    const u16x8 v2 = *reinterpret_cast<const u16x8*>(x + base + (long)W * C);
    const u16x8 v3 = *reinterpret_cast<const u16x8*>(x + base + (long)W * C + C);
    u16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = f2bf(0.25f * (bf2f(v0[i]) + bf2f(v1[i]) + bf2f(v2[i]) + bf2f(v3[i])));
    *reinterpret_cast<u16x8*>(y + (long)q * C + c) = o;
  }
}

// Gradient through the pooling, masked by the ReLU of the pooled tensor,
// plus an optional (already masked) skip gradient.
__global__ void pool2_bwd_kernel(const uint16_t* gy, const uint16_t* mask, const uint16_t* add, int N, int H, int W,
                                 int C, uint16_t* gx) {
  const long n = (long)N * H * W * C;
  const int Ho = H / 2, Wo = W / 2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    long r = e / C;
    const int x = (int)(r % W);
    r /= W;
    const int y = (int)(r % H);
    const long b = r / H;
    float v = 0.25f * bf2f(gy[((b * Ho + y / 2) * Wo + x / 2) * C + c]);
    if (mask && !(bf2f(mask[e]) > 0.f)) v = 0.f;
    if (add) v += bf2f(add[e]);
    gx[e] = f2bf(v);
  }
}

// cat[b, y, x, :] = [up2(d)[b, y, x, 0:Cu], e[b, y, x, 0:Cs]]
__global__ void up_concat_kernel(const uint16_t* d, const uint16_t* e, int N, int H, int W, int Cu, int Cs,
                                 uint16_t* cat) {
  const int C = Cu + Cs;
  const long n = (long)N * H * W * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long p = i / C;
    const int x = (int)(p % W);
    const int y = (int)((p / W) % H);
    const long b = p / ((long)W * H);
    cat[i] = c < Cu ? d[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu + c] : e[p * Cs + (c - Cu)];
  }
}

// The same, 8 channels (16 bytes) per thread with 32-bit pixel indices (Cu
// and Cs multiples of 8, 16-byte aligned tensors, N H W < 2^31).
__global__ void up_concat_v8_kernel(const uint16_t* d, const uint16_t* e, int N, int H, int W, int Cu, int Cs,
                                    uint16_t* cat) {
  const int C = Cu + Cs, G = C / 8;
  const long n = (long)N * H * W * G;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const unsigned p = (unsigned)(i / G);  // output pixel
    const int c = (int)(i - (long)p * G) * 8;
    const unsigned x = p % W, r = p / W, y = r % H, b = r / H;
    const uint16_t* src = c < Cu ? d + ((long)(b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu + c
                                 : e + (long)p * Cs + (c - Cu);
    *reinterpret_cast<u16x8*>(cat + (long)p * C + c) = *reinterpret_cast<const u16x8*>(src);
  }
}

// Split the gradient of a concat: the upsampled part is summed over each
// 2x2 block (gradient of nearest upsampling) and masked by the ReLU of d;
// the skip part is masked by the ReLU of e.
__global__ void up_concat_bwd_kernel(const uint16_t* gcat, const uint16_t* dmask, const uint16_t* emask, int N,
                                     int H, int W, int Cu, int Cs, uint16_t* gd, uint16_t* ge) {
  const int C = Cu + Cs;
  const int Hl = H / 2, Wl = W / 2;
  const long nd = (long)N * Hl * Wl * Cu;
  const long ne = (long)N * H * W * Cs;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nd + ne; i += (long)gridDim.x * blockDim.x) {
    if (i < nd) {
      const int c = (int)(i % Cu);
      const long p = i / Cu;
      const int x = (int)(p % Wl);
      const int y = (int)((p / Wl) % Hl);
      const long b = p / ((long)Wl * Hl);
      const long q = ((b * H + 2 * y) * W + 2 * x) * C + c;
      float s = bf2f(gcat[q]) + bf2f(gcat[q + C]) + bf2f(gcat[q + (long)W * C]) + bf2f(gcat[q + (long)W * C + C]);
      if (!(bf2f(dmask[i]) > 0.f)) s = 0.f;
      gd[i] = f2bf(s);
    } else {
      const long j = i - nd;
      const int c = (int)(j % Cs);
      const long p = j / Cs;
      float v = bf2f(gcat[p * C + Cu + c]);
      if (!(bf2f(emask[j]) > 0.f)) v = 0.f;
      ge[j] = f2bf(v);
    }
  }
}

// Loss against solver targets.  out: fp32 [P][Cpad] (channels 0..2 used);
// targets: three packed planes (Mx, My, a) scaled to (s_flux Mx, s_flux My,
// s_dual a).  Writes the output gradient (bf16, [P][Cpad]) and per-block
// partial sums of the squared error.
__global__ __launch_bounds__(256) void loss_kernel(const float* out, int Cpad, const float* tMx, const float* tMy,
                                                   const float* ta, float s_flux, float s_dual, long P,
                                                   uint16_t* gout, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  const float g = 2.f / (float)P;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) {
    const float t[3] = {tMx[p] * s_flux, tMy[p] * s_flux, ta[p] * s_dual};
    for (int c = 0; c < Cpad; ++c) {
      float d = 0.f;
      if (c < 3) {
        d = out[p * Cpad + c] - t[c];
        acc += (double)d * d;
      }
      gout[p * Cpad + c] = f2bf(g * d);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] / (double)P;
}

// Adam (Kingma and Ba) on the FP32 master copy; bf16 copy for compute.
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* pbf) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pbf) pbf[i] = f2bf(pi);
  }
}

// bf16 copy of FP32 values
__global__ void to_bf16_kernel(const float* x, long n, uint16_t* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

// Flipped, transposed weights for the input gradient: wt[ci][8 - t][co] = w[co][t][ci].
__global__ void flip_weights_kernel(const uint16_t* w, int Cout, int Cin, uint16_t* wt) {
  const long n = (long)Cout * 9 * Cin;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ci = (int)(i % Cin);
    const int t = (int)((i / Cin) % 9);
    const int co = (int)(i / (9L * Cin));
    wt[((long)ci * 9 + (8 - t)) * Cout + co] = w[i];
  }
}

// Network output -> solver state: Mx = out0 / s_flux, My = out1 / s_flux
// (structurally zero on the last column / row), a = out2 / s_dual.
__global__ void head_to_state_kernel(const float* out, int Cpad, int H, int W, long P, float s_flux, float s_dual,
                                     float* Mx, float* My, float* a) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) {
    const long q = p % ((long)H * W);
    const int y = (int)(q / W), x = (int)(q - (long)y * W);
    Mx[p] = x < W - 1 ? out[p * Cpad + 0] / s_flux : 0.f;
    My[p] = y < H - 1 ? out[p * Cpad + 1] / s_flux : 0.f;
    a[p] = out[p * Cpad + 2] / s_dual;
  }
}

// r = D M + dst - src (so the start satisfies the constraint).
__global__ void complete_residual_kernel(const float* Mx, const float* My, const float* src, const float* dst, int H,
                                         int W, long P, float* r) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < P; p += (long)gridDim.x * blockDim.x) {
    const long q = p % ((long)H * W);
    const int y = (int)(q / W), x = (int)(q - (long)y * W);
    const float dm = Mx[p] - (x > 0 ? Mx[p - 1] : 0.f) + My[p] - (y > 0 ? My[p - W] : 0.f);
    r[p] = dm + dst[p] - src[p];
  }
}

// ---------------------------------------------------------------------------
static int egrid(long n) { return (int)(n / 256 + 1 < 8192 ? n / 256 + 1 : 8192); }

hipError_t conv(const ConvArgs& a, hipStream_t s) {
  const long M = (long)a.N * a.H * a.W;
  // 128-pixel tiles (MI = 2; 64- and 256-pixel tiles were slower); 32
  // channels per tile when the layer has no more
  const unsigned gy = (unsigned)((M + 127) / 128);
  if (a.Cout <= 32)
    hipLaunchKernelGGL((convw_kernel<2, 2>), dim3((a.Cout + 31) / 32, gy), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((convw_kernel<2, 4>), dim3((a.Cout + 63) / 64, gy), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t wgrad(const WgradArgs& a, int splits, hipStream_t s) {
  const dim3 grid((9 * a.Cin + BN - 1) / BN, (a.Cout + BM - 1) / BM, splits);
  hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t sum_splits(const float* part, int splits, long n, float* dst, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(sum_splits_kernel, dim3(egrid(n)), dim3(256), 0, s, part, splits, n, dst, accumulate);
  return hipGetLastError();
}

hipError_t bias_grad(const uint16_t* gy, long P, int C, float* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(bias_grad_kernel, dim3(blocks), dim3(256), 0, s, gy, P, C, part);
  return hipGetLastError();
}

hipError_t pack_input(const float* src, const float* dst, float scale, long P, int Cpad, uint16_t* X, hipStream_t s) {
  hipLaunchKernelGGL(pack_input_kernel, dim3(egrid(P)), dim3(256), 0, s, src, dst, scale, P, Cpad, X);
  return hipGetLastError();
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

hipError_t pool2(const uint16_t* x, int N, int H, int W, int C, uint16_t* y, hipStream_t s) {
  if (C % 8 == 0 && aligned16(x) && aligned16(y) && (long)N * H * W < (1L << 31))
    hipLaunchKernelGGL(pool2_v8_kernel, dim3(egrid((long)N * H * W * C / 32)), dim3(256), 0, s, x, N, H, W, C, y);
  else
    hipLaunchKernelGGL(pool2_kernel, dim3(egrid((long)N * H * W * C / 4)), dim3(256), 0, s, x, N, H, W, C, y);
  return hipGetLastError();
}

hipError_t pool2_bwd(const uint16_t* gy, const uint16_t* mask, const uint16_t* add, int N, int H, int W, int C,
                     uint16_t* gx, hipStream_t s) {
  hipLaunchKernelGGL(pool2_bwd_kernel, dim3(egrid((long)N * H * W * C)), dim3(256), 0, s, gy, mask, add, N, H, W, C, gx);
  return hipGetLastError();
}

hipError_t up_concat(const uint16_t* d, const uint16_t* e, int N, int H, int W, int Cu, int Cs, uint16_t* cat,
                     hipStream_t s) {
  if (Cu % 8 == 0 && Cs % 8 == 0 && aligned16(d) && aligned16(e) && aligned16(cat) && (long)N * H * W < (1L << 31))
    hipLaunchKernelGGL(up_concat_v8_kernel, dim3(egrid((long)N * H * W * (Cu + Cs) / 8)), dim3(256), 0, s, d, e, N, H,
                       W, Cu, Cs, cat);
  else
    hipLaunchKernelGGL(up_concat_kernel, dim3(egrid((long)N * H * W * (Cu + Cs))), dim3(256), 0, s, d, e, N, H, W, Cu,
                       Cs, cat);
  return hipGetLastError();
}

hipError_t up_concat_bwd(const uint16_t* gcat, const uint16_t* dmask, const uint16_t* emask, int N, int H, int W,
                         int Cu, int Cs, uint16_t* gd, uint16_t* ge, hipStream_t s) {
  hipLaunchKernelGGL(up_concat_bwd_kernel, dim3(egrid((long)N * H * W * (Cu + Cs))), dim3(256), 0, s, gcat, dmask,
                     emask, N, H, W, Cu, Cs, gd, ge);
  return hipGetLastError();
}

hipError_t loss(const float* out, int Cpad, const float* tMx, const float* tMy, const float* ta, float s_flux,
                float s_dual, long P, uint16_t* gout, double* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, s, out, Cpad, tMx, tMy, ta, s_flux, s_dual, P, gout,
                     part);
  return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                float c1, float c2, uint16_t* pbf, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(egrid(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2, pbf);
  return hipGetLastError();
}

hipError_t to_bf16(const float* x, long n, uint16_t* y, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(egrid(n)), dim3(256), 0, s, x, n, y);
  return hipGetLastError();
}

hipError_t flip_weights(const uint16_t* w, int Cout, int Cin, uint16_t* wt, hipStream_t s) {
  hipLaunchKernelGGL(flip_weights_kernel, dim3(egrid((long)Cout * 9 * Cin)), dim3(256), 0, s, w, Cout, Cin, wt);
  return hipGetLastError();
}

hipError_t head_to_state(const float* out, int Cpad, int H, int W, long P, float s_flux, float s_dual, float* Mx,
                         float* My, float* a, hipStream_t s) {
  hipLaunchKernelGGL(head_to_state_kernel, dim3(egrid(P)), dim3(256), 0, s, out, Cpad, H, W, P, s_flux, s_dual, Mx,
                     My, a);
  return hipGetLastError();
}

hipError_t complete_residual(const float* Mx, const float* My, const float* src, const float* dst, int H, int W,
                             long P, float* r, hipStream_t s) {
  hipLaunchKernelGGL(complete_residual_kernel, dim3(egrid(P)), dim3(256), 0, s, Mx, My, src, dst, H, W, P, r);
  return hipGetLastError();
}

}  // namespace unet
