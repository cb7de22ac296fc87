// Internal declarations of the warm-start network kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace unet {

struct ConvArgs {
  const uint16_t* X;    // input NHWC bf16 [N][H][W][Cin], Cin % 8 == 0
  const uint16_t* Wt;   // weights bf16 [Cout][9][Cin]
  const float* bias;    // [Cout] or null
  uint16_t* Y;          // bf16 output [N][H][W][Cout] or null
  float* Yf;            // fp32 output or null
  const uint16_t* mask; // optional: zero the output where mask <= 0
  int N, H, W, Cin, Cout;
  int relu;
};

struct WgradArgs {
  const uint16_t* GY;   // output gradient bf16 [N][H][W][Cout], Cout % 8 == 0
  const uint16_t* X;    // forward input bf16 [N][H][W][Cin], Cin % 8 == 0
  float* part;          // [splits][Cout][9*Cin]
  int N, H, W, Cin, Cout;
};

hipError_t conv(const ConvArgs& a, hipStream_t s);
hipError_t wgrad(const WgradArgs& a, int splits, hipStream_t s);
hipError_t sum_splits(const float* part, int splits, long n, float* dst, int accumulate, hipStream_t s);
hipError_t bias_grad(const uint16_t* gy, long P, int C, float* part, int blocks, hipStream_t s);
hipError_t pack_input(const float* src, const float* dst, float scale, long P, int Cpad, uint16_t* X, hipStream_t s);
hipError_t pool2(const uint16_t* x, int N, int H, int W, int C, uint16_t* y, hipStream_t s);
hipError_t pool2_bwd(const uint16_t* gy, const uint16_t* mask, const uint16_t* add, int N, int H, int W, int C,
                     uint16_t* gx, hipStream_t s);
hipError_t up_concat(const uint16_t* d, const uint16_t* e, int N, int H, int W, int Cu, int Cs, uint16_t* cat,
                     hipStream_t s);
hipError_t up_concat_bwd(const uint16_t* gcat, const uint16_t* dmask, const uint16_t* emask, int N, int H, int W,
                         int Cu, int Cs, uint16_t* gd, uint16_t* ge, hipStream_t s);
hipError_t loss(const float* out, int Cpad, const float* tMx, const float* tMy, const float* ta, float s_flux,
                float s_dual, long P, uint16_t* gout, double* part, int blocks, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                float c1, float c2, uint16_t* pbf, hipStream_t s);
hipError_t to_bf16(const float* x, long n, uint16_t* y, hipStream_t s);
hipError_t flip_weights(const uint16_t* w, int Cout, int Cin, uint16_t* wt, hipStream_t s);
hipError_t head_to_state(const float* out, int Cpad, int H, int W, long P, float s_flux, float s_dual, float* Mx,
                         float* My, float* a, hipStream_t s);
hipError_t complete_residual(const float* Mx, const float* My, const float* src, const float* dst, int H, int W,
                             long P, float* r, hipStream_t s);

}  // namespace unet
