// Host runtime of the warm-start network: parameter layout, buffers, the
// forward / backward schedule of the U-Net, Adam, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/uotnet.h"
#include "uotnet_internal.hpp"

using namespace unet;

namespace {

#define NCHK(x)                                                              \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? UOT_ERR_OOM : UOT_ERR_DEVICE; \
  } while (0)

int pad8(int c) { return (c + 7) / 8 * 8; }

struct Conv {
  std::string name;
  int cin, cout;    // real channel counts (host layout)
  int cinp, coutp;  // padded to multiples of 8 (device layout)
  int level;
  bool relu;
  long woff, boff;  // offsets in the flat device parameter vector
};

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

}  // namespace

struct uotnet {
  uotnet_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int L = 4;
  std::vector<int> ch;
  std::vector<Conv> convs;
  long np = 0;                  // flat (padded) parameter count
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t* pbf = nullptr;      // bf16 copy of p
  uint16_t* wt = nullptr;       // flipped weights, same offsets as p
  int step = 0;
  // activations, per level l: enc a_l, e_l, pooled input p_l; decoder cat_l, b_l, d_l
  uint16_t* x0 = nullptr;
  std::vector<uint16_t*> a, e, pl, cat, bdec, d, gskip;
  float* out = nullptr;
  uint16_t *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *gout = nullptr;
  float* wpart = nullptr;
  size_t wpart_n = 0;
  float* bpart = nullptr;
  double* lpart = nullptr;
  double* h_lpart = nullptr;
  std::vector<void*> owned;

  long P(int l, int B) const { return (long)B * (cfg.height >> l) * (cfg.width >> l); }
  int H(int l) const { return cfg.height >> l; }
  int W(int l) const { return cfg.width >> l; }

  ~uotnet() {
    for (void* q : owned)
      if (q) (void)hipFree(q);
    if (h_lpart) (void)hipHostFree(h_lpart);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

constexpr int kCin = 16;    // input channels on the device (2 used)
constexpr int kCout = 8;    // head output channels on the device (3 used)
constexpr int kBiasBlocks = 256;
constexpr int kLossBlocks = 512;

template <class T>
uot_status own(uotnet* n, T** ptr, size_t count) {
  NCHK(dalloc(ptr, count));
  n->owned.push_back(*ptr);
  return UOT_OK;
}

void build_layers(uotnet* n) {
  const int L = n->L;
  auto add = [&](const std::string& nm, int ci, int co, int lvl, bool relu, int cip, int cop) {
    Conv c{nm, ci, co, cip, cop, lvl, relu, 0, 0};
    n->convs.push_back(c);
  };
  add("enc0a", 2, n->ch[0], 0, true, kCin, pad8(n->ch[0]));
  add("enc0b", n->ch[0], n->ch[0], 0, true, pad8(n->ch[0]), pad8(n->ch[0]));
  for (int l = 1; l < L; ++l) {
    add("enc" + std::to_string(l) + "a", n->ch[l - 1], n->ch[l], l, true, n->ch[l - 1], n->ch[l]);
    add("enc" + std::to_string(l) + "b", n->ch[l], n->ch[l], l, true, n->ch[l], n->ch[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    add("dec" + std::to_string(l) + "a", n->ch[l + 1] + n->ch[l], n->ch[l], l, true, n->ch[l + 1] + n->ch[l], n->ch[l]);
    add("dec" + std::to_string(l) + "b", n->ch[l], n->ch[l], l, true, n->ch[l], n->ch[l]);
  }
  add("head", n->ch[0], 3, 0, false, n->ch[0], kCout);
  long off = 0;
  for (Conv& c : n->convs) {
    c.woff = off;
    off += (long)c.coutp * 9 * c.cinp;
    c.boff = off;
    off += c.coutp;
  }
  n->np = off;
}

const Conv& layer(const uotnet* n, const std::string& nm) {
  for (const Conv& c : n->convs)
    if (c.name == nm) return c;
  return n->convs[0];
}

// regenerate the bf16 copy and the flipped weights from the FP32 master
uot_status refresh_weights(uotnet* n) {
  NCHK(to_bf16(n->p, n->np, n->pbf, n->stream));
  for (const Conv& c : n->convs) NCHK(flip_weights(n->pbf + c.woff, c.coutp, c.cinp, n->wt + c.woff, n->stream));
  return UOT_OK;
}

uot_status conv_fwd(uotnet* n, const Conv& c, int B, const uint16_t* X, uint16_t* Y, float* Yf) {
  ConvArgs a{X, n->pbf + c.woff, n->p + c.boff, Y, Yf, nullptr, B, n->H(c.level), n->W(c.level), c.cinp, c.coutp,
             c.relu ? 1 : 0};
  NCHK(conv(a, n->stream));
  return UOT_OK;
}

// weight and bias gradients of conv c for output gradient gz (pre-activation)
uot_status conv_wgrad(uotnet* n, const Conv& c, int B, const uint16_t* gz, const uint16_t* X) {
  const long P = n->P(c.level, B);
  const int blocks_xy = ((9 * c.cinp + 63) / 64) * ((c.coutp + 63) / 64);
  int splits = std::max(1, std::min<int>(2048 / std::max(1, blocks_xy), (int)(P / 1024)));
  const long nel = (long)c.coutp * 9 * c.cinp;
  splits = std::max(1, std::min<int>(splits, (int)(n->wpart_n / nel)));
  WgradArgs w{gz, X, n->wpart, B, n->H(c.level), n->W(c.level), c.cinp, c.coutp};
  NCHK(wgrad(w, splits, n->stream));
  NCHK(sum_splits(n->wpart, splits, nel, n->g + c.woff, 0, n->stream));
  NCHK(bias_grad(gz, P, c.coutp, n->bpart, kBiasBlocks, n->stream));
  NCHK(sum_splits(n->bpart, kBiasBlocks, c.coutp, n->g + c.boff, 0, n->stream));
  return UOT_OK;
}

// input gradient of conv c; mask = the ReLU output that fed c (or null)
uot_status conv_dgrad(uotnet* n, const Conv& c, int B, const uint16_t* gz, const uint16_t* mask, uint16_t* gx) {
  ConvArgs a{gz, n->wt + c.woff, nullptr, gx, nullptr, mask, B, n->H(c.level), n->W(c.level), c.coutp, c.cinp, 0};
  NCHK(conv(a, n->stream));
  return UOT_OK;
}

uot_status forward(uotnet* n, int B, const float* src, const float* dst, float in_scale) {
  const int L = n->L;
  NCHK(pack_input(src, dst, in_scale, n->P(0, B), kCin, n->x0, n->stream));
  for (int l = 0; l < L; ++l) {
    const uint16_t* in = n->x0;
    if (l > 0) {
      NCHK(pool2(n->e[l - 1], B, n->H(l - 1), n->W(l - 1), n->ch[l - 1], n->pl[l], n->stream));
      in = n->pl[l];
    }
    uot_status s = conv_fwd(n, layer(n, "enc" + std::to_string(l) + "a"), B, in, n->a[l], nullptr);
    if (s != UOT_OK) return s;
    s = conv_fwd(n, layer(n, "enc" + std::to_string(l) + "b"), B, n->a[l], n->e[l], nullptr);
    if (s != UOT_OK) return s;
  }
  const uint16_t* dd = n->e[L - 1];
  for (int l = L - 2; l >= 0; --l) {
    NCHK(up_concat(dd, n->e[l], B, n->H(l), n->W(l), n->ch[l + 1], n->ch[l], n->cat[l], n->stream));
    uot_status s = conv_fwd(n, layer(n, "dec" + std::to_string(l) + "a"), B, n->cat[l], n->bdec[l], nullptr);
    if (s != UOT_OK) return s;
    s = conv_fwd(n, layer(n, "dec" + std::to_string(l) + "b"), B, n->bdec[l], n->d[l], nullptr);
    if (s != UOT_OK) return s;
    dd = n->d[l];
  }
  return conv_fwd(n, layer(n, "head"), B, n->d[0], nullptr, n->out);
}

uot_status backward(uotnet* n, int B) {
  const int L = n->L;
  uint16_t* buf[3] = {n->g1, n->g2, n->g3};
  int cur = 0;
  auto next = [&]() { cur = (cur + 1) % 3; return buf[cur]; };
  const Conv& head = layer(n, "head");
  uot_status s = conv_wgrad(n, head, B, n->gout, n->d[0]);
  if (s != UOT_OK) return s;
  uint16_t* gz = buf[cur];
  s = conv_dgrad(n, head, B, n->gout, n->d[0], gz);
  if (s != UOT_OK) return s;
  for (int l = 0; l <= L - 2; ++l) {
    const Conv& cb = layer(n, "dec" + std::to_string(l) + "b");
    const Conv& ca = layer(n, "dec" + std::to_string(l) + "a");
    s = conv_wgrad(n, cb, B, gz, n->bdec[l]);
    if (s != UOT_OK) return s;
    uint16_t* ga = next();
    s = conv_dgrad(n, cb, B, gz, n->bdec[l], ga);
    if (s != UOT_OK) return s;
    s = conv_wgrad(n, ca, B, ga, n->cat[l]);
    if (s != UOT_OK) return s;
    uint16_t* gcat = next();
    s = conv_dgrad(n, ca, B, ga, nullptr, gcat);
    if (s != UOT_OK) return s;
    const uint16_t* dmask = (l + 1 == L - 1) ? n->e[L - 1] : n->d[l + 1];
    uint16_t* gd = next();
    NCHK(up_concat_bwd(gcat, dmask, n->e[l], B, n->H(l), n->W(l), n->ch[l + 1], n->ch[l], gd, n->gskip[l],
                       n->stream));
    gz = gd;
  }
  for (int l = L - 1; l >= 0; --l) {
    const Conv& cb = layer(n, "enc" + std::to_string(l) + "b");
    const Conv& ca = layer(n, "enc" + std::to_string(l) + "a");
    s = conv_wgrad(n, cb, B, gz, n->a[l]);
    if (s != UOT_OK) return s;
    uint16_t* ga = next();
    s = conv_dgrad(n, cb, B, gz, n->a[l], ga);
    if (s != UOT_OK) return s;
    const uint16_t* in = l > 0 ? n->pl[l] : n->x0;
    s = conv_wgrad(n, ca, B, ga, in);
    if (s != UOT_OK) return s;
    if (l > 0) {
      uint16_t* gp = next();
      s = conv_dgrad(n, ca, B, ga, nullptr, gp);
      if (s != UOT_OK) return s;
      uint16_t* ge = next();
      NCHK(pool2_bwd(gp, n->e[l - 1], n->gskip[l - 1], B, n->H(l - 1), n->W(l - 1), n->ch[l - 1], ge, n->stream));
      gz = ge;
    }
  }
  return UOT_OK;
}

uot_status alloc_all(uotnet* n) {
  const int L = n->L, B = n->cfg.batch_max;
  uot_status s;
#define OWN(ptr, cnt)              \
  do {                             \
    s = own(n, &(ptr), (cnt));     \
    if (s != UOT_OK) return s;     \
  } while (0)
  OWN(n->p, n->np);
  OWN(n->m, n->np);
  OWN(n->v, n->np);
  OWN(n->g, n->np);
  OWN(n->pbf, n->np);
  OWN(n->wt, n->np);
  OWN(n->x0, n->P(0, B) * kCin);
  n->a.assign(L, nullptr);
  n->e.assign(L, nullptr);
  n->pl.assign(L, nullptr);
  n->cat.assign(L, nullptr);
  n->bdec.assign(L, nullptr);
  n->d.assign(L, nullptr);
  n->gskip.assign(L, nullptr);
  size_t gmax = (size_t)n->P(0, B) * kCin;
  for (int l = 0; l < L; ++l) {
    OWN(n->a[l], n->P(l, B) * n->ch[l]);
    OWN(n->e[l], n->P(l, B) * n->ch[l]);
    gmax = std::max<size_t>(gmax, (size_t)n->P(l, B) * n->ch[l]);
    if (l > 0) {
      OWN(n->pl[l], n->P(l, B) * n->ch[l - 1]);
      gmax = std::max<size_t>(gmax, (size_t)n->P(l, B) * n->ch[l - 1]);
    }
    if (l < L - 1) {
      const int cc = n->ch[l + 1] + n->ch[l];
      OWN(n->cat[l], n->P(l, B) * cc);
      OWN(n->bdec[l], n->P(l, B) * n->ch[l]);
      OWN(n->d[l], n->P(l, B) * n->ch[l]);
      OWN(n->gskip[l], n->P(l, B) * n->ch[l]);
      gmax = std::max<size_t>(gmax, (size_t)n->P(l, B) * cc);
    }
  }
  OWN(n->g1, gmax);
  OWN(n->g2, gmax);
  OWN(n->g3, gmax);
  OWN(n->gout, n->P(0, B) * kCout);
  OWN(n->out, n->P(0, B) * kCout);
  size_t wmax = 0;
  for (const Conv& c : n->convs) wmax = std::max<size_t>(wmax, (size_t)c.coutp * 9 * c.cinp);
  n->wpart_n = wmax * 64;
  OWN(n->wpart, n->wpart_n);
  OWN(n->bpart, (size_t)kBiasBlocks * 256);
  OWN(n->lpart, kLossBlocks);
#undef OWN
  NCHK(hipHostMalloc((void**)&n->h_lpart, kLossBlocks * sizeof(double), hipHostMallocDefault));
  return UOT_OK;
}

// host layout <-> padded device layout
void to_host_layout(const uotnet* n, const std::vector<float>& dev, float* host) {
  long o = 0;
  for (const Conv& c : n->convs) {
    for (int co = 0; co < c.cout; ++co)
      for (int t = 0; t < 9; ++t)
        for (int ci = 0; ci < c.cin; ++ci) host[o++] = dev[c.woff + ((long)co * 9 + t) * c.cinp + ci];
    for (int co = 0; co < c.cout; ++co) host[o++] = dev[c.boff + co];
  }
}

void to_dev_layout(const uotnet* n, const float* host, std::vector<float>& dev) {
  dev.assign(n->np, 0.f);
  long o = 0;
  for (const Conv& c : n->convs) {
    for (int co = 0; co < c.cout; ++co)
      for (int t = 0; t < 9; ++t)
        for (int ci = 0; ci < c.cin; ++ci) dev[c.woff + ((long)co * 9 + t) * c.cinp + ci] = host[o++];
    for (int co = 0; co < c.cout; ++co) dev[c.boff + co] = host[o++];
  }
}

long host_count(const uotnet* n) {
  long o = 0;
  for (const Conv& c : n->convs) o += (long)c.cout * 9 * c.cin + c.cout;
  return o;
}

}  // namespace

extern "C" {

uot_status uotnet_create(const uotnet_config* cfg, void* hip_stream, uotnet** out) {
  if (!cfg || !out) return UOT_ERR_ARG;
  *out = nullptr;
  if (cfg->levels < 2 || cfg->levels > 4 || cfg->batch_max < 1) return UOT_ERR_ARG;
  for (int l = 0; l < cfg->levels; ++l)
    if (cfg->ch[l] < 8 || cfg->ch[l] % 8 != 0) return UOT_ERR_ARG;
  const int f = 1 << (cfg->levels - 1);
  if (cfg->height < f || cfg->width < f || cfg->height % f || cfg->width % f) return UOT_ERR_SHAPE;
  auto* n = new (std::nothrow) uotnet();
  if (!n) return UOT_ERR_OOM;
  n->cfg = *cfg;
  n->L = cfg->levels;
  n->ch.assign(cfg->ch, cfg->ch + cfg->levels);
  if (hip_stream) {
    n->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&n->stream) != hipSuccess) {
      delete n;
      return UOT_ERR_DEVICE;
    }
    n->own_stream = true;
  }
  build_layers(n);
  uot_status s = alloc_all(n);
  if (s != UOT_OK) {
    delete n;
    return s;
  }
  // He-normal weights in the host layout, zero biases
  std::vector<float> host(host_count(n));
  std::mt19937_64 rng(cfg->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  long o = 0;
  for (const Conv& c : n->convs) {
    const double sd = std::sqrt(2.0 / (9.0 * c.cin));
    for (long i = 0; i < (long)c.cout * 9 * c.cin; ++i) host[o++] = (float)(sd * nd(rng));
    for (int i = 0; i < c.cout; ++i) host[o++] = 0.f;
  }
  s = uotnet_set_params(n, host.data(), (int64_t)host.size());
  if (s != UOT_OK) {
    delete n;
    return s;
  }
  *out = n;
  return UOT_OK;
}

void uotnet_destroy(uotnet* net) { delete net; }

int64_t uotnet_num_params(const uotnet* net) { return net ? host_count(net) : -1; }

uot_status uotnet_get_params(uotnet* n, float* host, int64_t cnt) {
  if (!n || !host || cnt != host_count(n)) return UOT_ERR_ARG;
  std::vector<float> dev(n->np);
  NCHK(hipMemcpyAsync(dev.data(), n->p, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  to_host_layout(n, dev, host);
  return UOT_OK;
}

uot_status uotnet_get_grads(uotnet* n, float* host, int64_t cnt) {
  if (!n || !host || cnt != host_count(n)) return UOT_ERR_ARG;
  std::vector<float> dev(n->np);
  NCHK(hipMemcpyAsync(dev.data(), n->g, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  to_host_layout(n, dev, host);
  return UOT_OK;
}

uot_status uotnet_set_params(uotnet* n, const float* host, int64_t cnt) {
  if (!n || !host || cnt != host_count(n)) return UOT_ERR_ARG;
  std::vector<float> dev;
  to_dev_layout(n, host, dev);
  NCHK(hipMemcpyAsync(n->p, dev.data(), n->np * sizeof(float), hipMemcpyHostToDevice, n->stream));
  NCHK(hipMemsetAsync(n->m, 0, n->np * sizeof(float), n->stream));
  NCHK(hipMemsetAsync(n->v, 0, n->np * sizeof(float), n->stream));
  NCHK(hipMemsetAsync(n->g, 0, n->np * sizeof(float), n->stream));
  n->step = 0;
  uot_status s = refresh_weights(n);
  if (s != UOT_OK) return s;
  NCHK(hipStreamSynchronize(n->stream));
  return UOT_OK;
}

uot_status uotnet_warm_state(uotnet* n, int32_t B, const float* src, const float* dst, float in_scale, float s_flux,
                             float s_dual, uot_state* st) {
  if (!n || !src || !dst || !st || !st->Mx || !st->My || !st->a || !st->r) return UOT_ERR_ARG;
  if (B < 1 || B > n->cfg.batch_max) return UOT_ERR_SHAPE;
  if (!(s_flux > 0.f) || !(s_dual > 0.f)) return UOT_ERR_ARG;
  uot_status s = forward(n, B, src, dst, in_scale);
  if (s != UOT_OK) return s;
  const long P = n->P(0, B);
  NCHK(head_to_state(n->out, kCout, n->cfg.height, n->cfg.width, P, s_flux, s_dual, st->Mx, st->My, st->a, n->stream));
  NCHK(complete_residual(st->Mx, st->My, src, dst, n->cfg.height, n->cfg.width, P, st->r, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  return UOT_OK;
}

uot_status uotnet_train_step(uotnet* n, int32_t B, const float* src, const float* dst, float in_scale,
                             const float* tMx, const float* tMy, const float* ta, float s_flux, float s_dual, float lr,
                             double* loss_out) {
  if (!n || !src || !dst || !tMx || !tMy || !ta || !(lr >= 0.f)) return UOT_ERR_ARG;
  if (B < 1 || B > n->cfg.batch_max) return UOT_ERR_SHAPE;
  uot_status s = forward(n, B, src, dst, in_scale);
  if (s != UOT_OK) return s;
  const long P = n->P(0, B);
  NCHK(loss(n->out, kCout, tMx, tMy, ta, s_flux, s_dual, P, n->gout, n->lpart, kLossBlocks, n->stream));
  NCHK(hipMemcpyAsync(n->h_lpart, n->lpart, kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, n->stream));
  s = backward(n, B);
  if (s != UOT_OK) return s;
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
  NCHK(adam(n->p, n->g, n->m, n->v, n->np, lr, b1, b2, 1e-8f, c1, c2, n->pbf, n->stream));
  for (const Conv& c : n->convs) NCHK(flip_weights(n->pbf + c.woff, c.coutp, c.cinp, n->wt + c.woff, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  if (loss_out) {
    double acc = 0.0;
    for (int i = 0; i < kLossBlocks; ++i) acc += n->h_lpart[i];
    *loss_out = acc;
  }
  return UOT_OK;
}

uot_status uotnet_conv(int32_t op, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout, const uint16_t* X,
                       const uint16_t* Wt, const uint16_t* G, const float* bias, int32_t relu, float* out,
                       void* hip_stream) {
  if (N < 1 || H < 1 || W < 1 || Cin < 8 || Cout < 8 || Cin % 8 || Cout % 8 || !out) return UOT_ERR_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  if (op == 0) {
    if (!X || !Wt) return UOT_ERR_ARG;
    ConvArgs a{X, Wt, bias, nullptr, out, nullptr, N, H, W, Cin, Cout, relu ? 1 : 0};
    NCHK(conv(a, s));
  } else if (op == 1) {
    if (!G || !Wt) return UOT_ERR_ARG;
    uint16_t* wt = nullptr;
    NCHK(hipMalloc((void**)&wt, (size_t)Cout * 9 * Cin * sizeof(uint16_t)));
    hipError_t e = flip_weights(Wt, Cout, Cin, wt, s);
    ConvArgs a{G, wt, nullptr, nullptr, out, nullptr, N, H, W, Cout, Cin, 0};
    if (e == hipSuccess) e = conv(a, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(wt);
    NCHK(e);
  } else if (op == 2) {
    if (!G || !X) return UOT_ERR_ARG;
    const long P = (long)N * H * W;
    const long nel = (long)Cout * 9 * Cin;
    const int splits = (int)std::max<long>(1, std::min<long>(32, P / 256));
    float* part = nullptr;
    NCHK(hipMalloc((void**)&part, (size_t)splits * nel * sizeof(float)));
    WgradArgs w{G, X, part, N, H, W, Cin, Cout};
    hipError_t e = wgrad(w, splits, s);
    if (e == hipSuccess) e = sum_splits(part, splits, nel, out, 0, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    NCHK(e);
  } else {
    return UOT_ERR_ARG;
  }
  NCHK(hipStreamSynchronize(s));
  return UOT_OK;
}

}  // extern "C"
