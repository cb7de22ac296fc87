// Host runtime of the ADMM solvers that call the UOT prox (C ABI of
// include/uot_admm.h).
//
// UOT-DF (Sec. IV-A, Algorithm 2).  One ADMM iteration is three groups of
// launches on the handle's stream: the element-wise s/x/centre step, the
// prox passes (the fused Algorithm-1 kernel in the one-argument-fixed mode,
// warm-started: its state stays on the device between ADMM iterations), and
// the element-wise multiplier step.  A check window of ADMM iterations is
// captured once as a HIP graph and replayed; on the window's last iteration
// the element-wise kernels leave residual partials, one reduction adds them
// and three doubles come back to the host, which decides whether to stop.
// The prox state ping-pongs between two copies; a window flips the copy it
// ends in when it holds an odd number of prox launches, so graphs are kept
// for both starting copies.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "uot.h"
#include "uot_admm.h"
#include "uot_admm_internal.hpp"

using namespace uot;

namespace {

#define DFCHK(x)                          \
  do {                                    \
    if ((x) != hipSuccess) return UOT_ERR_DEVICE; \
  } while (0)

constexpr int NPLANES = 5;  // prox state: Mx, My, r, a (prox dual), x1 (= z)

struct GraphSlot {
  hipGraphExec_t exec = nullptr;
  int W = -1;
  const void *y = nullptr, *phi = nullptr, *s0 = nullptr;
};

}  // namespace

struct uotdf_handle {
  uotdf_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;  // NULL was passed: a stream of our own (graphs cannot capture the null stream)
  int device = 0, num_cu = 256;
  long n = 0;
  int resid = R_P1;
  float *s = nullptr, *x = nullptr, *a = nullptr, *b = nullptr, *p = nullptr, *zo = nullptr;
  float* st[2][NPLANES] = {};
  PairInfo* d_pair = nullptr;
  Tile* d_tiles = nullptr;
  int32_t* d_ntiles = nullptr;
  int32_t* d_active = nullptr;
  int ntiles = 0, shape = 4, T = 1, grid = 8, launches_per_iter = 1;
  double* d_partial = nullptr;
  double* d_sums = nullptr;
  double* h_sums = nullptr;  // pinned
  int nblocks = 1;
  int parity = 0;            // copy holding the current prox state
  GraphSlot graphs[2];
  hipEvent_t e0 = nullptr, e1 = nullptr;

  ~uotdf_handle() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (float* q : {s, x, a, b, p, zo})
      if (q) (void)hipFree(q);
    for (auto& c : st)
      for (float* q : c)
        if (q) (void)hipFree(q);
    if (d_pair) (void)hipFree(d_pair);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_ntiles) (void)hipFree(d_ntiles);
    if (d_active) (void)hipFree(d_active);
    if (d_partial) (void)hipFree(d_partial);
    if (d_sums) (void)hipFree(d_sums);
    if (h_sums) (void)hipHostFree(h_sums);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

Planes prox_planes(uotdf_handle* h, int c) {
  float** q = h->st[c];
  return Planes{q[0], q[1], h->prm.balanced ? nullptr : q[2], q[3], nullptr, q[4]};
}

DfArgs df_args(uotdf_handle* h, const float* y, const float* phi, bool record) {
  const uotdf_params& P = h->prm;
  return DfArgs{h->n, y, phi, h->s, h->x, h->a, h->b, h->p, h->zo, h->st[h->parity][4], (float)P.rho,
                (float)(P.lam / (2.0 * P.rho)), record ? 1 : 0, h->d_partial};
}

// The prox passes of one ADMM iteration (Algorithm 1 in the one-argument-
// fixed mode, warm-started from the state copy of the current parity).
uot_status enqueue_prox(uotdf_handle* h, const float* s0) {
  const uotdf_params& P = h->prm;
  for (int left = P.prox_iters; left > 0;) {
    const int k = std::min(h->T, left);
    IterArgs it{prox_planes(h, h->parity), prox_planes(h, h->parity ^ 1), nullptr, s0, h->p, h->d_pair,
                h->d_tiles, h->d_ntiles, h->d_active, k};
    DFCHK(launch_iter(UOT_PROX_FIXED, h->resid, P.bc, h->shape, h->grid, it, h->stream));
    h->parity ^= 1;
    left -= k;
  }
  return UOT_OK;
}

// W ADMM iterations with residual partials on the last, then the reduction
// and the copy of the three sums to the host (not waited for).
uot_status enqueue_window(uotdf_handle* h, int W, const float* y, const float* phi, const float* s0) {
  // s- and x-steps of the first iteration; then per iteration the prox
  // passes and the multiplier steps, fused with the next iteration's s- and
  // x-steps inside the window
  DFCHK(launch_df_sx(df_args(h, y, phi, W == 1), h->stream));
  for (int i = 0; i < W; ++i) {
    uot_status s = enqueue_prox(h, s0);
    if (s != UOT_OK) return s;
    if (i + 1 < W) DFCHK(launch_df_absx(df_args(h, y, phi, i + 2 == W), h->stream));
    else DFCHK(launch_df_ab(df_args(h, y, phi, true), h->stream));
  }
  DFCHK(launch_df_reduce(h->d_partial, h->nblocks, h->d_sums, h->stream));
  DFCHK(hipMemcpyAsync(h->h_sums, h->d_sums, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  return UOT_OK;
}

uot_status run_window(uotdf_handle* h, int W, const float* y, const float* phi, const float* s0, bool use_graph) {
  if (!use_graph) return enqueue_window(h, W, y, phi, s0);
  const int start = h->parity;
  GraphSlot& g = h->graphs[start];
  if (!(g.exec && g.W == W && g.y == y && g.phi == phi && g.s0 == s0)) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipGraph_t graph = nullptr;
    DFCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    uot_status st = enqueue_window(h, W, y, phi, s0);
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (st != UOT_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      h->parity = start;
      return st != UOT_OK ? st : UOT_ERR_DEVICE;
    }
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      h->parity = start;
      return UOT_ERR_DEVICE;
    }
    g.W = W;
    g.y = y;
    g.phi = phi;
    g.s0 = s0;
    // capturing advanced the host's parity bookkeeping; the replay below does it again
    h->parity = start;
  }
  DFCHK(hipGraphLaunch(g.exec, h->stream));
  if ((W * h->launches_per_iter) & 1) h->parity ^= 1;
  return UOT_OK;
}

double elapsed_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

uot_status uotdf_check_params(const uotdf_params* p) {
  if (!p) return UOT_ERR_ARG;
  if (p->nx < 1 || p->ny < 1) return UOT_ERR_SHAPE;
  if (!(p->kappa > 0.0) || !(p->rho > 0.0) || !(p->lam >= 0.0) || !std::isfinite(p->kappa) ||
      !std::isfinite(p->rho) || !std::isfinite(p->lam) || !std::isfinite(p->eps))
    return UOT_ERR_ARG;
  if (!p->balanced && (!(p->mu > 0.0) || !std::isfinite(p->mu))) return UOT_ERR_ARG;
  if (p->residual_p != 1 && p->residual_p != 2) return UOT_ERR_ARG;
  if (p->bc != 0 && p->bc != 1) return UOT_ERR_ARG;
  if (p->prox_iters < 1 || p->max_iter < 1 || p->check_every < 1) return UOT_ERR_ARG;
  if (!(p->prox_tau_ratio >= 0.0) || !std::isfinite(p->prox_tau_ratio)) return UOT_ERR_ARG;
  return UOT_OK;
}

uot_status uotdf_create(const uotdf_params* prm, void* hip_stream, uotdf_handle** out) {
  if (!out) return UOT_ERR_ARG;
  *out = nullptr;
  uot_status s = uotdf_check_params(prm);
  if (s != UOT_OK) return s;
  uotdf_handle* h = new (std::nothrow) uotdf_handle();
  if (!h) return UOT_ERR_OOM;
  h->prm = *prm;
  h->n = (long)prm->nx * prm->ny;
  h->resid = prm->balanced ? R_BAL : (prm->residual_p == 2 ? R_P2 : R_P1);
  auto fail = [&](uot_status e) {
    delete h;
    return e;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return fail(UOT_ERR_DEVICE);
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess) return fail(UOT_ERR_DEVICE);
    h->own_stream = true;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cu > 0)
    h->num_cu = cu;
  const size_t bytes = (size_t)h->n * sizeof(float);
  for (float** q : {&h->s, &h->x, &h->a, &h->b, &h->p, &h->zo})
    if (hipMalloc((void**)q, bytes) != hipSuccess) return fail(UOT_ERR_OOM);
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < NPLANES; ++k)
      if (hipMalloc((void**)&h->st[c][k], bytes) != hipSuccess) return fail(UOT_ERR_OOM);

  // the prox as one Algorithm-1 pair: fixed argument s0, step kappa / rho
  const double k2 = uot_knorm2(prm->nx, prm->ny, UOT_PROX_FIXED, prm->balanced, prm->bc);
  const double t = 0.99 / std::sqrt(k2);
  const double rr = prm->prox_tau_ratio > 0.0 ? std::sqrt(prm->prox_tau_ratio) : 1.0;
  const double t1 = t * rr, t2 = t / rr;  // tau1 tau2 ||K||^2 = 0.98 whatever the ratio
  const double rho_prox = prm->kappa / prm->rho;
  // kernel shape: one pass per ADMM iteration -> the single-step kernel;
  // several -> the temporally blocked kernel, up to 4 passes per launch
  if (prm->prox_iters == 1) {
    h->shape = h->n <= (1L << 16) ? 4 : 116;
    h->T = 1;
  } else {
    h->shape = h->n <= (1L << 18) ? 4008 : 4016;
    h->T = 4;
  }
  h->launches_per_iter = (prm->prox_iters + h->T - 1) / h->T;
  const int rows = h->shape >= 1000 ? h->shape % 1000 : h->shape % 100;
  std::vector<Tile> tiles;
  for (int y = 0; y < prm->ny; y += rows)
    for (int x = 0; x < prm->nx; x += TX) tiles.push_back(Tile{0, x, y, (int32_t)tiles.size()});
  h->ntiles = (int)tiles.size();
  PairInfo P{};
  P.off = 0;
  P.nx = prm->nx;
  P.ny = prm->ny;
  P.tau1 = (float)t1;
  P.tau2 = (float)t2;
  P.theta = (float)(t1 / (rho_prox + t1));
  P.mutau = (float)(prm->mu * t1);
  P.inv2mt = (float)(1.0 / (1.0 + 2.0 * prm->mu * t1));
  P.tile_begin = 0;
  P.tile_count = h->ntiles;
  P.pitch = prm->nx;
  const int32_t one = 1;
  if (hipMalloc((void**)&h->d_pair, sizeof(PairInfo)) != hipSuccess ||
      hipMalloc((void**)&h->d_tiles, tiles.size() * sizeof(Tile)) != hipSuccess ||
      hipMalloc((void**)&h->d_ntiles, sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void**)&h->d_active, sizeof(int32_t)) != hipSuccess)
    return fail(UOT_ERR_OOM);
  if (hipMemcpy(h->d_pair, &P, sizeof(PairInfo), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_ntiles, &h->ntiles, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_active, &one, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return fail(UOT_ERR_DEVICE);
  int occ = 0;
  if (iter_occupancy(UOT_PROX_FIXED, h->resid, prm->bc, h->shape, &occ) != hipSuccess || occ <= 0) occ = 2;
  long g = std::min<long>(h->ntiles, (long)h->num_cu * occ);
  h->grid = (int)std::max<long>(8, (g + 7) / 8 * 8);
  h->nblocks = df_blocks(h->n);
  if (hipMalloc((void**)&h->d_partial, 3 * (size_t)h->nblocks * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_sums, 3 * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&h->h_sums, 3 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(UOT_ERR_OOM);
  if (hipEventCreate(&h->e0) != hipSuccess || hipEventCreate(&h->e1) != hipSuccess) return fail(UOT_ERR_DEVICE);
  *out = h;
  return UOT_OK;
}

uot_status uotdf_solve(uotdf_handle* h, const float* y, const float* phi, const float* s0, float* s_out,
                       uotdf_report* rep) {
  if (!h || !y || !s0 || !s_out || !rep) return UOT_ERR_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  const uotdf_params& P = h->prm;
  std::memset(rep, 0, sizeof(*rep));
  if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
  // inputs: finite, s0 >= 0
  DFCHK(launch_df_validate(h->n, y, phi, s0, h->d_partial, h->stream));
  DFCHK(launch_df_reduce(h->d_partial, h->nblocks, h->d_sums, h->stream));
  DFCHK(hipMemcpyAsync(h->h_sums, h->d_sums, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  if (h->h_sums[0] > 0.0) return UOT_ERR_NONFINITE;
  if (h->h_sums[1] > 0.0) return UOT_ERR_NEGATIVE;
  // every variable and the prox state start at zero (Algorithm 2)
  const size_t bytes = (size_t)h->n * sizeof(float);
  for (float* q : {h->s, h->x, h->a, h->b, h->p, h->zo}) DFCHK(hipMemsetAsync(q, 0, bytes, h->stream));
  for (auto& c : h->st)
    for (float* q : c) DFCHK(hipMemsetAsync(q, 0, bytes, h->stream));
  h->parity = 0;

  const bool use_graph = !(P.flags & UOT_NO_GRAPH);
  const int W = P.check_every;
  const int nwin = P.max_iter / W, tail = P.max_iter % W;
  int k = 0;
  bool conv = false;
  double rp = std::nan(""), rd = std::nan("");
  DFCHK(hipEventRecord(h->e0, h->stream));
  auto test = [&](int iters) -> uot_status {
    DFCHK(hipStreamSynchronize(h->stream));
    rp = std::sqrt(std::max(0.0, h->h_sums[0]));
    rd = P.rho * std::sqrt(std::max(0.0, h->h_sums[1] + h->h_sums[2]));
    k = iters;
    if (P.eps > 0.0 && rp < P.eps && rd < P.eps) conv = true;
    return UOT_OK;
  };
  for (int w = 0; w < nwin && !conv; ++w) {
    uot_status s = run_window(h, W, y, phi, s0, use_graph);
    if (s != UOT_OK) return s;
    s = test((w + 1) * W);
    if (s != UOT_OK) return s;
  }
  if (!conv && tail > 0) {
    uot_status s = enqueue_window(h, tail, y, phi, s0);
    if (s != UOT_OK) return s;
    s = test(P.max_iter);
    if (s != UOT_OK) return s;
  }
  DFCHK(hipEventRecord(h->e1, h->stream));
  DFCHK(hipMemcpyAsync(s_out, h->s, bytes, hipMemcpyDeviceToDevice, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  float ms = 0.f;
  DFCHK(hipEventElapsedTime(&ms, h->e0, h->e1));
  rep->iters = k;
  rep->converged = conv ? 1 : 0;
  rep->r_primal = rp;
  rep->r_dual = rd;
  rep->ms_per_iter = k > 0 ? (double)ms / k : 0.0;
  rep->seconds = elapsed_s(t0);
  return UOT_OK;
}

uot_status uotdf_copy_planes(uotdf_handle* h, float* x, float* z, float* a, float* b) {
  if (!h) return UOT_ERR_ARG;
  const size_t bytes = (size_t)h->n * sizeof(float);
  const float* src[4] = {h->x, h->st[h->parity][4], h->a, h->b};
  float* dst[4] = {x, z, a, b};
  for (int i = 0; i < 4; ++i)
    if (dst[i]) DFCHK(hipMemcpyAsync(dst[i], src[i], bytes, hipMemcpyDeviceToDevice, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

void uotdf_destroy(uotdf_handle* h) { delete h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// RPCA+UOT-DF (Sec. IV-B, Algorithm 3).  One ADMM iteration: rp_sx (the s-,
// L- and x-steps and the prox centres), the singular-value threshold of L + D (Gram
// matrix, its reduction, the warm-started Jacobi eigensolve, the apply with
// the D step), the prox passes of the T - 1 frame pairs (the fused
// Algorithm-1 kernel in the full-prox mode over a batch of pairs), and
// rp_dual (the multiplier steps).  Windows, graphs and the two prox-state copies as
// for UOT-DF.

namespace {
constexpr int RP_NPLANES = 6;  // prox state: Mx, My, r, a, x0 (= z), x1 (= w)
}

struct rpca_handle {
  rpca_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0, num_cu = 256;
  long npx = 0, n = 0, np1 = 0;  // pixels per frame, of all frames, of the pair frames
  int npairs = 1;                // T - 1, or 2 (T - 1) with the signed sparse part (+ pairs, then - pairs)
  int resid = R_P1;
  float *S = nullptr, *L = nullptr, *X = nullptr, *Tn = nullptr, *A = nullptr, *D = nullptr;
  float* Sm = nullptr;  // S- (signed sparse part only)
  float *B = nullptr, *C = nullptr, *P0 = nullptr, *P1 = nullptr, *zo = nullptr, *wo = nullptr;
  float* st[2][RP_NPLANES] = {};
  double *d_gpart = nullptr, *d_G = nullptr, *d_V = nullptr, *d_lam = nullptr;
  float* d_Wm = nullptr;
  int* d_sweeps = nullptr;
  int gblocks = 1;
  PairInfo* d_pairs = nullptr;
  Tile* d_tiles = nullptr;
  int32_t* d_ntiles = nullptr;
  int32_t* d_active = nullptr;
  int ntiles = 0, shape = 4, T = 1, grid = 8, launches_per_iter = 1;
  double* d_partial = nullptr;
  double* d_sums = nullptr;
  double* h_sums = nullptr;
  int bx = 1;       // pixel blocks per frame of the (bx, T) grids of rp_sx and rp_dual
  int sblocks = 1;  // blocks of the svt apply (64 pixels each per pass)
  int vblocks = 1;  // blocks of the input check
  int pstride = 1;  // partials per residual slot
  int parity = 0;
  GraphSlot graphs[2];
  hipEvent_t e0 = nullptr, e1 = nullptr;

  ~rpca_handle() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (float* q : {S, Sm, L, X, Tn, A, D, B, C, P0, P1, zo, wo, d_Wm})
      if (q) (void)hipFree(q);
    for (auto& c : st)
      for (float* q : c)
        if (q) (void)hipFree(q);
    for (double* q : {d_gpart, d_G, d_V, d_lam, d_partial, d_sums})
      if (q) (void)hipFree(q);
    if (d_sweeps) (void)hipFree(d_sweeps);
    if (d_pairs) (void)hipFree(d_pairs);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_ntiles) (void)hipFree(d_ntiles);
    if (d_active) (void)hipFree(d_active);
    if (h_sums) (void)hipHostFree(h_sums);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

Planes rp_planes(rpca_handle* h, int c) {
  float** q = h->st[c];
  return Planes{q[0], q[1], h->prm.balanced ? nullptr : q[2], q[3], q[4], q[5]};
}

RpArgs rp_args(rpca_handle* h, const float* y, const float* phi, bool record) {
  RpArgs a{};
  a.npx = h->npx;
  a.T = h->prm.frames;
  a.y = y;
  a.phi = phi;
  a.S = h->S;
  a.L = h->L;
  a.X = h->X;
  a.Tn = h->Tn;
  a.A = h->A;
  a.D = h->D;
  a.B = h->B;
  a.C = h->C;
  a.P0 = h->P0;
  a.P1 = h->P1;
  a.zo = h->zo;
  a.wo = h->wo;
  a.Z = h->st[h->parity][4];
  a.W = h->st[h->parity][5];
  a.rho = (float)h->prm.rho;
  a.lam = (float)h->prm.lam;
  a.record = record ? 1 : 0;
  a.partial = h->d_partial;
  a.Wm = h->d_Wm;
  a.pstride = h->pstride;
  a.Sm = h->Sm;
  a.mo = (long)(h->prm.frames - 1) * h->npx;
  return a;
}

// One ADMM iteration, i-th of a window of W.  The S-, L- and X-steps of
// the first iteration run alone; the multiplier steps of every other
// iteration run fused with the next iteration's S-, L- and X-steps, and
// the window's last multiplier steps alone with the residual partials.
uot_status rp_iteration(rpca_handle* h, const float* y, const float* phi, int i, int W) {
  const rpca_params& P = h->prm;
  const bool record = i == W - 1;
  RpArgs a = rp_args(h, y, phi, record);
  if (i == 0) DFCHK(launch_rp_sx(a, h->bx, h->stream));
  DFCHK(launch_rp_gram(a, h->gblocks, h->d_gpart, h->stream));
  DFCHK(launch_rp_gram_reduce(h->d_gpart, h->gblocks, P.frames, h->d_G, h->stream));
  DFCHK(launch_rp_eig(h->d_G, P.frames, P.gam / P.rho, h->d_V, h->d_lam, h->d_Wm, h->d_sweeps,
                      h->stream));
  DFCHK(launch_rp_svt_apply(a, h->sblocks, h->stream));
  for (int left = P.prox_iters; left > 0;) {
    const int k = std::min(h->T, left);
    IterArgs it{rp_planes(h, h->parity), rp_planes(h, h->parity ^ 1), nullptr, h->P0, h->P1, h->d_pairs,
                h->d_tiles, h->d_ntiles, h->d_active, k};
    DFCHK(launch_iter(UOT_PROX, h->resid, P.bc, h->shape, h->grid, it, h->stream));
    h->parity ^= 1;
    left -= k;
  }
  a.Z = h->st[h->parity][4];
  a.W = h->st[h->parity][5];
  if (record) {
    DFCHK(launch_rp_dual(a, h->bx, h->stream));
  } else {
    a.record = i + 1 == W - 1 ? 1 : 0;  // the next iteration's S/L/X part
    DFCHK(launch_rp_dualsx(a, h->bx, h->stream));
  }
  return UOT_OK;
}

// partials per residual slot after a recorded iteration (slots 0 and 4:
// rp_dual, 1: rp_sx, 2 and 3: the svt apply)
RpCounts rp_counts(const rpca_handle* h) {
  const int f = h->bx * h->prm.frames;
  return RpCounts{{f, f, h->sblocks, h->sblocks, f}};
}

uot_status rp_window(rpca_handle* h, int W, const float* y, const float* phi) {
  for (int i = 0; i < W; ++i) {
    uot_status s = rp_iteration(h, y, phi, i, W);
    if (s != UOT_OK) return s;
  }
  DFCHK(launch_rp_reduce(h->d_partial, h->pstride, rp_counts(h), h->d_sums, h->stream));
  DFCHK(hipMemcpyAsync(h->h_sums, h->d_sums, RP_SLOTS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  return UOT_OK;
}

uot_status rp_run_window(rpca_handle* h, int W, const float* y, const float* phi, bool use_graph) {
  if (!use_graph) return rp_window(h, W, y, phi);
  const int start = h->parity;
  GraphSlot& g = h->graphs[start];
  if (!(g.exec && g.W == W && g.y == y && g.phi == phi)) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipGraph_t graph = nullptr;
    DFCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    uot_status st = rp_window(h, W, y, phi);
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    h->parity = start;
    if (st != UOT_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return st != UOT_OK ? st : UOT_ERR_DEVICE;
    }
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return UOT_ERR_DEVICE;
    }
    g.W = W;
    g.y = y;
    g.phi = phi;
    g.s0 = nullptr;
  }
  DFCHK(hipGraphLaunch(g.exec, h->stream));
  if ((W * h->launches_per_iter) & 1) h->parity ^= 1;
  return UOT_OK;
}

}  // namespace

extern "C" {

uot_status rpca_check_params(const rpca_params* p) {
  if (!p) return UOT_ERR_ARG;
  if (p->nx < 1 || p->ny < 1) return UOT_ERR_SHAPE;
  if (p->frames < 2 || p->frames > RP_MAX_FRAMES) return UOT_ERR_SHAPE;
  if (!(p->kappa > 0.0) || !(p->rho > 0.0) || !(p->lam >= 0.0) || !(p->gam >= 0.0) || !std::isfinite(p->kappa) ||
      !std::isfinite(p->rho) || !std::isfinite(p->lam) || !std::isfinite(p->gam) || !std::isfinite(p->eps))
    return UOT_ERR_ARG;
  if (!p->balanced && (!(p->mu > 0.0) || !std::isfinite(p->mu))) return UOT_ERR_ARG;
  if (p->residual_p != 1 && p->residual_p != 2) return UOT_ERR_ARG;
  if (p->bc != 0 && p->bc != 1) return UOT_ERR_ARG;
  if (p->prox_iters < 1 || p->max_iter < 1 || p->check_every < 1) return UOT_ERR_ARG;
  if (!(p->prox_tau_ratio >= 0.0) || !std::isfinite(p->prox_tau_ratio)) return UOT_ERR_ARG;
  if (p->signed_sparse != 0 && p->signed_sparse != 1) return UOT_ERR_ARG;
  return UOT_OK;
}

uot_status rpca_create(const rpca_params* prm, void* hip_stream, rpca_handle** out) {
  if (!out) return UOT_ERR_ARG;
  *out = nullptr;
  uot_status s = rpca_check_params(prm);
  if (s != UOT_OK) return s;
  rpca_handle* h = new (std::nothrow) rpca_handle();
  if (!h) return UOT_ERR_OOM;
  h->prm = *prm;
  h->npx = (long)prm->nx * prm->ny;
  h->n = h->npx * prm->frames;
  h->npairs = (prm->signed_sparse ? 2 : 1) * (prm->frames - 1);
  h->np1 = h->npx * h->npairs;
  h->resid = prm->balanced ? R_BAL : (prm->residual_p == 2 ? R_P2 : R_P1);
  auto fail = [&](uot_status e) {
    delete h;
    return e;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return fail(UOT_ERR_DEVICE);
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess) return fail(UOT_ERR_DEVICE);
    h->own_stream = true;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cu > 0)
    h->num_cu = cu;
  const size_t fb = (size_t)h->n * sizeof(float), pb = (size_t)h->np1 * sizeof(float);
  for (float** q : {&h->S, &h->L, &h->X, &h->Tn, &h->A, &h->D})
    if (hipMalloc((void**)q, fb) != hipSuccess) return fail(UOT_ERR_OOM);
  if (prm->signed_sparse && hipMalloc((void**)&h->Sm, fb) != hipSuccess) return fail(UOT_ERR_OOM);
  for (float** q : {&h->B, &h->C, &h->P0, &h->P1, &h->zo, &h->wo})
    if (hipMalloc((void**)q, pb) != hipSuccess) return fail(UOT_ERR_OOM);
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < RP_NPLANES; ++k)
      if (hipMalloc((void**)&h->st[c][k], pb) != hipSuccess) return fail(UOT_ERR_OOM);
  const int Tf = prm->frames, npairs_g = Tf * (Tf + 1) / 2;
  // two Gram blocks per CU: with one, a block's chunk loads are exposed (36.4 us
  // on 64 frames of 256^2, 26.6 with two); with four, the reduction of the
  // partials costs more than the Gram saves
  h->gblocks = (int)std::min<long>(2 * h->num_cu, std::max<long>(1, (h->npx + 63) / 64));
  if (hipMalloc((void**)&h->d_gpart, (size_t)h->gblocks * npairs_g * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_G, (size_t)npairs_g * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_V, (size_t)Tf * Tf * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_Wm, (size_t)Tf * Tf * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&h->d_lam, RP_MAX_FRAMES * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_sweeps, sizeof(int)) != hipSuccess)
    return fail(UOT_ERR_OOM);

  // the frame pairs as one batch of Algorithm-1 problems (full prox, step kappa / rho)
  const double k2 = uot_knorm2(prm->nx, prm->ny, UOT_PROX, prm->balanced, prm->bc);
  const double t = 0.99 / std::sqrt(k2);
  const double rr = prm->prox_tau_ratio > 0.0 ? std::sqrt(prm->prox_tau_ratio) : 1.0;
  const double t1 = t * rr, t2 = t / rr;
  const double rho_prox = prm->kappa / prm->rho;
  if (prm->prox_iters == 1) {
    h->shape = h->np1 <= (1L << 16) ? 4 : 116;
    h->T = 1;
  } else {
    h->shape = h->np1 <= (1L << 18) ? 4008 : 4016;
    h->T = 4;
  }
  h->launches_per_iter = (prm->prox_iters + h->T - 1) / h->T;
  const int rows = h->shape >= 1000 ? h->shape % 1000 : h->shape % 100;
  std::vector<PairInfo> pairs(h->npairs);
  std::vector<Tile> tiles;
  for (int b = 0; b < h->npairs; ++b) {
    PairInfo& P = pairs[b];
    P.off = (int64_t)b * h->npx;
    P.nx = prm->nx;
    P.ny = prm->ny;
    P.tau1 = (float)t1;
    P.tau2 = (float)t2;
    P.theta = (float)(t1 / (rho_prox + t1));
    P.mutau = (float)(prm->mu * t1);
    P.inv2mt = (float)(1.0 / (1.0 + 2.0 * prm->mu * t1));
    P.tile_begin = (int32_t)tiles.size();
    for (int y = 0; y < prm->ny; y += rows)
      for (int x = 0; x < prm->nx; x += TX) tiles.push_back(Tile{b, x, y, (int32_t)tiles.size()});
    P.tile_count = (int32_t)tiles.size() - P.tile_begin;
    P.pitch = prm->nx;
  }
  h->ntiles = (int)tiles.size();
  std::vector<int32_t> ones(h->npairs, 1);
  if (hipMalloc((void**)&h->d_pairs, pairs.size() * sizeof(PairInfo)) != hipSuccess ||
      hipMalloc((void**)&h->d_tiles, tiles.size() * sizeof(Tile)) != hipSuccess ||
      hipMalloc((void**)&h->d_ntiles, sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void**)&h->d_active, ones.size() * sizeof(int32_t)) != hipSuccess)
    return fail(UOT_ERR_OOM);
  if (hipMemcpy(h->d_pairs, pairs.data(), pairs.size() * sizeof(PairInfo), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_ntiles, &h->ntiles, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_active, ones.data(), ones.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return fail(UOT_ERR_DEVICE);
  int occ = 0;
  if (iter_occupancy(UOT_PROX, h->resid, prm->bc, h->shape, &occ) != hipSuccess || occ <= 0) occ = 2;
  long g = std::min<long>(h->ntiles, (long)h->num_cu * occ);
  h->grid = (int)std::max<long>(8, (g + 7) / 8 * 8);
  h->bx = (int)std::min<long>((h->npx + 255) / 256, std::max(1, 2048 / Tf));
  h->sblocks = (int)std::min<long>(512, (h->npx + 127) / 128);
  h->vblocks = df_blocks(h->n);
  h->pstride = std::max(std::max(h->bx * Tf, h->sblocks), h->vblocks);
  if (hipMalloc((void**)&h->d_partial, RP_SLOTS * (size_t)h->pstride * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->d_sums, RP_SLOTS * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&h->h_sums, RP_SLOTS * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(UOT_ERR_OOM);
  if (hipEventCreate(&h->e0) != hipSuccess || hipEventCreate(&h->e1) != hipSuccess) return fail(UOT_ERR_DEVICE);
  *out = h;
  return UOT_OK;
}

uot_status rpca_solve(rpca_handle* h, const float* y, const float* phi, float* S_out, float* L_out,
                      rpca_report* rep) {
  if (!h || !y || !rep) return UOT_ERR_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  const rpca_params& P = h->prm;
  std::memset(rep, 0, sizeof(*rep));
  if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
  DFCHK(launch_rp_validate(h->n, y, phi, h->d_partial, h->vblocks, h->stream));
  DFCHK(launch_rp_reduce(h->d_partial, h->pstride, RpCounts{{h->vblocks, 0, 0, 0, 0}}, h->d_sums, h->stream));
  DFCHK(hipMemcpyAsync(h->h_sums, h->d_sums, RP_SLOTS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  if (h->h_sums[0] > 0.0) return UOT_ERR_NONFINITE;
  // every variable and the prox states start at zero; the eigenvectors at I
  const size_t fb = (size_t)h->n * sizeof(float), pb = (size_t)h->np1 * sizeof(float);
  for (float* q : {h->S, h->L, h->X, h->Tn, h->A, h->D}) DFCHK(hipMemsetAsync(q, 0, fb, h->stream));
  if (h->Sm) DFCHK(hipMemsetAsync(h->Sm, 0, fb, h->stream));
  for (float* q : {h->B, h->C, h->P0, h->P1, h->zo, h->wo}) DFCHK(hipMemsetAsync(q, 0, pb, h->stream));
  for (auto& c : h->st)
    for (float* q : c) DFCHK(hipMemsetAsync(q, 0, pb, h->stream));
  const int Tf = P.frames;
  std::vector<double> eye((size_t)Tf * Tf, 0.0);
  for (int i = 0; i < Tf; ++i) eye[(size_t)i * Tf + i] = 1.0;
  DFCHK(hipMemcpyAsync(h->d_V, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  h->parity = 0;

  const bool use_graph = !(P.flags & UOT_NO_GRAPH);
  const int W = P.check_every;
  const int nwin = P.max_iter / W, tail = P.max_iter % W;
  int k = 0;
  bool conv = false;
  double rp = std::nan(""), rd = std::nan("");
  DFCHK(hipEventRecord(h->e0, h->stream));
  auto test = [&](int iters) -> uot_status {
    DFCHK(hipStreamSynchronize(h->stream));
    const double* v = h->h_sums;
    rp = std::sqrt(std::max(0.0, v[0] + v[2]));
    rd = P.rho * std::sqrt(std::max(0.0, v[1] + v[3] + v[4]));
    k = iters;
    if (P.eps > 0.0 && rp < P.eps && rd < P.eps) conv = true;
    return UOT_OK;
  };
  for (int w = 0; w < nwin && !conv; ++w) {
    uot_status s = rp_run_window(h, W, y, phi, use_graph);
    if (s != UOT_OK) return s;
    s = test((w + 1) * W);
    if (s != UOT_OK) return s;
  }
  if (!conv && tail > 0) {
    uot_status s = rp_window(h, tail, y, phi);
    if (s != UOT_OK) return s;
    s = test(P.max_iter);
    if (s != UOT_OK) return s;
  }
  DFCHK(hipEventRecord(h->e1, h->stream));
  if (S_out && h->Sm) DFCHK(launch_rp_sub(h->n, h->S, h->Sm, S_out, h->stream));
  else if (S_out) DFCHK(hipMemcpyAsync(S_out, h->S, fb, hipMemcpyDeviceToDevice, h->stream));
  if (L_out) DFCHK(hipMemcpyAsync(L_out, h->L, fb, hipMemcpyDeviceToDevice, h->stream));
  int sweeps = 0;
  DFCHK(hipMemcpyAsync(&sweeps, h->d_sweeps, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  float ms = 0.f;
  DFCHK(hipEventElapsedTime(&ms, h->e0, h->e1));
  rep->iters = k;
  rep->converged = conv ? 1 : 0;
  rep->r_primal = rp;
  rep->r_dual = rd;
  rep->ms_per_iter = k > 0 ? (double)ms / k : 0.0;
  rep->seconds = elapsed_s(t0);
  rep->jacobi_sweeps = sweeps;  // 0 when the warm start was refined
  return UOT_OK;
}

uot_status rpca_copy_planes(rpca_handle* h, float* X, float* Tn, float* A, float* D, float* Z, float* W, float* B,
                            float* C) {
  if (!h) return UOT_ERR_ARG;
  const size_t fb = (size_t)h->n * sizeof(float), pb = (size_t)h->np1 * sizeof(float);
  const float* src[8] = {h->X, h->Tn, h->A, h->D, h->st[h->parity][4], h->st[h->parity][5], h->B, h->C};
  float* dst[8] = {X, Tn, A, D, Z, W, B, C};
  for (int i = 0; i < 8; ++i)
    if (dst[i]) DFCHK(hipMemcpyAsync(dst[i], src[i], i < 4 ? fb : pb, hipMemcpyDeviceToDevice, h->stream));
  DFCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

uot_status rpca_copy_sparse(rpca_handle* h, float* Sp, float* Sm) {
  if (!h) return UOT_ERR_ARG;
  const size_t fb = (size_t)h->n * sizeof(float);
  if (Sp) DFCHK(hipMemcpyAsync(Sp, h->S, fb, hipMemcpyDeviceToDevice, h->stream));
  if (Sm) {
    if (h->Sm) DFCHK(hipMemcpyAsync(Sm, h->Sm, fb, hipMemcpyDeviceToDevice, h->stream));
    else DFCHK(hipMemsetAsync(Sm, 0, fb, h->stream));
  }
  DFCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

void rpca_destroy(rpca_handle* h) { delete h; }

}  // extern "C"
