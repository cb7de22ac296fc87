// Host runtime of the unbalanced Beckmann OT prox solver: argument checks,
// step-size planning (Theorem 1), tile lists for ragged batches, graph
// capture of check windows, the device-side stopping loop and the reports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/uot.h"
#include "uot_internal.hpp"
#include "uot_plan.hpp"

using namespace uot;
using namespace uot::planner;

namespace {

int resid_of(const uot_params& p) { return p.balanced ? R_BAL : (p.residual_p == 2 ? R_P2 : R_P1); }

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double seconds() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

// Tile-shape cache filled by the autotuner, keyed by (mode, resid, bc, size class).
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_key(int mode, int resid, int bc, long total_px) {
  int cls = 0;
  while ((1L << (2 * cls + 12)) < total_px && cls < 12) ++cls;  // 4^k * 4096 buckets
  char buf[96];
  std::snprintf(buf, sizeof(buf), "gfx950:m%d:r%d:b%d:c%d", mode, resid, bc, cls);
  return buf;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("UOT_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[128];
  int ty;
  while (std::fscanf(f, " \"%127[^\"]\" : %d ,", key, &ty) == 2) g_tune_cache[key] = ty;
  std::fclose(f);
}

void tune_store_locked() {
  const char* path = std::getenv("UOT_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : g_tune_cache)
    std::fprintf(f, "  \"%s\" : %d%s\n", kv.first.c_str(), kv.second, ++i < g_tune_cache.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
}

bool aligned4(const void* p) { return p == nullptr || ((uintptr_t)p & 3u) == 0; }

template <class T>
hipError_t grow(T** p, size_t* cap, size_t n) {
  if (n <= *cap && *p) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t want = std::max<size_t>(n, 1);
  hipError_t e = hipMalloc((void**)p, want * sizeof(T));
  if (e == hipSuccess) *cap = want;
  return e;
}

}  // namespace

struct uot_handle {
  uot_params prm{};
  // workspace borrowed from the no-allocation scratch: never freed, and no
  // path that would allocate (graphs, autotuning, the Poisson certificate)
  bool borrowed = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int num_cu = 256;

  // ping-pong shadow state and the c plane
  float* B[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t capB[6] = {0, 0, 0, 0, 0, 0};
  float* cplane = nullptr;
  size_t cap_c = 0;

  Tile* d_tiles = nullptr;      // full list (check/setup)
  size_t cap_tiles = 0;
  Tile* d_live = nullptr;       // live list (iteration)
  size_t cap_live = 0;
  int32_t* d_nlive = nullptr;
  size_t cap_nlive = 0;
  double* d_partial = nullptr;
  size_t cap_partial = 0;

  PairInfo* d_pairs = nullptr;
  size_t cap_pairs = 0;
  double* d_sums = nullptr;
  size_t cap_sums = 0;
  int32_t* d_i32 = nullptr;     // active | iters | status | n_active
  size_t cap_i32 = 0;
  double* d_f64 = nullptr;      // rel_res | xnorm | inv_s
  size_t cap_f64 = 0;
  float* d_invs = nullptr;
  size_t cap_invs = 0;

  double* h_sums = nullptr;     // pinned
  size_t cap_hsums = 0;
  int32_t* h_i32 = nullptr;     // pinned
  size_t cap_hi32 = 0;

  std::vector<Tile> h_live;     // kept alive across async uploads

  // Poisson solve: DCT-II matrices by size, scratch planes, partial sums
  std::map<int, float*> dct;
  float* pw[4] = {nullptr, nullptr, nullptr, nullptr};  // t1 | t2 | phi | rhs
  size_t cap_pw[4] = {0, 0, 0, 0};
  double* d_pp = nullptr;
  size_t cap_pp = 0;

  // per-pair (iterations, rel_res) at every check of the last solve with
  // UOT_RECORD_HISTORY
  std::vector<std::vector<std::pair<int32_t, double>>> hist;
  bool have_hist = false;

  // Douglas-Rachford: w and u planes (5 each), its partial sums, its graph
  float* drbuf = nullptr;
  size_t cap_drbuf = 0;
  double* d_drp = nullptr;
  size_t cap_drp = 0;
  double* h_drp = nullptr;
  hipGraphExec_t drexec = nullptr;
  int dr_w = 0;
  const void* dr_key[4] = {};
  double* h_pp = nullptr;       // pinned

  // cached graphs: [burst][parity], burst 0 one check window, 1 a burst of
  // several windows between host polls; parity 1 starts from the shadow copy
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  std::vector<unsigned char> gkey[2][2];
  int32_t* d_mask = nullptr;    // per-pair flags of a masked copy
  size_t cap_mask = 0;

  // UOT_PROFILE: per-window timing lines (stderr, or appended to a file)
  FILE* prof = nullptr;
  bool prof_own = false;
  hipEvent_t pev[2] = {nullptr, nullptr};
  long prof_solves = 0;

  ~uot_handle() {
    if (prof_own && prof) std::fclose(prof);
    if (borrowed) return;
    for (auto& e : pev)
      if (e) (void)hipEventDestroy(e);
    for (auto& row : gexec)
      for (auto& g : row)
        if (g) (void)hipGraphExecDestroy(g);
    if (drexec) (void)hipGraphExecDestroy(drexec);
    if (drbuf) (void)hipFree(drbuf);
    if (d_drp) (void)hipFree(d_drp);
    if (h_drp) (void)hipHostFree(h_drp);
    for (auto& p : B)
      if (p) (void)hipFree(p);
    void* dev[] = {cplane, d_tiles, d_live, d_nlive, d_partial, d_pairs, d_sums, d_i32, d_f64, d_invs, d_mask};
    for (void* p : dev)
      if (p) (void)hipFree(p);
    if (h_sums) (void)hipHostFree(h_sums);
    if (h_i32) (void)hipHostFree(h_i32);
    for (auto& kv : dct) (void)hipFree(kv.second);
    for (auto& p : pw)
      if (p) (void)hipFree(p);
    if (d_pp) (void)hipFree(d_pp);
    if (h_pp) (void)hipHostFree(h_pp);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

extern "C" {

const char* uot_status_string(uot_status s) {
  switch (s) {
    case UOT_OK: return "ok";
    case UOT_ERR_ARG: return "invalid argument";
    case UOT_ERR_SHAPE: return "inconsistent grid sizes or offsets";
    case UOT_ERR_STEP: return "step sizes violate tau1*tau2*||K||^2 < 1";
    case UOT_ERR_NONFINITE: return "non-finite value in an input image or warm-start state";
    case UOT_ERR_NEGATIVE: return "negative pixel in an input image";
    case UOT_ERR_DEVICE: return "HIP device error";
    case UOT_ERR_OOM: return "device memory allocation failed";
    case UOT_ERR_MASS: return "balanced zero-flux problem with unequal masses";
    case UOT_ERR_TOO_LARGE: return "problem larger than the no-allocation scratch";
  }
  return "unknown status";
}

double uot_knorm2(int32_t nx, int32_t ny, int32_t mode, int32_t balanced, int32_t bc) {
  return planner::knorm2_of(nx, ny, mode, balanced, bc);
}

uot_status uot_check_params(const uot_params* p) { return planner::check_params(p); }

uot_status uot_create(const uot_params* prm, void* hip_stream, uot_handle** out) {
  if (!out) return UOT_ERR_ARG;
  *out = nullptr;
  uot_status st = uot_check_params(prm);
  if (st != UOT_OK) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UOT_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return UOT_ERR_DEVICE;
  auto* h = new (std::nothrow) uot_handle();
  if (!h) return UOT_ERR_OOM;
  h->prm = *prm;
  h->device = dev;
  h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      delete h;
      return UOT_ERR_DEVICE;
    }
    h->own_stream = true;
  }
  // UOT_PROFILE=1: per-window timing on stderr; any other value except 0
  // names a file the lines are appended to
  if (const char* pv = std::getenv("UOT_PROFILE")) {
    if (pv[0] && std::strcmp(pv, "0") != 0) {
      if (std::strcmp(pv, "1") == 0) {
        h->prof = stderr;
      } else {
        h->prof = std::fopen(pv, "a");
        h->prof_own = h->prof != nullptr;
      }
    }
  }
  *out = h;
  return UOT_OK;
}

void uot_destroy(uot_handle* h) { delete h; }

}  // extern "C"

namespace {

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) {                         \
      if (std::getenv("UOT_DEBUG"))                 \
        std::fprintf(stderr, "uot: %s failed: %s (%s:%d)\n", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      return e_ == hipErrorOutOfMemory ? UOT_ERR_OOM : UOT_ERR_DEVICE; \
    }                                               \
  } while (0)

double image_scale(const double* setup_sums) {
  const double s = setup_sums[U_MAXIN];
  return std::isfinite(s) && s > 0.0 ? s : 1.0;
}

// The per-pair step fields the kernels read.
void set_steps(const uot_params& p, PairInfo& P, double t1, double t2) {
  P.tau1 = (float)t1;
  P.tau2 = (float)t2;
  P.theta = p.mode == UOT_DIST ? 0.f : (float)(t1 / (p.rho + t1));
  P.mutau = (float)(p.mu * t1);
  P.inv2mt = (float)(1.0 / (1.0 + 2.0 * p.mu * t1));
}

struct Job {
  int B = 0;
  std::vector<PairInfo> pairs;
  std::vector<Tile> tiles;
  std::vector<double> knorm2;
  long total_px = 0;  // extent of the packed planes (elements)
  long npx = 0;       // pixels of all pairs
  int ty = 8;        // rows per tile
  int shape = 8;     // kernel shape code: rows, or 100 + rows for the vectorised kernel
  bool vec_ok = false;
};

Planes planes_of(const uot_state& s) { return Planes{s.Mx, s.My, s.r, s.a, s.x0, s.x1}; }

// Grid of the persistent iteration kernel: enough resident blocks to fill
// every CU, rounded to a multiple of the 8 XCDs.
// Template code of the fused kernels and the check: bit 0 the boundary
// reading, bit 1 the anisotropic flux norm.
int bcn_of(const uot_params& p) { return p.bc | (p.norm == UOT_NORM_ANISO ? 2 : 0); }

long group_cap(const uot_handle* h) { return planner::group_cap_of(h->prm.max_groups); }

int iter_grid(uot_handle* h, int mode, int resid, int bc, int ty, int ntiles, bool chk = false) {
  int occ = 0;
  const hipError_t e = chk ? iter_chk_occupancy(mode, resid, bc, ty, &occ) : iter_occupancy(mode, resid, bc, ty, &occ);
  if (e != hipSuccess || occ <= 0) occ = chk ? 2 : 4;
  long g = std::min<long>((long)ntiles, (long)h->num_cu * occ);
  g = std::max<long>(8, (g + 7) / 8 * 8);
  return (int)std::min(g, group_cap(h));
}

int aux_grid(uot_handle* h, int ntiles) {
  return (int)std::max<long>(1, std::min<long>(std::min(ntiles, h->num_cu * 8), group_cap(h)));
}

uot_status validate_state(const uot_params& p, const uot_state* s) {
  if (!s || !s->Mx || !s->My || !s->a) return UOT_ERR_ARG;
  if (!p.balanced && !s->r) return UOT_ERR_ARG;
  if (p.mode == UOT_PROX && (!s->x0 || !s->x1)) return UOT_ERR_ARG;
  if (p.mode == UOT_PROX_FIXED && !s->x1) return UOT_ERR_ARG;
  return UOT_OK;
}

// Where the pairs of a call live in the packed planes (host arrays of B):
// pixel (x, y) of pair b is element offset[b] + y * pitch[b] + x; pitch ==
// nullptr means pitch[b] = nx[b] (rows packed back to back).
struct Layout {
  int B;
  const int32_t *nx, *ny, *pitch;
  const int64_t* offset;
  int32_t pitch_of(int b) const { return pitch ? pitch[b] : nx[b]; }
};

uot_status plan(uot_handle* h, const Layout& L, Job& J, int force_ty = 0, bool* cached = nullptr,
                bool ptrs_aligned = false) {
  const uot_params& p = h->prm;
  const int B = L.B;
  const int32_t *nx = L.nx, *ny = L.ny;
  const int64_t* offset = L.offset;
  if (B < 1 || !nx || !ny || !offset) return UOT_ERR_ARG;
  J.B = B;
  J.pairs.resize(B);
  J.knorm2.resize(B);
  long total = 0, npx = 0;
  const uot_status ls = planner::check_layout(B, nx, ny, L.pitch, offset, &total, &npx);
  if (ls != UOT_OK) return ls;
  J.total_px = total;
  J.npx = npx;
  J.vec_ok = ptrs_aligned;
  const int resid = resid_of(p);
  // tile rows: explicit, autotuned, or heuristic
  int ty = force_ty > 0 ? force_ty : p.tile_rows;
  if (cached) *cached = true;
  if (ty == 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune_cache.find(tune_key(p.mode, resid, bcn_of(p), npx));
    if (cached) *cached = it != g_tune_cache.end();
    ty = it != g_tune_cache.end() ? it->second : heuristic_shape(npx);
  }
  if (ty >= 1000 && !planner::blocked_pitch_ok(B, nx, L.pitch)) ty = shape_single(ty);
  // the vectorised kernels (100 * variant + rows) take any row layout but
  // need every plane 4-byte aligned; otherwise the scalar kernel of the same
  // rows runs
  if (ty >= 100 && !J.vec_ok) ty = shape_rows(ty);
  J.shape = ty;
  ty = shape_rows(ty);
  J.ty = ty;
  J.tiles.clear();
  for (int b = 0; b < B; ++b) {
    const double k2 = uot_knorm2(nx[b], ny[b], p.mode, p.balanced, p.bc);
    J.knorm2[b] = k2;
    double t1 = p.tau1, t2 = p.tau2;
    if (t1 == 0.0) default_steps(k2, 1.0, &t1, &t2);  // rescaled once the image scale is known
    if (!(p.flags & UOT_UNSAFE_STEPS) && t1 * t2 * k2 >= 1.0) return UOT_ERR_STEP;
    PairInfo& P = J.pairs[b];
    P.off = offset[b];
    P.nx = nx[b];
    P.ny = ny[b];
    set_steps(p, P, t1, t2);
    P.tile_begin = (int32_t)J.tiles.size();
    for (int y = 0; y < ny[b]; y += ty)
      for (int x = 0; x < nx[b]; x += TX) J.tiles.push_back(Tile{b, x, y, (int32_t)J.tiles.size()});
    P.tile_count = (int32_t)J.tiles.size() - P.tile_begin;
    P.pitch = L.pitch_of(b);
  }
  return UOT_OK;
}

uot_status ensure_workspace(uot_handle* h, const Job& J) {
  const uot_params& p = h->prm;
  const size_t px = (size_t)J.total_px;
  const int resid = resid_of(p);
  const bool need[6] = {true, true, resid != R_BAL, true, p.mode == UOT_PROX, p.mode != UOT_DIST};
  for (int i = 0; i < 6; ++i)
    if (need[i]) HIPCHK(grow(&h->B[i], &h->capB[i], px));
  if (p.mode == UOT_DIST) HIPCHK(grow(&h->cplane, &h->cap_c, px));
  const size_t nt = J.tiles.size();
  HIPCHK(grow(&h->d_tiles, &h->cap_tiles, nt));
  HIPCHK(grow(&h->d_live, &h->cap_live, nt));
  HIPCHK(grow(&h->d_nlive, &h->cap_nlive, 1));
  HIPCHK(grow(&h->d_partial, &h->cap_partial, nt * NS));
  HIPCHK(grow(&h->d_pairs, &h->cap_pairs, (size_t)J.B));
  HIPCHK(grow(&h->d_sums, &h->cap_sums, (size_t)J.B * NS));
  HIPCHK(grow(&h->d_i32, &h->cap_i32, (size_t)J.B * 3 + 1));
  HIPCHK(grow(&h->d_f64, &h->cap_f64, (size_t)J.B * 3));
  HIPCHK(grow(&h->d_invs, &h->cap_invs, (size_t)J.B));
  HIPCHK(grow(&h->d_mask, &h->cap_mask, (size_t)J.B));
  if (h->cap_hsums < (size_t)J.B * NS) {
    if (h->h_sums) (void)hipHostFree(h->h_sums);
    h->h_sums = nullptr;
    h->cap_hsums = 0;
    HIPCHK(hipHostMalloc((void**)&h->h_sums, (size_t)J.B * NS * sizeof(double), hipHostMallocDefault));
    h->cap_hsums = (size_t)J.B * NS;
  }
  if (h->cap_hi32 < (size_t)J.B * 3 + 1) {
    if (h->h_i32) (void)hipHostFree(h->h_i32);
    h->h_i32 = nullptr;
    h->cap_hi32 = 0;
    HIPCHK(hipHostMalloc((void**)&h->h_i32, ((size_t)J.B * 3 + 1) * sizeof(int32_t), hipHostMallocDefault));
    h->cap_hi32 = (size_t)J.B * 3 + 1;
  }
  return UOT_OK;
}

Planes shadow_planes(uot_handle* h) { return Planes{h->B[0], h->B[1], h->B[2], h->B[3], h->B[4], h->B[5]}; }

// Uploads the live tile list: tiles of pairs whose flag is set.
uot_status upload_live(uot_handle* h, const Job& J, const int32_t* active_host) {
  h->h_live.clear();
  for (const Tile& t : J.tiles)
    if (active_host[t.pair]) h->h_live.push_back(t);
  const int32_t n = (int32_t)h->h_live.size();
  if (n > 0)
    HIPCHK(hipMemcpyAsync(h->d_live, h->h_live.data(), n * sizeof(Tile), hipMemcpyHostToDevice, h->stream));
  h->h_i32[(size_t)J.B * 3] = n;
  HIPCHK(hipMemcpyAsync(h->d_nlive, &h->h_i32[(size_t)J.B * 3], sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

// Setup pass: validation, c = q - p, state init.  Fills per-pair sums on the host.
uot_status run_setup(uot_handle* h, const Job& J, const float* src, const float* dst, const uot_state* st,
                     bool warm, bool write_state) {
  const uot_params& p = h->prm;
  SetupArgs sa{};
  sa.src = src;
  sa.dst = dst;
  sa.c = h->cplane;
  sa.st = planes_of(*st);
  sa.mode = p.mode;
  sa.resid = resid_of(p);
  sa.bc = p.bc;
  sa.warm = warm ? 1 : 0;
  sa.write_state = write_state ? 1 : 0;
  sa.write_c = 1;
  sa.pairs = h->d_pairs;
  sa.tiles = h->d_tiles;
  sa.ntiles = (int32_t)J.tiles.size();
  sa.tile_rows = J.ty;
  sa.partial = h->d_partial;
  HIPCHK(launch_setup(aux_grid(h, sa.ntiles), sa, h->stream));
  HIPCHK(launch_pair_reduce(h->d_pairs, J.B, h->d_partial, kMaxSlotsSetup, h->d_sums, h->stream));
  HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, (size_t)J.B * NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

// cold: with UOT_WARM_FALLBACK, set for the pairs whose warm state holds a
// non-finite value (they are restarted from zeros); otherwise such a pair
// fails the call.
uot_status check_setup_sums(uot_handle* h, const Job& J, bool warm, std::vector<int32_t>* cold = nullptr) {
  const uot_params& p = h->prm;
  if (cold) cold->assign(J.B, 0);
  for (int b = 0; b < J.B; ++b) {
    const double* S = h->h_sums + (size_t)b * NS;
    if (S[U_NONFIN_IN] > 0) return UOT_ERR_NONFINITE;
    if (warm && S[U_NONFIN_ST] > 0) {
      if (!cold || !(p.flags & UOT_WARM_FALLBACK)) return UOT_ERR_NONFINITE;
      (*cold)[b] = 1;
    }
    if (S[U_NEG] > 0 && !(p.flags & UOT_ALLOW_SIGNED)) return UOT_ERR_NEGATIVE;
    if (p.mode == UOT_DIST && p.balanced && p.bc == 0) {
      const double m = std::max({std::fabs(S[U_SUMS]), std::fabs(S[U_SUMD]), 1e-30});
      if (std::fabs(S[U_SUMS] - S[U_SUMD]) > 1e-4 * m) return UOT_ERR_MASS;
    }
  }
  return UOT_OK;
}

// Scales the default steps of every pair by its image scale (from the
// setup sums in `scale`) and uploads the pair records.  No-op when the
// caller gave the steps.
uot_status scale_default_steps(uot_handle* h, Job& J, const std::vector<double>& scale) {
  const uot_params& p = h->prm;
  if (p.tau1 != 0.0) return UOT_OK;
  for (int b = 0; b < J.B; ++b) {
    double t1, t2;
    default_steps(J.knorm2[b], scale[b], &t1, &t2);
    set_steps(p, J.pairs[b], t1, t2);
  }
  HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), J.B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
  return UOT_OK;
}

std::vector<double> image_scales(const uot_handle* h, int B) {
  std::vector<double> sc(B);
  for (int b = 0; b < B; ++b) sc[b] = image_scale(h->h_sums + (size_t)b * NS);
  return sc;
}

struct Reporter {
  // per-pair final fields computed on the host from the final check sums
  static void fill(const uot_params& p, const PairInfo& P, const double* S, double xnorm_dist, uot_report* r,
                   double dual_prox, bool have_dual_prox, double bal_primal = std::nan("")) {
    const int resid = resid_of(p);
    const double mu = p.mu, rho = p.rho;
    const double quad = p.mode == UOT_DIST ? 0.0 : S[S_QUAD] / (2.0 * rho);
    double obj = S[S_MNORM] + quad;
    if (resid != R_BAL) obj += mu * S[S_RPEN];
    r->objective = obj;
    r->feas = std::sqrt(std::max(0.0, S[S_PRES2]));
    const double xn = p.mode == UOT_DIST ? xnorm_dist : std::sqrt(S[S_X0SQ]) + std::sqrt(S[S_X1SQ]);
    const double pr = std::sqrt(S[S_PRES2]) / std::max(xn, 1e-30);
    const double du = std::sqrt(S[S_STAT2]) / std::max(std::sqrt(S[S_KA2]), 1e-30);
    r->rel_res = std::max(pr, du);
    r->tau1 = P.tau1;
    r->tau2 = P.tau2;
    r->primal = r->dual = r->rel_gap = std::nan("");
    if (resid == R_BAL) {
      // DIST with the zero-flux boundary: the primal bound comes from the
      // Poisson feasibility repair; the dual needs only ||(D* a)_i|| <= 1
      if (p.mode == UOT_DIST && std::isfinite(bal_primal)) {
        r->primal = bal_primal;
        r->dual = S[S_LIN] / std::max(1.0, S[S_MAXG]);
        r->rel_gap = (r->primal - r->dual) / std::max(std::fabs(r->primal), 1e-30);
      }
      return;
    }
    r->primal = S[S_MNORM] + mu * S[S_EPEN] + quad;
    double s = std::max(1.0, S[S_MAXG]);
    if (resid == R_P1) s = std::max(s, S[S_MAXA] / mu);
    if (p.mode == UOT_DIST) {
      r->dual = S[S_LIN] / s;
      if (resid == R_P2) r->dual -= S[S_A2] / (s * s) / (4.0 * mu);
    } else if (have_dual_prox) {
      r->dual = dual_prox;
    }
    if (std::isfinite(r->dual)) r->rel_gap = (r->primal - r->dual) / std::max(std::fabs(r->primal), 1e-30);
  }
};

double scale_of(const uot_params& p, const double* S) {
  double s = std::max(1.0, S[S_MAXG]);
  if (resid_of(p) == R_P1) s = std::max(s, S[S_MAXA] / p.mu);
  return s;
}

// Dual values of the PROX modes (second pass once the scale s is known).
uot_status prox_duals(uot_handle* h, const Job& J, const float* src, const float* dst, const float* a_plane,
                      const double* sums, std::vector<double>& out) {
  const uot_params& p = h->prm;
  std::vector<float> invs(J.B);
  for (int b = 0; b < J.B; ++b) invs[b] = (float)(1.0 / scale_of(p, sums + (size_t)b * NS));
  HIPCHK(hipMemcpyAsync(h->d_invs, invs.data(), J.B * sizeof(float), hipMemcpyHostToDevice, h->stream));
  DualArgs da{};
  da.a = a_plane;
  da.x_src = src;
  da.x_dst = dst;
  da.inv_s = h->d_invs;
  da.pairs = h->d_pairs;
  da.tiles = h->d_tiles;
  da.ntiles = (int32_t)J.tiles.size();
  da.tile_rows = J.ty;
  da.mode = p.mode;
  da.resid = resid_of(p);
  da.rho = (float)p.rho;
  da.mu = (float)p.mu;
  da.partial = h->d_partial;
  HIPCHK(launch_dual(aux_grid(h, da.ntiles), da, h->stream));
  HIPCHK(launch_pair_reduce(h->d_pairs, J.B, h->d_partial, 0u, h->d_sums, h->stream));
  std::vector<double> tmp((size_t)J.B * NS);
  HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, (size_t)J.B * NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out.resize(J.B);
  for (int b = 0; b < J.B; ++b) out[b] = h->h_sums[(size_t)b * NS];
  return UOT_OK;
}

struct Launch {
  uot_handle* h;
  const Job* J;
  IterArgs fwd, bwd;   // A -> B and B -> A
  CheckArgs chk;
  DecideArgs dec;
  int grid_iter, grid_single, grid_aux, grid_chk, resid;
};

// One launch of `steps` iterations: the shape's own kernel, or its
// single-step kernel when steps == 1.
hipError_t launch_steps(uot_handle* h, int resid, int shape, int steps, int grid_multi, int grid_single,
                        IterArgs a) {
  const uot_params& p = h->prm;
  if (steps <= 1 || shape_steps(shape) == 1)
    return launch_iter(p.mode, resid, bcn_of(p), shape_single(shape), grid_single, a, h->stream);
  a.steps = steps;
  return launch_iter(p.mode, resid, bcn_of(p), shape, grid_multi, a, h->stream);
}

// The launches of one window of W iterations.  With a check on a blocked
// shape the window's last launch is the check variant (fused_schedule);
// with a check on a one-step shape every launch runs one iteration and the
// separate check kernel compares the last two; without a check the window
// is plain launches of up to T iterations.  The number of launches may be
// odd: the window then ends in the other copy of the state.
std::vector<int> window_schedule(const Launch& L, int W, bool check) {
  const int T = shape_steps(L.J->shape);
  if (check && T > 1) return fused_schedule(W, T, shape_chk_steps(L.J->shape));
  return step_schedule(W, T, check, false);
}

// Launches of one window of W iterations starting from copy `parity` (0:
// the caller's planes, 1: the shadow), then the check when there is one.
uot_status enqueue_window(Launch& L, int W, bool check, int parity) {
  uot_handle* h = L.h;
  const uot_params& p = h->prm;
  const bool fused = check && shape_steps(L.J->shape) > 1;
  const std::vector<int> sched = window_schedule(L, W, check);
  for (size_t i = 0; i < sched.size(); ++i) {
    IterArgs a = ((i + parity) & 1) ? L.bwd : L.fwd;
    if (fused && i + 1 == sched.size()) {
      a.steps = sched[i];
      a.chk = h->d_partial;
      HIPCHK(launch_iter_chk(p.mode, L.resid, bcn_of(p), L.J->shape, L.grid_chk, a, h->stream));
    } else {
      HIPCHK(launch_steps(h, L.resid, L.J->shape, sched[i], L.grid_iter, L.grid_single, a));
    }
  }
  if (check) {
    if (!fused) HIPCHK(launch_check(p.mode, L.resid, bcn_of(p), L.grid_aux, L.chk, h->stream));
    HIPCHK(launch_reduce_decide(L.dec, h->d_partial, h->stream));
  }
  return UOT_OK;
}

// Launches per window (its parity decides which copy a window ends in).
int window_launches(const Launch& L, int W, bool check) { return (int)window_schedule(L, W, check).size(); }

uot_status get_graph(Launch& L, int W, bool check, int reps, int parity, hipGraphExec_t* out) {
  uot_handle* h = L.h;
  const int per = window_launches(L, W, check);
  hipGraphExec_t& slot = h->gexec[reps == 1 ? 0 : 1][parity];
  std::vector<unsigned char>& skey = h->gkey[reps == 1 ? 0 : 1][parity];
  std::vector<unsigned char> key;
  auto put = [&](const void* d, size_t n) {
    const unsigned char* c = (const unsigned char*)d;
    key.insert(key.end(), c, c + n);
  };
  put(&L.fwd, sizeof(L.fwd));
  put(&L.chk, sizeof(L.chk));
  put(&L.dec, sizeof(L.dec));
  put(&W, sizeof(W));
  put(&reps, sizeof(reps));
  put(&parity, sizeof(parity));
  int c = check;
  put(&c, sizeof(c));
  put(&L.grid_iter, sizeof(int));
  put(&L.grid_chk, sizeof(int));
  put(&L.J->shape, sizeof(int));
  put(&h->prm, sizeof(h->prm));
  if (slot && key == skey) {
    *out = slot;
    return UOT_OK;
  }
  if (slot) {
    (void)hipGraphExecDestroy(slot);
    slot = nullptr;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  uot_status st = UOT_OK;
  int par = parity;
  for (int r = 0; r < reps && st == UOT_OK; ++r) {
    st = enqueue_window(L, W, check, par);
    par ^= per & 1;
  }
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (st != UOT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  HIPCHK(e);
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  slot = ex;
  skey = key;
  *out = ex;
  return UOT_OK;
}

// Orthonormal DCT-II matrix of size n, C[k][i] = s_k cos(pi (2i+1) k / (2n)),
// cached on the device per size.
uot_status get_dct(uot_handle* h, int n, const float** out) {
  auto it = h->dct.find(n);
  if (it != h->dct.end()) {
    *out = it->second;
    return UOT_OK;
  }
  std::vector<float> m((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    const double s = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
    for (int i = 0; i < n; ++i) m[(size_t)k * n + i] = (float)(s * std::cos(kPi * (2.0 * i + 1) * k / (2.0 * n)));
  }
  float* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, m.size() * sizeof(float)));
  hipError_t e = hipMemcpy(d, m.data(), m.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return UOT_ERR_DEVICE;
  }
  h->dct[n] = d;
  *out = d;
  return UOT_OK;
}

uot_status ensure_poisson(uot_handle* h, size_t px) {
  for (int i = 0; i < 4; ++i) HIPCHK(grow(&h->pw[i], &h->cap_pw[i], px));
  HIPCHK(grow(&h->d_pp, &h->cap_pp, 1024));
  if (!h->h_pp) HIPCHK(hipHostMalloc((void**)&h->h_pp, 1024 * sizeof(double), hipHostMallocDefault));
  return UOT_OK;
}

// phi = (alpha I + D D*)^{-1} rhs on one grid (scratch planes pw[0], pw[1]).
uot_status poisson_grid(uot_handle* h, int nx, int ny, double alpha, const float* rhs, float* phi) {
  const float *cx = nullptr, *cy = nullptr;
  uot_status s = get_dct(h, nx, &cx);
  if (s != UOT_OK) return s;
  s = get_dct(h, ny, &cy);
  if (s != UOT_OK) return s;
  HIPCHK(poisson_solve(cx, cy, nx, ny, (float)alpha, rhs, phi, h->pw[0], h->pw[1], h->stream));
  return UOT_OK;
}

// Feasibility repair of a balanced DIST state (zero-flux boundary): with
// e = D M + c and phi = (D D*)^+ e, the flux M - D* phi satisfies the
// constraint; its l2,1 norm is a certified upper bound on the value.
uot_status balanced_primal(uot_handle* h, const Job& J, const float* src, const float* dst, const uot_state* st,
                           std::vector<double>& out) {
  out.assign(J.B, std::nan(""));
  size_t maxpx = 0;
  for (const PairInfo& P : J.pairs) maxpx = std::max<size_t>(maxpx, (size_t)P.nx * P.ny);
  uot_status s = ensure_poisson(h, maxpx);
  if (s != UOT_OK) return s;
  for (int b = 0; b < J.B; ++b) {
    const PairInfo& P = J.pairs[b];
    const long o = P.off;
    HIPCHK(launch_infeasibility(st->Mx + o, st->My + o, src + o, dst + o, h->pw[3], P.nx, P.ny, P.pitch, h->stream));
    s = poisson_grid(h, P.nx, P.ny, 0.0, h->pw[3], h->pw[2]);
    if (s != UOT_OK) return s;
    const int nb = repaired_norm_blocks(P.nx, P.ny);
    HIPCHK(launch_repaired_norm(st->Mx + o, st->My + o, h->pw[2], P.nx, P.ny, P.pitch, h->prm.norm, h->d_pp,
                                h->stream));
    HIPCHK(hipMemcpyAsync(h->h_pp, h->d_pp, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += h->h_pp[i];
    out[b] = acc;
  }
  return UOT_OK;
}

// Autotuner: times every tile shape on this very workload (the caller's
// state after setup is read, the shadow copy is written, nothing else
// changes), keeps the fastest for the (mode, variant, boundary, size class)
// key, persists the table to $UOT_AUTOTUNE_CACHE when set, and re-plans J.
uot_status autotune(uot_handle* h, const Layout& L, const float* src, const float* dst, uot_state* st, Job& J) {
  const int B = L.B;
  const uot_params& p = h->prm;
  const int resid = resid_of(p);
  std::vector<int> cand = {4, 8, 16, 32};
  if (J.vec_ok) {
    for (int c : {116, 132, 316, 332, 4004, 4008, 2016, 4016, 8016, 4032, 8032}) cand.push_back(c);
  }
  Job J4;
  uot_status s = plan(h, L, J4, 4);
  if (s != UOT_OK) return s;
  s = ensure_workspace(h, J4);  // the 4-row list is the longest
  if (s != UOT_OK) return s;
  std::vector<int32_t> ones(B, 1);
  HIPCHK(hipMemcpyAsync(h->d_i32, ones.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  const Planes A = planes_of(*st), Bp = shadow_planes(h);
  const float* cptr = p.mode == UOT_DIST ? h->cplane : nullptr;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_ty = J.shape;
  for (int ty : cand) {
    Job Jt;
    s = plan(h, L, Jt, ty, nullptr, J.vec_ok);
    if (s != UOT_OK) break;
    HIPCHK(hipMemcpyAsync(h->d_pairs, Jt.pairs.data(), B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
    s = upload_live(h, Jt, ones.data());
    if (s != UOT_OK) break;
    const IterArgs fwd{A, Bp, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, h->d_i32};
    const int grid = iter_grid(h, p.mode, resid, bcn_of(p), Jt.shape, (int)Jt.tiles.size());
    const int T = shape_steps(Jt.shape);
    for (int i = 0; i < 2; ++i) HIPCHK(launch_steps(h, resid, Jt.shape, T, grid, grid, fwd));
    HIPCHK(hipEventRecord(e0, h->stream));
    for (int i = 0; i < 10; ++i) HIPCHK(launch_steps(h, resid, Jt.shape, T, grid, grid, fwd));
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ms /= (float)T;  // per iteration
    if (ms < best) {
      best = ms;
      best_ty = Jt.shape;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != UOT_OK) return s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(p.mode, resid, bcn_of(p), J.npx)] = best_ty;
    tune_store_locked();
  }
  s = plan(h, L, J, best_ty, nullptr, J.vec_ok);
  if (s != UOT_OK) return s;
  s = ensure_workspace(h, J);
  if (s != UOT_OK) return s;
  HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

uot_status solve_core(uot_handle* h, const Layout& lay, const float* src, const float* dst, uot_state* st,
                      uot_report* reps) {
  const int B = lay.B;
  Timer timer;
  const uot_params& p = h->prm;
  if (!src || !dst || !reps) return UOT_ERR_ARG;
  uot_status s = validate_state(p, st);
  if (s != UOT_OK) return s;
  Job J;
  bool cached = true;
  const bool ptrs_aligned = aligned4(src) && aligned4(dst) && aligned4(st->Mx) && aligned4(st->My) &&
                            aligned4(st->r) && aligned4(st->a) && aligned4(st->x0) && aligned4(st->x1);
  s = plan(h, lay, J, 0, &cached, ptrs_aligned);
  if (s != UOT_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
  s = ensure_workspace(h, J);
  if (s != UOT_OK) return s;
  const int resid = resid_of(p);
  const bool warm = (p.flags & UOT_WARM_START) != 0;

  HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, h->stream));
  s = run_setup(h, J, src, dst, st, warm, true);
  if (s != UOT_OK) return s;
  std::vector<int32_t> cold;
  s = check_setup_sums(h, J, warm, &cold);
  if (s != UOT_OK) return s;
  if (std::find(cold.begin(), cold.end(), 1) != cold.end()) {
    // the rejected warm states start from zeros, as a cold solve would
    HIPCHK(hipMemcpyAsync(h->d_mask, cold.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_zero_pairs(planes_of(*st), h->d_pairs, h->d_tiles, (int)J.tiles.size(), J.ty, h->d_mask,
                             aux_grid(h, (int)J.tiles.size()), h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  const std::vector<double> scale = image_scales(h, B);
  if ((p.flags & UOT_AUTOTUNE) && p.tile_rows == 0 && !cached) {
    s = autotune(h, lay, src, dst, st, J);
    if (s != UOT_OK) return s;
  }
  s = scale_default_steps(h, J, scale);
  if (s != UOT_OK) return s;

  // per-pair host bookkeeping
  int32_t* h_active = h->h_i32;
  int32_t* h_iters = h->h_i32 + B;
  int32_t* h_status = h->h_i32 + 2 * B;
  std::vector<double> xnorm(B), relres(B, std::nan(""));
  for (int b = 0; b < B; ++b) {
    const double* S = h->h_sums + (size_t)b * NS;
    xnorm[b] = std::sqrt(S[U_SQS]) + std::sqrt(S[U_SQD]);
    h_active[b] = 1;
    h_iters[b] = 0;
    h_status[b] = UOT_MAX_ITER;
    if (p.mode == UOT_DIST && !warm && S[U_SQS] == 0.0 && S[U_SQD] == 0.0) {
      h_active[b] = 0;  // zero images: the zero state is optimal
      h_status[b] = UOT_CONVERGED;
      relres[b] = 0.0;
    }
    if (p.max_iter == 0 && h_active[b]) h_active[b] = 0;
  }
  int32_t* d_active = h->d_i32;
  int32_t* d_iters = h->d_i32 + B;
  int32_t* d_status = h->d_i32 + 2 * B;
  double* d_rel = h->d_f64;
  double* d_xn = h->d_f64 + B;
  double* d_alpha = h->d_f64 + 2 * B;
  HIPCHK(hipMemcpyAsync(h->d_i32, h->h_i32, (size_t)B * 3 * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(d_xn, xnorm.data(), B * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(d_rel, relres.data(), B * sizeof(double), hipMemcpyHostToDevice, h->stream));
  std::vector<double> alpha0(B, 0.5);
  HIPCHK(hipMemcpyAsync(d_alpha, alpha0.data(), B * sizeof(double), hipMemcpyHostToDevice, h->stream));
  s = upload_live(h, J, h_active);
  if (s != UOT_OK) return s;

  Launch L{};
  L.h = h;
  L.J = &J;
  L.resid = resid;
  L.grid_iter = iter_grid(h, p.mode, resid, bcn_of(p), J.shape, (int)J.tiles.size());
  L.grid_single = iter_grid(h, p.mode, resid, bcn_of(p), shape_single(J.shape), (int)J.tiles.size());
  if (shape_steps(J.shape) > 1) L.grid_chk = iter_grid(h, p.mode, resid, bcn_of(p), J.shape, (int)J.tiles.size(), true);
  L.grid_aux = aux_grid(h, (int)J.tiles.size());
  const Planes A = planes_of(*st), Bp = shadow_planes(h);
  const float* cptr = p.mode == UOT_DIST ? h->cplane : nullptr;
  L.fwd = IterArgs{A, Bp, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, d_active};
  L.bwd = IterArgs{Bp, A, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, d_active};
  L.chk = CheckArgs{A, Bp, 0, 0, cptr, src, dst, h->d_pairs, h->d_tiles, (int32_t)J.tiles.size(), J.ty, d_active,
                    h->d_partial};
  const bool record = (p.flags & UOT_RECORD_HISTORY) != 0;
  const bool check = p.tol > 0.0 || record;
  int W = std::max(2, p.check_every > 0 ? p.check_every : 20);
  W += W & 1;
  const bool adaptive = check && (p.flags & UOT_ADAPTIVE_STEPS);
  L.dec = DecideArgs{h->d_pairs, h->d_sums, d_xn, d_active, d_iters, d_status, d_rel, B, W,
                     p.max_iter, check ? 1 : 0, 0, p.mode, n_identity(p.mode, p.balanced), p.tol,
                     adaptive ? 1 : 0, d_alpha, p.mu, p.rho, 0, 0};

  int n_active = 0;
  for (int b = 0; b < B; ++b) n_active += h_active[b];
  // Windows of W iterations.  Without a check the last window of the solve is
  // the tail, so the solve always ends in a single-iteration launch (the final
  // evaluation compares the last two iterates).
  const int nwin = check ? p.max_iter / W : std::max(0, p.max_iter - 1) / W;
  const int tail = p.max_iter - nwin * W;
  const bool use_graph = !(p.flags & UOT_NO_GRAPH);
  const int per = window_launches(L, W, check);  // launches per window
  // windows: the device decides convergence; the host polls every few windows
  // (every window when the history is recorded).  A full burst of windows
  // between polls replays one captured graph (an even number of windows when
  // a window flips the copy, so a burst starts and ends in the same copy); a
  // shorter last burst replays the one-window graphs.
  // UOT_PROFILE: one window per poll, each bracketed by events
  const bool prof = h->prof != nullptr && !h->borrowed;
  long solve_no = 0;
  if (prof) {
    for (auto& e : h->pev)
      if (!e) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipStreamSynchronize(h->stream));
    solve_no = ++h->prof_solves;
    std::fprintf(h->prof, "uot_profile solve=%ld setup pairs=%d tiles=%zu shape=%d window=%d check=%d host_ms=%.3f\n",
                 solve_no, B, J.tiles.size(), J.shape, W, check ? 1 : 0, 1e3 * timer.seconds());
  }
  int poll = (record || prof) ? 1 : std::min(32, std::max(1, 256 / W));
  if ((per & 1) && poll > 1) poll += poll & 1;
  hipGraphExec_t gx[2] = {nullptr, nullptr}, gxn = nullptr;
  if (n_active > 0 && nwin > 0 && use_graph) {
    s = get_graph(L, W, check, 1, 0, &gx[0]);
    if (s != UOT_OK) return s;
    if (per & 1) {
      s = get_graph(L, W, check, 1, 1, &gx[1]);
      if (s != UOT_OK) return s;
    }
    if (poll > 1 && nwin >= poll) {
      s = get_graph(L, W, check, poll, 0, &gxn);
      if (s != UOT_OK) return s;
    }
  }
  h->have_hist = record;
  h->hist.assign(record ? B : 0, {});
  std::vector<double> hrel(record ? B : 0);
  std::vector<int32_t> hprev_active(record ? B : 0);
  int done_iters = 0;  // iterations of pairs that never stop early (fixed mode)
  int w = 0;
  int par = 0;  // copy holding the iterate of the pairs still running
  while (w < nwin && n_active > 0) {
    const int burst = std::min(poll, nwin - w);
    if (prof) HIPCHK(hipEventRecord(h->pev[0], h->stream));
    if (gxn && burst == poll) {
      HIPCHK(hipGraphLaunch(gxn, h->stream));
      par ^= (burst * per) & 1;
    } else {
      for (int i = 0; i < burst; ++i) {
        if (gx[par]) {
          HIPCHK(hipGraphLaunch(gx[par], h->stream));
        } else {
          s = enqueue_window(L, W, check, par);
          if (s != UOT_OK) return s;
        }
        par ^= per & 1;
      }
    }
    w += burst;
    done_iters += burst * W;
    float prof_ms = 0.f;
    if (prof) {
      HIPCHK(hipEventRecord(h->pev[1], h->stream));
      HIPCHK(hipEventSynchronize(h->pev[1]));
      HIPCHK(hipEventElapsedTime(&prof_ms, h->pev[0], h->pev[1]));
      if (!check)
        std::fprintf(h->prof, "uot_profile solve=%ld window=%d iters=%d live_pairs=%d gpu_ms=%.4f\n", solve_no, w,
                     done_iters, n_active, prof_ms);
    }
    if (check) {
      if (record) {
        for (int b = 0; b < B; ++b) hprev_active[b] = h_active[b];
        HIPCHK(hipMemcpyAsync(hrel.data(), d_rel, B * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      }
      HIPCHK(hipMemcpyAsync(h->h_i32, h->d_i32, (size_t)B * 3 * sizeof(int32_t), hipMemcpyDeviceToHost,
                            h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      if (record)
        for (int b = 0; b < B; ++b)
          if (hprev_active[b]) h->hist[b].emplace_back(h->h_i32[B + b], hrel[b]);
      int now = 0;
      for (int b = 0; b < B; ++b) now += h_active[b] ? 1 : 0;
      if (prof)
        std::fprintf(h->prof, "uot_profile solve=%ld window=%d iters=%d live_pairs=%d stopped=%d gpu_ms=%.4f\n",
                     solve_no, w, done_iters, n_active, n_active - now, prof_ms);
      if (now == 0) {
        n_active = 0;
        break;
      }
      if (now < n_active) {  // compact the live tile list
        s = upload_live(h, J, h_active);
        if (s != UOT_OK) return s;
      }
      n_active = now;
    }
  }
  if (!check) {
    // fixed iteration count: every active pair ran the windows
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  // Pairs that stopped at a check after an odd number of copy flips hold
  // their iterate in the shadow copy: copy it back.  A pair that stopped at
  // the check of window k (iterations k W) has seen k windows.
  if (check && (per & 1)) {
    std::vector<int32_t> back(B, 0);
    bool any = false;
    for (int b = 0; b < B; ++b) {
      const int wins = W > 0 ? h->h_i32[B + b] / W : 0;
      back[b] = !h_active[b] && h->h_i32[2 * B + b] != UOT_MAX_ITER && ((wins * per) & 1);
      any = any || back[b];
    }
    if (any) {
      HIPCHK(hipMemcpyAsync(h->d_mask, back.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
      HIPCHK(launch_copy_active(A, Bp, h->d_pairs, h->d_tiles, (int)J.tiles.size(), J.ty, h->d_mask, L.grid_aux,
                                h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
  }
  // tail iterations for pairs still running, from the copy that holds them;
  // the tail ends in a single-iteration launch
  const bool run_tail = n_active > 0 && tail > 0;
  const std::vector<int> tsched = step_schedule(tail, shape_steps(J.shape), true, false);
  if (run_tail) {
    for (size_t i = 0; i < tsched.size(); ++i)
      HIPCHK(launch_steps(h, resid, J.shape, tsched[i], L.grid_iter, L.grid_single,
                          ((i + par) & 1) ? L.bwd : L.fwd));
    par ^= tsched.size() & 1;
  }
  const bool in_shadow = n_active > 0 && par == 1;
  // final evaluation of every pair, then the final decision
  CheckArgs fin = L.chk;
  if (p.max_iter == 0) fin.B = A;  // no iteration ran: no previous iterate
  fin.swap_active = in_shadow ? 1 : 0;
  fin.all_pairs = 1;
  HIPCHK(launch_check(p.mode, resid, bcn_of(p), L.grid_aux, fin, h->stream));
  DecideArgs fd = L.dec;
  fd.W = check ? (run_tail ? tail : 0) : (done_iters + (run_tail ? tail : 0));
  fd.check = 1;
  fd.tol = check ? p.tol : 0.0;
  fd.final_pass = 1;
  // no iteration since the last window's check: its rel_res is the current
  // iterate's (the copy behind may hold an older iterate than the previous)
  fd.keep_rel = (check && !run_tail && nwin > 0) ? 1 : 0;
  if (in_shadow) {
    // pairs still active hold their iterate in the shadow copy: copy it back
    // before the decision clears their flag
    HIPCHK(launch_copy_active(A, Bp, h->d_pairs, h->d_tiles, (int)J.tiles.size(), J.ty, d_active, L.grid_aux,
                              h->stream));
  }
  // Pairs that stopped in an earlier window keep their recorded status and
  // rel_res; the final decision re-evaluates only still-active pairs.
  HIPCHK(launch_reduce_decide(fd, h->d_partial, h->stream));
  HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, (size_t)B * NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(h->h_i32, h->d_i32, (size_t)B * 3 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(relres.data(), d_rel, B * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (adaptive)
    HIPCHK(hipMemcpyAsync(J.pairs.data(), h->d_pairs, B * sizeof(PairInfo), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<double> sums(h->h_sums, h->h_sums + (size_t)B * NS);
  std::vector<double> duals;
  const bool need_dual = p.mode != UOT_DIST && resid != R_BAL;
  if (need_dual) {
    s = prox_duals(h, J, src, dst, st->a, sums.data(), duals);
    if (s != UOT_OK) return s;
  }
  std::vector<double> bal(B, std::nan(""));
  if (p.mode == UOT_DIST && resid == R_BAL && p.bc == 0 && !h->borrowed) {
    s = balanced_primal(h, J, src, dst, st, bal);
    if (s != UOT_OK) return s;
  }
  const double secs = timer.seconds();
  if (prof) {
    std::fprintf(h->prof, "uot_profile solve=%ld end windows=%d tail=%d host_ms=%.3f\n", solve_no, w,
                 run_tail ? tail : 0, 1e3 * secs);
    std::fflush(h->prof);
  }
  for (int b = 0; b < B; ++b) {
    uot_report& r = reps[b];
    std::memset(&r, 0, sizeof(r));
    Reporter::fill(p, J.pairs[b], sums.data() + (size_t)b * NS, xnorm[b], &r, need_dual ? duals[b] : 0.0,
                   need_dual, bal[b]);
    r.iters = h->h_i32[B + b];
    r.status = h->h_i32[2 * B + b];
    r.seconds = secs;
    r.tile_rows = J.shape;
    r.cold_start = cold[b];
    // rel_res as the stopping rule last evaluated it (at the check where the
    // pair stopped, or at its last iterate)
    if (std::isfinite(relres[b])) r.rel_res = relres[b];
    // the final evaluation, unless the pair stopped at an earlier check
    if (record && (h->hist[b].empty() || h->hist[b].back().first != r.iters))
      h->hist[b].emplace_back(r.iters, r.rel_res);
  }
  return UOT_OK;
}

// iters iterations from `in` into `out` (see uot_step).
uot_status step_core(uot_handle* h, const Layout& L, const float* src, const float* dst, const uot_state* in,
                     uot_state* out, int32_t iters) {
  const uot_params& p = h->prm;
  if (!src || !dst || !in || !out || iters < 0) return UOT_ERR_ARG;
  uot_status s = validate_state(p, in);
  if (s != UOT_OK) return s;
  s = validate_state(p, out);
  if (s != UOT_OK) return s;
  const Planes pi = planes_of(*in), po = planes_of(*out);
  const float* const vin[6] = {pi.Mx, pi.My, pi.r, pi.a, pi.x0, pi.x1};
  const float* const vout[6] = {po.Mx, po.My, po.r, po.a, po.x0, po.x1};
  for (const float* a : vin)
    for (const float* b : vout)
      if (a && a == b) return UOT_ERR_ARG;
  Job J;
  const bool ptrs_aligned = aligned4(src) && aligned4(dst) && aligned4(in->Mx) && aligned4(in->My) &&
                            aligned4(in->r) && aligned4(in->a) && aligned4(in->x0) && aligned4(in->x1) &&
                            aligned4(out->Mx) && aligned4(out->My) && aligned4(out->r) && aligned4(out->a) &&
                            aligned4(out->x0) && aligned4(out->x1);
  s = plan(h, L, J, 0, nullptr, ptrs_aligned);
  if (s != UOT_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
  const int resid = resid_of(p);
  const bool need[6] = {true, true, resid != R_BAL, true, p.mode == UOT_PROX, p.mode != UOT_DIST};
  if (iters == 0) {
    const size_t n = (size_t)J.total_px * sizeof(float);
    float* const dsts[6] = {po.Mx, po.My, po.r, po.a, po.x0, po.x1};
    for (int i = 0; i < 6; ++i)
      if (need[i]) HIPCHK(hipMemcpyAsync(dsts[i], vin[i], n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return UOT_OK;
  }
  s = ensure_workspace(h, J);
  if (s != UOT_OK) return s;
  HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), J.B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                        h->stream));
  s = run_setup(h, J, src, dst, in, true, false);  // validates `in`, writes c; the state is only read
  if (s != UOT_OK) return s;
  s = check_setup_sums(h, J, true);
  if (s != UOT_OK) return s;
  s = scale_default_steps(h, J, image_scales(h, J.B));
  if (s != UOT_OK) return s;
  for (int b = 0; b < J.B; ++b) h->h_i32[b] = 1;
  HIPCHK(hipMemcpyAsync(h->d_i32, h->h_i32, (size_t)J.B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  s = upload_live(h, J, h->h_i32);
  if (s != UOT_OK) return s;
  const int grid = iter_grid(h, p.mode, resid, bcn_of(p), J.shape, (int)J.tiles.size());
  const int grid1 = iter_grid(h, p.mode, resid, bcn_of(p), shape_single(J.shape), (int)J.tiles.size());
  const Planes sh = shadow_planes(h);
  const float* cptr = p.mode == UOT_DIST ? h->cplane : nullptr;
  // launch i writes `out` when an even number of launches follows it, else
  // the shadow; the first reads `in`, every other one its predecessor's output
  const std::vector<int> sched = step_schedule(iters, shape_steps(J.shape), false, false);
  const int n = (int)sched.size();
  Planes from = pi;
  for (int i = 0; i < n; ++i) {
    const Planes to = ((n - 1 - i) % 2 == 0) ? po : sh;
    const IterArgs a{from, to, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, h->d_i32};
    HIPCHK(launch_steps(h, resid, J.shape, sched[i], grid, grid1, a));
    from = to;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return UOT_OK;
}

// Back-to-back fused-iteration launches over a batch layout, replayed from one
// captured graph and bracketed by events (every pair live).
uot_status time_core(uot_handle* h, const Layout& L, const float* src, const float* dst, uot_state* st,
                     int32_t n, double* ms_per_iter, int32_t* tile_rows) {
  const int B = L.B;
  const uot_params& p = h->prm;
  if (!src || !dst || !ms_per_iter || n < 1) return UOT_ERR_ARG;
  uot_status s = validate_state(p, st);
  if (s != UOT_OK) return s;
  Job J;
  const bool ptrs_aligned = aligned4(src) && aligned4(dst) && aligned4(st->Mx) && aligned4(st->My) &&
                            aligned4(st->r) && aligned4(st->a) && aligned4(st->x0) && aligned4(st->x1);
  s = plan(h, L, J, 0, nullptr, ptrs_aligned);
  if (s != UOT_OK) return s;
  if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
  s = ensure_workspace(h, J);
  if (s != UOT_OK) return s;
  HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), B * sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                        h->stream));
  s = run_setup(h, J, src, dst, st, true, false);
  if (s != UOT_OK) return s;
  s = scale_default_steps(h, J, image_scales(h, B));
  if (s != UOT_OK) return s;
  for (int b = 0; b < B; ++b) h->h_i32[b] = 1;
  HIPCHK(hipMemcpyAsync(h->d_i32, h->h_i32, (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  s = upload_live(h, J, h->h_i32);
  if (s != UOT_OK) return s;
  const int resid = resid_of(p);
  const int grid = iter_grid(h, p.mode, resid, bcn_of(p), J.shape, (int)J.tiles.size());
  const Planes A = planes_of(*st), Bp = shadow_planes(h);
  const float* cptr = p.mode == UOT_DIST ? h->cplane : nullptr;
  const IterArgs fwd{A, Bp, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, h->d_i32};
  const IterArgs bwd{Bp, A, cptr, src, dst, h->d_pairs, h->d_live, h->d_nlive, h->d_i32};
  const int nn = n + (n & 1);
  const int T = shape_steps(J.shape);  // iterations per launch
  // the launches are captured once and replayed, as the solver does
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < nn && le == hipSuccess; ++i)
    le = launch_steps(h, resid, J.shape, T, grid, grid, (i & 1) ? bwd : fwd);
  hipError_t ce = hipStreamEndCapture(h->stream, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return UOT_ERR_DEVICE;
  }
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(ie);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipGraphLaunch(ex, h->stream));  // warm replay
  HIPCHK(hipEventRecord(e0, h->stream));
  HIPCHK(hipGraphLaunch(ex, h->stream));
  HIPCHK(hipEventRecord(e1, h->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ex);
  *ms_per_iter = (double)ms / nn;
  if (tile_rows) *tile_rows = J.shape;
  return UOT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// The no-allocation workspace: one fixed device array per GPU (each device
// holds its own copy at its own address), located once per device with
// hipGetSymbolAddress; host code uses only that address, never the array's
// name, which on the host is a stand-in symbol and not a device address.
static __device__ __align__(256) unsigned char scratch[UOT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// The scratch address on the current device `dev`.
uot_status scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return UOT_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return UOT_ERR_DEVICE;
    g_scratch[dev] = (unsigned char*)p;
  }
  *out = g_scratch[dev];
  return UOT_OK;
}

// Hands out 256-byte-aligned pieces of the scratch.
struct Carver {
  unsigned char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n, size_t* cap) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(base + off);
    off += std::max<size_t>(n, 1) * sizeof(T);
    *cap = std::max<size_t>(n, 1);
    return p;
  }
};

}  // namespace

extern "C" {

uot_status uot_solve_noalloc(const uot_params* prm, void* hip_stream, const float* src, const float* dst,
                             uot_state* st, uot_report* rep) {
  if (!prm || !src || !dst || !st || !rep) return UOT_ERR_ARG;
  uot_status s = uot_check_params(prm);
  if (s != UOT_OK) return s;
  if (prm->flags & UOT_AUTOTUNE) return UOT_ERR_ARG;
  if (prm->nx < 1 || prm->ny < 1) return UOT_ERR_SHAPE;
  const int32_t nx = prm->nx, ny = prm->ny, pitch = prm->pitch > 0 ? prm->pitch : prm->nx;
  const int64_t off = 0;
  if ((int64_t)pitch * (ny - 1) + nx > (int64_t)UOT_NOALLOC_MAX_PIXELS) return UOT_ERR_TOO_LARGE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UOT_ERR_DEVICE;
  unsigned char* base = nullptr;
  s = scratch_of(dev, &base);
  if (s != UOT_OK) return s;
  try {
    uot_handle h;
    h.borrowed = true;
    h.prm = *prm;
    h.prm.flags |= UOT_NO_GRAPH;
    h.stream = (hipStream_t)hip_stream;
    h.device = dev;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      h.num_cu = cu;
    const Layout lay{1, &nx, &ny, &pitch, &off};
    Job J;
    const bool ptrs_aligned = aligned4(src) && aligned4(dst) && aligned4(st->Mx) && aligned4(st->My) &&
                              aligned4(st->r) && aligned4(st->a) && aligned4(st->x0) && aligned4(st->x1);
    s = plan(&h, lay, J, 0, nullptr, ptrs_aligned);  // the plan solve_core will make: sizes only
    if (s != UOT_OK) return s;
    const size_t px = (size_t)J.total_px, nt = J.tiles.size();
    if (nt > (size_t)UOT_NOALLOC_MAX_TILES) return UOT_ERR_TOO_LARGE;
    Carver c{base};
    for (int i = 0; i < 6; ++i) h.B[i] = c.take<float>(px, &h.capB[i]);
    h.cplane = c.take<float>(px, &h.cap_c);
    h.d_tiles = c.take<Tile>(nt, &h.cap_tiles);
    h.d_live = c.take<Tile>(nt, &h.cap_live);
    h.d_nlive = c.take<int32_t>(1, &h.cap_nlive);
    h.d_partial = c.take<double>(nt * NS, &h.cap_partial);
    h.d_pairs = c.take<PairInfo>(1, &h.cap_pairs);
    h.d_sums = c.take<double>(NS, &h.cap_sums);
    h.d_i32 = c.take<int32_t>(4, &h.cap_i32);
    h.d_f64 = c.take<double>(3, &h.cap_f64);
    h.d_invs = c.take<float>(1, &h.cap_invs);
    h.d_mask = c.take<int32_t>(1, &h.cap_mask);
    if (c.off > (size_t)UOT_NOALLOC_SCRATCH_BYTES) return UOT_ERR_TOO_LARGE;
    // the host side of the per-pair records: plain (pageable) memory
    double hsums[NS];
    int32_t hi32[4];
    h.h_sums = hsums;
    h.cap_hsums = NS;
    h.h_i32 = hi32;
    h.cap_hi32 = 4;
    s = solve_core(&h, lay, src, dst, st, rep);
    if (hipStreamSynchronize(h.stream) != hipSuccess && s == UOT_OK) s = UOT_ERR_DEVICE;
    return s;
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_solve(uot_handle* h, const float* src, const float* dst, uot_state* st, uot_report* rep) {
  if (!h) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.nx < 1 || p.ny < 1) return UOT_ERR_SHAPE;
  const int32_t nx = p.nx, ny = p.ny, pitch = p.pitch > 0 ? p.pitch : p.nx;
  const int64_t off = 0;
  try {
    return solve_core(h, Layout{1, &nx, &ny, &pitch, &off}, src, dst, st, rep);
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_solve_batched(uot_handle* h, int32_t B, const int32_t* nx, const int32_t* ny, const int64_t* offset,
                             const float* src, const float* dst, uot_state* packed, uot_report* reps) {
  return uot_solve_batched_pitched(h, B, nx, ny, nullptr, offset, src, dst, packed, reps);
}

uot_status uot_solve_batched_pitched(uot_handle* h, int32_t B, const int32_t* nx, const int32_t* ny,
                                     const int32_t* pitch, const int64_t* offset, const float* src,
                                     const float* dst, uot_state* packed, uot_report* reps) {
  if (!h) return UOT_ERR_ARG;
  try {
    return solve_core(h, Layout{B, nx, ny, pitch, offset}, src, dst, packed, reps);
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_step(uot_handle* h, const float* src, const float* dst, const uot_state* in, uot_state* out,
                    int32_t iters) {
  if (!h) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.nx < 1 || p.ny < 1) return UOT_ERR_SHAPE;
  const int32_t nx = p.nx, ny = p.ny, pitch = p.pitch > 0 ? p.pitch : p.nx;
  const int64_t off = 0;
  try {
    return step_core(h, Layout{1, &nx, &ny, &pitch, &off}, src, dst, in, out, iters);
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_time_iterations(uot_handle* h, const float* src, const float* dst, uot_state* st, int32_t n,
                               double* ms_per_iter, int32_t* tile_rows) {
  if (!h) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.nx < 1 || p.ny < 1) return UOT_ERR_SHAPE;
  const int32_t nx = p.nx, ny = p.ny, pitch = p.pitch > 0 ? p.pitch : p.nx;
  const int64_t off = 0;
  try {
    return time_core(h, Layout{1, &nx, &ny, &pitch, &off}, src, dst, st, n, ms_per_iter, tile_rows);
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_time_iterations_batched(uot_handle* h, int32_t B, const int32_t* nx, const int32_t* ny,
                                       const int32_t* pitch, const int64_t* offset, const float* src,
                                       const float* dst, uot_state* packed, int32_t n, double* ms_per_iter,
                                       int32_t* tile_rows) {
  if (!h) return UOT_ERR_ARG;
  try {
    return time_core(h, Layout{B, nx, ny, pitch, offset}, src, dst, packed, n, ms_per_iter, tile_rows);
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_objective(uot_handle* h, const float* src, const float* dst, const uot_state* st,
                         const uot_state* prev, uot_report* out) {
  if (!h || !src || !dst || !out) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.nx < 1 || p.ny < 1) return UOT_ERR_SHAPE;
  uot_status s = validate_state(p, st);
  if (s != UOT_OK) return s;
  if (prev && validate_state(p, prev) != UOT_OK) return UOT_ERR_ARG;
  try {
    Timer timer;
    const int32_t nx = p.nx, ny = p.ny, pitch = p.pitch > 0 ? p.pitch : p.nx;
    const int64_t off = 0;
    Job J;
    s = plan(h, Layout{1, &nx, &ny, &pitch, &off}, J);
    if (s != UOT_OK) return s;
    if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
    s = ensure_workspace(h, J);
    if (s != UOT_OK) return s;
    HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                          h->stream));
    // c = q - p is written into the workspace; the state is only read
    SetupArgs sa{};
    sa.src = src;
    sa.dst = dst;
    sa.c = h->cplane;
    sa.st = planes_of(*st);
    sa.mode = p.mode;
    sa.resid = resid_of(p);
    sa.bc = p.bc;
    sa.warm = 1;
    sa.write_state = 0;
    sa.write_c = 1;
    sa.pairs = h->d_pairs;
    sa.tiles = h->d_tiles;
    sa.ntiles = (int32_t)J.tiles.size();
    sa.tile_rows = J.ty;
    sa.partial = h->d_partial;
    HIPCHK(launch_setup(aux_grid(h, sa.ntiles), sa, h->stream));
    HIPCHK(launch_pair_reduce(h->d_pairs, 1, h->d_partial, kMaxSlotsSetup, h->d_sums, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const double xn = std::sqrt(h->h_sums[U_SQS]) + std::sqrt(h->h_sums[U_SQD]);
    s = scale_default_steps(h, J, image_scales(h, 1));
    if (s != UOT_OK) return s;
    int32_t one = 1;
    HIPCHK(hipMemcpyAsync(h->d_i32, &one, sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    const uot_state* q = prev ? prev : st;
    CheckArgs ck{planes_of(*st), planes_of(*q), 0, 1, p.mode == UOT_DIST ? h->cplane : nullptr, src, dst,
                 h->d_pairs, h->d_tiles, (int32_t)J.tiles.size(), J.ty, h->d_i32, h->d_partial};
    HIPCHK(launch_check(p.mode, resid_of(p), bcn_of(p), aux_grid(h, ck.ntiles), ck, h->stream));
    HIPCHK(launch_pair_reduce(h->d_pairs, 1, h->d_partial, kMaxSlotsCheck, h->d_sums, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<double> sums(h->h_sums, h->h_sums + NS);
    std::vector<double> duals;
    const bool need_dual = p.mode != UOT_DIST && resid_of(p) != R_BAL;
    if (need_dual) {
      s = prox_duals(h, J, src, dst, st->a, sums.data(), duals);
      if (s != UOT_OK) return s;
    }
    std::vector<double> bal(1, std::nan(""));
    if (p.mode == UOT_DIST && p.balanced && p.bc == 0) {
      s = balanced_primal(h, J, src, dst, st, bal);
      if (s != UOT_OK) return s;
    }
    std::memset(out, 0, sizeof(*out));
    Reporter::fill(p, J.pairs[0], sums.data(), xn, out, need_dual ? duals[0] : 0.0, need_dual, bal[0]);
    out->status = (sums[S_NONFIN] > 0) ? UOT_DIVERGED : UOT_MAX_ITER;
    out->seconds = timer.seconds();
    return UOT_OK;
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_history(uot_handle* h, int32_t pair, int32_t* iters, double* rel_res, int32_t cap, int32_t* n) {
  if (!h || !n || cap < 0 || !h->have_hist || pair < 0 || pair >= (int32_t)h->hist.size()) return UOT_ERR_ARG;
  const auto& v = h->hist[pair];
  *n = (int32_t)v.size();
  const int32_t m = std::min<int32_t>(cap, (int32_t)v.size());
  for (int32_t i = 0; i < m; ++i) {
    if (iters) iters[i] = v[i].first;
    if (rel_res) rel_res[i] = v[i].second;
  }
  return UOT_OK;
}

uot_status uot_dr_solve(uot_handle* h, const float* src, const float* dst, uot_state* st, double gamma,
                        uot_dr_report* rep) {
  if (!h || !src || !dst || !st || !rep || !(gamma > 0.0) || !std::isfinite(gamma)) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.nx < 1 || p.ny < 1) return UOT_ERR_SHAPE;
  if (p.bc != 0 || (p.pitch != 0 && p.pitch != p.nx)) return UOT_ERR_ARG;
  if (p.max_iter < 0 || p.check_every < 1) return UOT_ERR_ARG;
  const int resid = resid_of(p);
  if (!st->Mx || !st->My || (resid != R_BAL && !st->r) || (p.mode == UOT_PROX && (!st->x0 || !st->x1)) ||
      (p.mode == UOT_PROX_FIXED && !st->x1))
    return UOT_ERR_ARG;
  std::memset(rep, 0, sizeof(*rep));
  try {
    Timer timer;
    const int32_t nx = p.nx, ny = p.ny, pitch = p.nx;
    const int64_t off = 0;
    Job J;
    uot_status s = plan(h, Layout{1, &nx, &ny, &pitch, &off}, J);
    if (s != UOT_OK) return s;
    if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
    s = ensure_workspace(h, J);
    if (s != UOT_OK) return s;
    HIPCHK(hipMemcpyAsync(h->d_pairs, J.pairs.data(), sizeof(PairInfo), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_tiles, J.tiles.data(), J.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                          h->stream));
    // input checks only (the state is neither read nor written here)
    SetupArgs sa{};
    sa.src = src;
    sa.dst = dst;
    sa.c = h->cplane;
    sa.st = planes_of(*st);
    sa.mode = p.mode;
    sa.resid = resid;
    sa.bc = p.bc;
    sa.warm = 0;
    sa.write_state = 0;
    sa.write_c = 0;
    sa.pairs = h->d_pairs;
    sa.tiles = h->d_tiles;
    sa.ntiles = (int32_t)J.tiles.size();
    sa.tile_rows = J.ty;
    sa.partial = h->d_partial;
    HIPCHK(launch_setup(aux_grid(h, sa.ntiles), sa, h->stream));
    HIPCHK(launch_pair_reduce(h->d_pairs, 1, h->d_partial, kMaxSlotsSetup, h->d_sums, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_sums, h->d_sums, NS * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    s = check_setup_sums(h, J, false);
    if (s != UOT_OK) return s;

    const long n = (long)nx * ny;
    s = ensure_poisson(h, (size_t)n);
    if (s != UOT_OK) return s;
    const float *cx = nullptr, *cy = nullptr;
    if ((s = get_dct(h, nx, &cx)) != UOT_OK || (s = get_dct(h, ny, &cy)) != UOT_OK) return s;
    HIPCHK(grow(&h->drbuf, &h->cap_drbuf, (size_t)n * 10));
    const int nb = dr_blocks(n);
    HIPCHK(grow(&h->d_drp, &h->cap_drp, (size_t)3 * nb));
    if (!h->h_drp)
      HIPCHK(hipHostMalloc((void**)&h->h_drp, 3 * DR_MAX_BLOCKS * sizeof(double), hipHostMallocDefault));
    DrArgs a{};
    float* wb = h->drbuf;
    float* ub = h->drbuf + 5 * n;
    a.z = planes_of(*st);
    a.z.a = nullptr;
    if (resid == R_BAL) a.z.r = nullptr;
    if (p.mode == UOT_DIST) a.z.x0 = a.z.x1 = nullptr;
    if (p.mode == UOT_PROX_FIXED) a.z.x0 = nullptr;
    a.w = Planes{wb, wb + n, a.z.r ? wb + 2 * n : nullptr, nullptr, a.z.x0 ? wb + 3 * n : nullptr,
                 a.z.x1 ? wb + 4 * n : nullptr};
    a.u = Planes{ub, ub + n, a.z.r ? ub + 2 * n : nullptr, nullptr, a.z.x0 ? ub + 3 * n : nullptr,
                 a.z.x1 ? ub + 4 * n : nullptr};
    a.src = src;
    a.dst = dst;
    a.nx = nx;
    a.ny = ny;
    a.mode = p.mode;
    a.resid = resid;
    a.aniso = p.norm == UOT_NORM_ANISO ? 1 : 0;
    a.gamma = (float)gamma;
    a.mu = (float)p.mu;
    a.rho = (float)p.rho;
    // identity blocks of K among the variables: K K^T = D D* + nid I
    const int nid = (a.z.r ? 1 : 0) + (a.z.x0 ? 1 : 0) + (a.z.x1 ? 1 : 0);
    float* e = h->pw[3];
    float* phi = h->pw[2];
    HIPCHK(hipMemsetAsync(h->drbuf, 0, (size_t)n * 5 * sizeof(float), h->stream));
    auto iteration = [&](bool record) -> uot_status {
      HIPCHK(launch_dr_prox_rhs(a, e, h->stream));
      HIPCHK(poisson_solve(cx, cy, nx, ny, (float)nid, e, phi, h->pw[0], h->pw[1], h->stream));
      HIPCHK(launch_dr_update(a, phi, record ? 1 : 0, h->d_drp, h->stream));
      return UOT_OK;
    };
    const bool use_graph = !(p.flags & UOT_NO_GRAPH);
    const int W = p.check_every;
    const void* key[4] = {src, dst, st->Mx, (const void*)(intptr_t)n};
    if (use_graph && (!h->drexec || h->dr_w != W || std::memcmp(key, h->dr_key, sizeof(key)) != 0 ||
                      p.max_iter / W == 0)) {
      if (h->drexec) (void)hipGraphExecDestroy(h->drexec);
      h->drexec = nullptr;
    }
    int k = 0;
    bool conv = false;
    double res = std::nan("");
    auto test = [&]() -> uot_status {
      HIPCHK(hipMemcpyAsync(h->h_drp, h->d_drp, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      double d2 = 0.0, z2 = 0.0;
      for (int b = 0; b < nb; ++b) {
        d2 += h->h_drp[2 * b];
        z2 += h->h_drp[2 * b + 1];
      }
      res = std::sqrt(d2) / std::max(1.0, std::sqrt(z2));
      if (!std::isfinite(res)) return UOT_OK;
      if (p.tol > 0.0 && res <= p.tol) conv = true;
      return UOT_OK;
    };
    struct Events {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      ~Events() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
      }
    } ev;
    HIPCHK(hipEventCreate(&ev.e0));
    HIPCHK(hipEventCreate(&ev.e1));
    HIPCHK(hipEventRecord(ev.e0, h->stream));
    while (k + W <= p.max_iter && !conv) {
      if (use_graph) {
        if (!h->drexec) {
          hipGraph_t g = nullptr;
          HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
          uot_status cs = UOT_OK;
          for (int i = 0; i < W && cs == UOT_OK; ++i) cs = iteration(i == W - 1);
          hipError_t ce = hipStreamEndCapture(h->stream, &g);
          if (cs != UOT_OK || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return cs != UOT_OK ? cs : UOT_ERR_DEVICE;
          }
          hipError_t ie = hipGraphInstantiate(&h->drexec, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (ie != hipSuccess) return UOT_ERR_DEVICE;
          h->dr_w = W;
          std::memcpy(h->dr_key, key, sizeof(key));
        }
        HIPCHK(hipGraphLaunch(h->drexec, h->stream));
      } else {
        for (int i = 0; i < W; ++i) {
          s = iteration(i == W - 1);
          if (s != UOT_OK) return s;
        }
      }
      k += W;
      if ((s = test()) != UOT_OK) return s;
      if (!std::isfinite(res)) break;
    }
    if (!conv && std::isfinite(res) && k < p.max_iter) {
      const int tail = p.max_iter - k;
      for (int i = 0; i < tail; ++i) {
        s = iteration(i == tail - 1);
        if (s != UOT_OK) return s;
      }
      k = p.max_iter;
      if ((s = test()) != UOT_OK) return s;
    }
    HIPCHK(hipEventRecord(ev.e1, h->stream));
    // objective of z and its constraint violation
    HIPCHK(launch_dr_objective(a, h->d_drp, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_drp, h->d_drp, 3 * nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double fm = 0.0, pen = 0.0, quad = 0.0;
    for (int b = 0; b < nb; ++b) {
      fm += h->h_drp[3 * b];
      pen += h->h_drp[3 * b + 1];
      quad += h->h_drp[3 * b + 2];
    }
    HIPCHK(launch_dr_rhs(a, 1, nullptr, h->d_drp, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_drp, h->d_drp, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double f2 = 0.0;
    for (int b = 0; b < nb; ++b) f2 += h->h_drp[b];
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    rep->iters = k;
    rep->status = !std::isfinite(res) ? UOT_DIVERGED : (conv ? UOT_CONVERGED : UOT_MAX_ITER);
    rep->fixed_point_res = res;
    rep->objective = fm + (resid != R_BAL ? p.mu * pen : 0.0) + (p.mode == UOT_DIST ? 0.0 : quad / (2.0 * p.rho));
    rep->infeasibility = std::sqrt(f2);
    rep->ms_per_iter = k > 0 ? (double)ms / k : 0.0;
    rep->seconds = timer.seconds();
    return UOT_OK;
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_poisson(uot_handle* h, int32_t nx, int32_t ny, double alpha, const float* rhs, float* phi) {
  if (!h || !rhs || !phi || !(alpha >= 0.0) || !std::isfinite(alpha)) return UOT_ERR_ARG;
  if (nx < 1 || ny < 1) return UOT_ERR_SHAPE;
  if (rhs == phi) return UOT_ERR_ARG;
  try {
    if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
    uot_status s = ensure_poisson(h, (size_t)nx * ny);
    if (s != UOT_OK) return s;
    s = poisson_grid(h, nx, ny, alpha, rhs, phi);
    if (s != UOT_OK) return s;
    HIPCHK(hipStreamSynchronize(h->stream));
    return UOT_OK;
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

uot_status uot_init_poisson(uot_handle* h, int32_t B, const int32_t* nx, const int32_t* ny, const int64_t* offset,
                            const float* src, const float* dst, uot_state* packed) {
  return uot_init_poisson_pitched(h, B, nx, ny, nullptr, offset, src, dst, packed);
}

uot_status uot_init_poisson_pitched(uot_handle* h, int32_t B, const int32_t* nx, const int32_t* ny,
                                    const int32_t* pitch, const int64_t* offset, const float* src,
                                    const float* dst, uot_state* packed) {
  if (!h || !src || !dst) return UOT_ERR_ARG;
  const uot_params& p = h->prm;
  if (p.bc != 0) return UOT_ERR_ARG;
  uot_status s = validate_state(p, packed);
  if (s != UOT_OK) return s;
  try {
    Job J;
    s = plan(h, Layout{B, nx, ny, pitch, offset}, J, 8);
    if (s != UOT_OK) return s;
    if (hipSetDevice(h->device) != hipSuccess) return UOT_ERR_DEVICE;
    size_t maxpx = 0;
    for (const PairInfo& P : J.pairs) maxpx = std::max<size_t>(maxpx, (size_t)P.nx * P.ny);
    s = ensure_poisson(h, maxpx);
    if (s != UOT_OK) return s;
    for (int b = 0; b < B; ++b) {
      const PairInfo& P = J.pairs[b];
      const long o = P.off;
      // rhs = c = dst - src: the infeasibility of the zero flux
      HIPCHK(launch_infeasibility(nullptr, nullptr, src + o, dst + o, h->pw[3], P.nx, P.ny, P.pitch, h->stream));
      s = poisson_grid(h, P.nx, P.ny, 0.0, h->pw[3], h->pw[2]);
      if (s != UOT_OK) return s;
      Planes st = planes_of(*packed);
      Planes at{st.Mx + o, st.My + o, st.r ? st.r + o : nullptr, st.a + o, st.x0 ? st.x0 + o : nullptr,
                st.x1 ? st.x1 + o : nullptr};
      HIPCHK(launch_poisson_start(h->pw[2], src + o, dst + o, at, P.nx, P.ny, P.pitch, p.mode, p.balanced,
                                  h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return UOT_OK;
  } catch (...) {
    return UOT_ERR_OOM;
  }
}

}  // extern "C"
