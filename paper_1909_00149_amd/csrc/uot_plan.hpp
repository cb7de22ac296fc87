// Host planning of the solver that needs no GPU: parameter checks, the
// step-size bound of Theorem 1, kernel shape codes, launch schedules of a
// check window and the validation of a batch layout.  Plain C++ (no HIP), so
// that it also builds into the host-only sanitizer test of the planner.
#pragma once

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/uot.h"

namespace uot {
namespace planner {

constexpr double kPi = 3.14159265358979323846;

// lambda_max of the 1-D factor of D D*: zero-flux ends (bc = 0) or the
// literal boundary (bc = 1, the last edge free).
inline double lam1d(int n, int bc) {
  if (bc == 0) {
    const double s = std::sin(kPi * (n - 1) / (2.0 * n));
    return 4.0 * s * s;
  }
  const double s = std::sin(kPi * (2.0 * n - 1) / (2.0 * (2.0 * n + 1)));
  return 4.0 * s * s;
}

// Identity blocks of K in each mode (x0, x1 and r where they are free).
inline int n_identity(int mode, int balanced) {
  const int base = mode == UOT_DIST ? 1 : (mode == UOT_PROX ? 3 : 2);
  return base - (balanced ? 1 : 0);
}

// ||K||^2 = lambda_max(D D*) (the Kronecker sum of the two 1-D factors) + the
// identity blocks; -1 on bad arguments.
inline double knorm2_of(int32_t nx, int32_t ny, int32_t mode, int32_t balanced, int32_t bc) {
  if (nx < 1 || ny < 1 || mode < 0 || mode > 2 || bc < 0 || bc > 1) return -1.0;
  return lam1d(nx, bc) + lam1d(ny, bc) + n_identity(mode, balanced ? 1 : 0);
}

// Default steps (tau1 = tau2 = 0 in the params).  The problem is
// 1-homogeneous in the images: scaling p and q by t scales M and r by t and
// leaves the multiplier a unchanged, and running the iteration on the
// scaled images is running it on the originals with tau1 / t and tau2 t.
// The default therefore follows the image scale s (the largest |pixel| of
// the pair's two images; 1 if that is zero):
//   tau1 = 0.99 s / ||K||,   tau2 = 0.99 / (s ||K||),
// so the iterates of scaled images are the scaled iterates, and the
// product tau1 tau2 ||K||^2 = 0.98 < 1 (Theorem 1) whatever s is.
inline void default_steps(double k2, double scale, double* t1, double* t2) {
  const double k = std::sqrt(k2);
  *t1 = 0.99 * scale / k;
  *t2 = 0.99 / (scale * k);
}


// Default kernel shape by size (the codes are listed with shape_rows below).
// Measured on one MI355X, per iteration: the blocked kernels take 1.55 us at
// 256^2 with 64 x 4 tiles (1.78 with 64 x 8; single-step: 3.7 us, the launch
// floor), 2.1 us at 512^2 with 64 x 8 (2.5 with 64 x 4), 60 us at 4096^2
// (121) and 56 us on a 14.7 Mpx ragged batch (110).
inline int heuristic_shape(long npx) {
  // temporally blocked, 4 iterations per launch: the smaller the grid, the
  // smaller the tile, so that enough workgroups hide the latency of the
  // steps' barriers; above 2^18 pixels 64 x 16 tiles (less halo work)
  return npx <= (1L << 16) ? 4004 : (npx <= (1L << 18) ? 4008 : 4016);
}

// Kernel shape codes: rows (4, 8, 16, 32) = the scalar kernel; 100 + rows =
// the vectorised kernel; 300 + rows = the same with non-temporal stores;
// 1000 * T + rows = T iterations per launch (temporally blocked), whose
// single steps run the vectorised kernel of the same rows (the scalar one
// for 8 rows, which the vectorised form does not have).
inline int shape_rows(int code) { return code >= 1000 ? code % 1000 : code % 100; }
inline int shape_steps(int code) { return code >= 1000 ? code / 1000 : 1; }
inline int shape_single(int code) {
  if (code < 1000) return code;
  const int rows = code % 1000;
  return rows % 16 == 0 ? 100 + rows : rows;
}
// The blocked kernels address a tile's region by 32-bit byte offsets from
// its first cell, which hold (region rows + 1) x pitch pixels for every
// blocked shape (at most 49 rows) while the pitch is at most 2^24; wider
// rows run the single-step kernel of the same rows.
constexpr long kBlockedMaxPitch = 1L << 24;
inline bool blocked_pitch_ok(int B, const int32_t* nx, const int32_t* pitch) {
  for (int b = 0; b < B; ++b)
    if ((long)(pitch ? pitch[b] : nx[b]) > kBlockedMaxPitch) return false;
  return true;
}

// Steps of the check variant of a blocked shape (the window's last launch,
// halo one more than that): 4 for the 4- and 8-step shapes of 4 to 16
// rows, 2 for 2016 and the 32-row shapes (fewer registers).
inline int shape_chk_steps(int code) {
  switch (code) {
    case 4004: case 4008: case 4016: case 8016: return 4;
    case 2016: case 4032: case 8032: return 2;
  }
  return 1;
}
inline bool shape_known(int code) {
  switch (code) {
    case 4: case 8: case 16: case 32: case 116: case 132: case 316: case 332:
    case 4004: case 4008: case 2016: case 4016: case 8016: case 4032: case 8032: return true;
  }
  return false;
}

// Iterations per launch for n iterations with up to T per launch.  With
// last_single the final launch runs one iteration (the convergence check
// compares the last two iterates, which must both be in the ping-pong
// buffers); with even the number of launches is even, so the iterate ends in
// the buffer it started in.  The iterations are spread evenly over the
// launches.
inline std::vector<int> step_schedule(int n, int T, bool last_single, bool even) {
  std::vector<int> v;
  if (n <= 0) return v;
  if (T <= 1) return std::vector<int>(n, 1);
  const int R = last_single ? n - 1 : n;
  int k = (R + T - 1) / T;
  int total = k + (last_single ? 1 : 0);
  if (even && (total & 1)) {
    if (k + 1 > R) return std::vector<int>(n, 1);
    ++k;
  }
  for (int i = 0; i < k; ++i) v.push_back(R / k + (i < R % k ? 1 : 0));
  if (last_single) v.push_back(1);
  return v;
}

// A check window of n iterations on a blocked shape: launches of up to T
// iterations, the last one (the check variant) of up to F, spread evenly.
// The number of launches may be odd: the window then ends in the other
// copy of the state.
inline std::vector<int> fused_schedule(int n, int T, int F) {
  std::vector<int> v;
  if (n <= 0) return v;
  const int f = std::min(F, n);
  const int R = n - f;
  const int k = (R + T - 1) / T;
  for (int i = 0; i < k; ++i) v.push_back(R / k + (i < R % k ? 1 : 0));
  v.push_back(f);
  return v;
}


// The caller's cap on the persistent grids (uot_params.max_groups), rounded
// down to a multiple of the 8 XCDs, at least 8; no cap when 0.
inline long group_cap_of(int max_groups) { return max_groups > 0 ? std::max(8, max_groups / 8 * 8) : LONG_MAX; }

// Validation of the parameters (everything uot_create checks before any
// device work).
inline uot_status check_params(const uot_params* p) {
  if (!p) return UOT_ERR_ARG;
  if (p->mode < 0 || p->mode > 2) return UOT_ERR_ARG;
  if (p->balanced != 0 && p->balanced != 1) return UOT_ERR_ARG;
  if (!p->balanced && p->residual_p != 1 && p->residual_p != 2) return UOT_ERR_ARG;
  if (p->bc != 0 && p->bc != 1) return UOT_ERR_ARG;
  if (p->norm != UOT_NORM_ISO && p->norm != UOT_NORM_ANISO) return UOT_ERR_ARG;
  if (!p->balanced && !(p->mu > 0.0 && std::isfinite(p->mu))) return UOT_ERR_ARG;
  if (p->mode != UOT_DIST && !(p->rho > 0.0 && std::isfinite(p->rho))) return UOT_ERR_ARG;
  if (!(p->tau1 >= 0.0 && p->tau2 >= 0.0) || !std::isfinite(p->tau1) || !std::isfinite(p->tau2)) return UOT_ERR_ARG;
  if ((p->tau1 == 0.0) != (p->tau2 == 0.0)) return UOT_ERR_ARG;
  if (p->max_groups < 0) return UOT_ERR_ARG;
  if (p->max_iter < 0 || p->check_every < 0) return UOT_ERR_ARG;
  if (!std::isfinite(p->tol)) return UOT_ERR_ARG;
  switch (p->tile_rows) {
    case 0: case 4: case 8: case 16: case 32: case 116: case 132: case 316: case 332:
    case 4004: case 4008: case 2016: case 4016: case 8016: case 4032: case 8032: break;
    default: return UOT_ERR_ARG;
  }
  if ((p->flags & UOT_ALLOW_SIGNED) && p->mode != UOT_DIST) return UOT_ERR_ARG;
  if (p->nx < 0 || p->ny < 0) return UOT_ERR_SHAPE;
  if (p->pitch != 0 && p->pitch < p->nx) return UOT_ERR_SHAPE;
  if (p->nx > 0 && p->ny > 0 && p->tau1 > 0.0 && !(p->flags & UOT_UNSAFE_STEPS)) {
    const double k2 = knorm2_of(p->nx, p->ny, p->mode, p->balanced, p->bc);
    if (p->tau1 * p->tau2 * k2 >= 1.0) return UOT_ERR_STEP;
  }
  return UOT_OK;
}

// A batch layout: pair b spans [offset[b], offset[b] + pitch[b] (ny[b] - 1)
// + nx[b]) of the packed planes (pitch == nullptr: pitch = nx).  Every pair
// must be non-empty with pitch >= nx and offset >= 0, and no two spans may
// overlap.  *total receives the extent of the packed planes, *npx the pixels.
inline uot_status check_layout(int B, const int32_t* nx, const int32_t* ny, const int32_t* pitch,
                               const int64_t* offset, long* total, long* npx) {
  if (B < 1 || !nx || !ny || !offset) return UOT_ERR_ARG;
  std::vector<std::pair<int64_t, int64_t>> ranges(B);
  long tot = 0, n = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t pb = pitch ? pitch[b] : nx[b];
    if (nx[b] < 1 || ny[b] < 1 || offset[b] < 0 || pb < nx[b]) return UOT_ERR_SHAPE;
    const int64_t extent = pb * (ny[b] - 1) + nx[b];
    if (offset[b] > INT64_MAX - extent) return UOT_ERR_SHAPE;
    ranges[b] = {offset[b], offset[b] + extent};
    tot = std::max<long>(tot, offset[b] + extent);
    n += (long)nx[b] * ny[b];
  }
  std::sort(ranges.begin(), ranges.end());
  for (int b = 1; b < B; ++b)
    if (ranges[b].first < ranges[b - 1].second) return UOT_ERR_SHAPE;
  *total = tot;
  *npx = n;
  return UOT_OK;
}

}  // namespace planner
}  // namespace uot
