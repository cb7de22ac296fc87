// Internal declarations shared by the host runtime and the HIP kernels of
// the unbalanced Beckmann OT prox solver (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace uot {

constexpr int TX = 64;        // tile width: one 64-lane wavefront per row
constexpr int BLOCK = 256;    // threads per workgroup (4 wavefronts)
constexpr int NS = 16;        // per-tile partial-sum slots

// Residual variants of the iteration.
enum Resid { R_BAL = 0, R_P1 = 1, R_P2 = 2 };

// Partial-sum slots written by the check kernel (per tile, then per pair).
enum CheckSlot {
  S_PRES2 = 0,  // sum (K z)^2
  S_STAT2 = 1,  // sum of squared stationarity residual
  S_KA2 = 2,    // sum ||K* a||^2 terms
  S_X0SQ = 3,   // sum x0^2 (iterate)
  S_X1SQ = 4,   // sum x1^2 (iterate)
  S_MNORM = 5,  // sum ||M_i||_2
  S_RPEN = 6,   // sum |r| (p=1) or r^2 (p=2)
  S_EPEN = 7,   // sum |e| or e^2, e = D M - x0 + x1
  S_LIN = 8,    // DIST: sum a c;  PROX_FIXED: -sum a s
  S_QUAD = 9,   // sum (x - p)^2 over the free arguments
  S_MAXG = 10,  // max ||(D* a)_i||_2   (max-reduced)
  S_MAXA = 11,  // max |a_i|            (max-reduced)
  S_NONFIN = 12,// count of non-finite state entries
  S_A2 = 13,    // sum a^2
  S_SUMA = 14,  // sum a
};

// Partial-sum slots written by the setup kernel.
enum SetupSlot {
  U_NONFIN_IN = 0, U_NEG = 1, U_NONFIN_ST = 2, U_SUMS = 3, U_SUMD = 4, U_SQS = 5, U_SQD = 6,
  U_MAXIN = 7,  // max |pixel| over src and dst (max-reduced): the image scale of the default steps
};

inline constexpr uint32_t kMaxSlotsSetup = 1u << U_MAXIN;

inline constexpr uint32_t kMaxSlotsCheck = (1u << S_MAXG) | (1u << S_MAXA);

struct PairInfo {
  int64_t off;         // first pixel of the pair in the packed planes
  int32_t nx, ny;      // pixel (x, y) is element off + y * pitch + x
  float tau1, tau2;
  float theta;         // tau1 / (rho + tau1)
  float mutau;         // mu * tau1
  float inv2mt;        // 1 / (1 + 2 mu tau1)
  int32_t tile_begin;  // first tile of the pair in the full tile list
  int32_t tile_count;
  int32_t pitch;       // row stride in elements (>= nx)
};

struct Tile {
  int32_t pair, x0, y0, pad;  // pad: the tile's index in the full tile list
};

struct Planes {
  float *Mx, *My, *r, *a, *x0, *x1;
};

struct IterArgs {
  Planes in, out;
  const float* c;     // DIST: q - p
  const float* src;   // PROX: p0;  PROX_FIXED: s
  const float* dst;   // PROX: p1;  PROX_FIXED: p
  const PairInfo* pairs;
  const Tile* tiles;
  const int32_t* ntiles;
  const int32_t* active;
  int32_t steps;      // iterations per launch of the temporally blocked kernel
  int32_t pad_;
  double* chk;        // blocked kernel, one step: also the check's per-tile partial rows,
                      // at row Tile::pad (the tile's index in the full list)
};

struct CheckArgs {
  Planes A, B;        // ping-pong copies; current = A unless swap for the pair
  int swap_active;    // 1: pairs still active hold their current iterate in B
  int all_pairs;      // 1: evaluate inactive pairs too
  const float* c;
  const float* src;
  const float* dst;
  const PairInfo* pairs;
  const Tile* tiles;
  int32_t ntiles;
  int32_t tile_rows;
  const int32_t* active;
  double* partial;    // [ntiles][NS]
};

struct SetupArgs {
  const float* src;
  const float* dst;
  float* c;           // DIST only
  Planes st;
  int mode, resid, bc;
  int warm;           // 1: keep the caller's state (only its structural zeros are written)
  int write_state;    // 0: the state is only read
  int write_c;        // DIST: write c = q - p into the workspace
  const PairInfo* pairs;
  const Tile* tiles;
  int32_t ntiles;
  int32_t tile_rows;
  double* partial;
};

struct DecideArgs {
  PairInfo* pairs;      // steps are rewritten when adaptive
  double* sums;         // [B][NS], written by the fused reduction
  const double* xnorm;  // DIST: ||p|| + ||q|| per pair; other modes: unused
  int32_t* active;
  int32_t* iters;
  int32_t* status;
  double* rel_res;
  int32_t B;
  int32_t W;          // iterations since the last decision
  int32_t max_iter;
  int32_t check;      // 1: apply the stopping rule
  int32_t final_pass; // 1: decide every still-active pair (MAX_ITER if not converged)
  int32_t mode;
  int32_t nid;        // identity blocks in K
  double tol;
  int32_t adaptive;   // residual balancing of tau1/tau2
  double* alpha;      // per-pair adaptation factor
  double mu, rho;
  int32_t keep_rel;   // final pass right after a check: keep that check's rel_res
  int32_t pad_;
};

struct DualArgs {
  const float* a;
  const float* x_src;
  const float* x_dst;
  const float* inv_s;  // per pair
  const PairInfo* pairs;
  const Tile* tiles;
  int32_t ntiles, tile_rows, mode, resid;
  float rho, mu;
  double* partial;
};

// Douglas-Rachford splitting (uot_dr.hip): planes of w (iterate), z (the
// prox of w, the caller's state) and u = 2 z - w; one contiguous grid.
struct DrArgs {
  Planes w, z, u;
  const float *src, *dst;  // p0/p (x0's centre, DIST source), p1/q
  int32_t nx, ny, mode, resid, aniso;
  float gamma, mu, rho;
};
constexpr int DR_MAX_BLOCKS = 1024;  // blocks of the DR kernels (partials per block: 3 at most)
int dr_blocks(long n);
hipError_t launch_dr_prox_rhs(const DrArgs& a, float* out, hipStream_t s);  // z, u and e = K u - b
hipError_t launch_dr_rhs(const DrArgs& a, int of_z, float* out, double* partial, hipStream_t s);
hipError_t launch_dr_update(const DrArgs& a, const float* phi, int record, double* partial, hipStream_t s);
hipError_t launch_dr_objective(const DrArgs& a, double* partial, hipStream_t s);

// Per-mode instantiations (uot_iter_mode.hip compiled with UOT_MODE = 0, 1, 2).
hipError_t launch_iter_mode0(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_iter_mode1(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_iter_mode2(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t iter_occupancy_mode0(int resid, int bcn, int ty, int* n);
hipError_t iter_occupancy_mode1(int resid, int bcn, int ty, int* n);
hipError_t iter_occupancy_mode2(int resid, int bcn, int ty, int* n);
hipError_t iter_chk_occupancy_mode0(int resid, int bcn, int ty, int* n);
hipError_t iter_chk_occupancy_mode1(int resid, int bcn, int ty, int* n);
hipError_t iter_chk_occupancy_mode2(int resid, int bcn, int ty, int* n);
hipError_t launch_iter_chk_mode0(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_iter_chk_mode1(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_iter_chk_mode2(int resid, int bcn, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_check_mode0(int resid, int bcn, int grid, const CheckArgs& a, hipStream_t s);
hipError_t launch_check_mode1(int resid, int bcn, int grid, const CheckArgs& a, hipStream_t s);
hipError_t launch_check_mode2(int resid, int bcn, int grid, const CheckArgs& a, hipStream_t s);

hipError_t launch_iter(int mode, int resid, int bc, int ty, int grid, const IterArgs& a,
                       hipStream_t s);
hipError_t launch_check(int mode, int resid, int bc, int grid, const CheckArgs& a, hipStream_t s);
// One step of a blocked shape that also writes the check's partial rows for
// the iterate pair (in, out) into a.chk (the separate check kernel's rows).
hipError_t launch_iter_chk(int mode, int resid, int bc, int ty, int grid, const IterArgs& a, hipStream_t s);
hipError_t launch_setup(int grid, const SetupArgs& a, hipStream_t s);
hipError_t launch_pair_reduce(const PairInfo* pairs, int B, const double* partial, uint32_t max_mask,
                              double* sums, hipStream_t s);
// per-pair reduction of check partials fused with the stopping decision
hipError_t launch_reduce_decide(const DecideArgs& a, const double* partial, hipStream_t s);
hipError_t launch_copy_active(const Planes& dst, const Planes& src, const PairInfo* pairs,
                              const Tile* tiles, int ntiles, int tile_rows, const int32_t* active,
                              int grid, hipStream_t s);
hipError_t launch_dual(int grid, const DualArgs& a, hipStream_t s);
hipError_t launch_zero_pairs(const Planes& st, const PairInfo* pairs, const Tile* tiles, int ntiles, int tile_rows,
                             const int32_t* mask, int grid, hipStream_t s);
hipError_t iter_occupancy(int mode, int resid, int bc, int ty, int* blocks_per_cu);
// the same for the one-step check variant of a blocked shape
hipError_t iter_chk_occupancy(int mode, int resid, int bc, int ty, int* blocks_per_cu);

}  // namespace uot

namespace uot {
// Neumann-Poisson solve via the orthonormal DCT-II matrices Cx (nx x nx),
// Cy (ny x ny); t1, t2 are nx*ny scratch planes.
hipError_t poisson_solve(const float* Cx, const float* Cy, int nx, int ny, float alpha, const float* rhs,
                         float* phi, float* t1, float* t2, hipStream_t s);
hipError_t launch_sgemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                        float* C, int ldc, hipStream_t s);
// In the three helpers below the state and image planes have row stride
// pitch (>= nx); phi and e are contiguous nx*ny planes.
hipError_t launch_poisson_start(const float* phi, const float* src, const float* dst, const Planes& st, int nx,
                                int ny, int pitch, int mode, int balanced, hipStream_t s);
// Mx = My = nullptr: the zero flux.
hipError_t launch_infeasibility(const float* Mx, const float* My, const float* src, const float* dst, float* e,
                                int nx, int ny, int pitch, hipStream_t s);
int repaired_norm_blocks(int nx, int ny);
hipError_t launch_repaired_norm(const float* Mx, const float* My, const float* phi, int nx, int ny, int pitch,
                                int aniso, double* partial, hipStream_t s);
}  // namespace uot
