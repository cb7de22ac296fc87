// Host-only check of the solver's planner (paper_1909_00149_amd/csrc/
// uot_plan.hpp), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_host_sanitize.py: parameter validation on valid, invalid and
// fuzzed parameters, the step-size bound of Theorem 1 against a power
// iteration on the explicit D D*, the launch schedules of check windows and
// the validation of batch layouts.  Prints "ok" and exits 0 when every check
// holds; any failure prints its case and exits 1 (a sanitizer report aborts).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "uot_plan.hpp"

using namespace uot::planner;

static int g_fail = 0;
#define EXPECT(cond, ...)                        \
  do {                                           \
    if (!(cond)) {                               \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                  \
      std::printf("\n");                         \
      ++g_fail;                                  \
    }                                            \
  } while (0)

static uot_params base_params() {
  uot_params p{};
  p.nx = 64;
  p.ny = 48;
  p.mode = UOT_DIST;
  p.residual_p = 1;
  p.mu = 1.0;
  p.rho = 1.0;
  p.max_iter = 100;
  p.check_every = 20;
  return p;
}

// lambda_max(D D*) of an nx x ny grid by power iteration on the explicit
// operator: D M = Mx - Mx(left) + My - My(below), D* a = (a - a(right),
// a - a(above)), the right column / top row flux structurally zero when
// bc = 0 and free when bc = 1.
static double lam_power(int nx, int ny, int bc) {
  const int n = nx * ny;
  std::vector<double> a(n), mx(n), my(n), b(n);
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> u(-1, 1);
  for (auto& v : a) v = u(rng);
  double lam = 0;
  for (int it = 0; it < 4000; ++it) {
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int k = j * nx + i;
        const double ar = i + 1 < nx ? a[k + 1] : 0.0, au = j + 1 < ny ? a[k + nx] : 0.0;
        mx[k] = (bc == 0 && i == nx - 1) ? 0.0 : a[k] - ar;
        my[k] = (bc == 0 && j == ny - 1) ? 0.0 : a[k] - au;
      }
    double nrm = 0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int k = j * nx + i;
        b[k] = mx[k] - (i > 0 ? mx[k - 1] : 0.0) + my[k] - (j > 0 ? my[k - nx] : 0.0);
        nrm += b[k] * b[k];
      }
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return 0.0;  // the 1 x 1 grid: D D* = 0
    double dot = 0;
    for (int k = 0; k < n; ++k) dot += a[k] * b[k];
    lam = dot;
    for (int k = 0; k < n; ++k) a[k] = b[k] / nrm;
  }
  return lam;
}

int main() {
  // ---- parameters ----
  {
    uot_params p = base_params();
    EXPECT(check_params(&p) == UOT_OK, "base");
    EXPECT(check_params(nullptr) == UOT_ERR_ARG, "null");
    p.mode = 3;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "mode");
    p = base_params();
    p.mu = -1;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "mu");
    p = base_params();
    p.tau1 = 0.6;
    p.tau2 = 0.6;
    EXPECT(check_params(&p) == UOT_ERR_STEP, "steps over the bound");
    p.flags = UOT_UNSAFE_STEPS;
    EXPECT(check_params(&p) == UOT_OK, "unsafe steps");
    p = base_params();
    p.tau1 = 0.1;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "one step given");
    p = base_params();
    p.tile_rows = 17;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "tile rows");
    p = base_params();
    p.pitch = 10;
    EXPECT(check_params(&p) == UOT_ERR_SHAPE, "pitch < nx");
    p = base_params();
    p.max_groups = -8;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "max_groups");
    p = base_params();
    p.tol = NAN;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "tol");
    p = base_params();
    p.mode = UOT_PROX;
    p.flags = UOT_ALLOW_SIGNED;
    EXPECT(check_params(&p) == UOT_ERR_ARG, "signed prox");
    // fuzz: any combination of values must be classified without undefined
    // behaviour, twice alike
    std::mt19937_64 rng(1);
    const double dv[] = {0.0, -0.0, 1.0, -1.0, 1e-300, 1e300, INFINITY, -INFINITY, NAN, 0.35, 2.0};
    const int iv[] = {0, 1, 2, 3, -1, 4, 8, 16, 116, 4016, 8032, 1 << 30, -(1 << 30), INT32_MAX, INT32_MIN};
    for (int it = 0; it < 200000; ++it) {
      uot_params q{};
      auto I = [&]() { return iv[rng() % (sizeof(iv) / sizeof(iv[0]))]; };
      auto D = [&]() { return dv[rng() % (sizeof(dv) / sizeof(dv[0]))]; };
      q.nx = I(); q.ny = I(); q.mode = I(); q.balanced = I(); q.residual_p = I(); q.bc = I();
      q.mu = D(); q.rho = D(); q.tau1 = D(); q.tau2 = D(); q.max_iter = I(); q.check_every = I();
      q.tol = D(); q.flags = (uint32_t)rng(); q.tile_rows = I(); q.pitch = I(); q.norm = I(); q.max_groups = I();
      const uot_status a = check_params(&q), b = check_params(&q);
      EXPECT(a == b, "deterministic");
      EXPECT(a >= UOT_OK && a <= UOT_ERR_STEP, "status range %d", (int)a);
    }
  }
  // ---- Theorem 1's bound: closed-form lambda_max against the operator ----
  for (int bc = 0; bc < 2; ++bc)
    for (int nx : {1, 2, 3, 5, 8})
      for (int ny : {1, 2, 4, 7}) {
        const double lam = knorm2_of(nx, ny, UOT_DIST, 1, bc);  // balanced DIST: no identity block
        const double ref = lam_power(nx, ny, bc);
        EXPECT(std::fabs(lam - ref) <= 1e-9 * std::max(1.0, ref), "lambda_max %dx%d bc %d: %.12f vs %.12f", nx, ny,
               bc, lam, ref);
      }
  EXPECT(knorm2_of(0, 4, 0, 0, 0) < 0 && knorm2_of(4, 4, 5, 0, 0) < 0, "bad knorm2 arguments");
  {
    double t1, t2;
    for (double s : {1e-9, 1e-4, 1.0, 1e6}) {
      default_steps(7.9, s, &t1, &t2);
      EXPECT(std::fabs(t1 * t2 * 7.9 - 0.9801) < 1e-12, "default steps product at scale %g", s);
      EXPECT(std::fabs(t1 / t2 - s * s) <= 1e-12 * s * s, "default steps ratio at scale %g", s);
    }
  }
  // ---- schedules ----
  for (int T : {1, 2, 4, 8})
    for (int n = 0; n <= 130; ++n)
      for (int ls = 0; ls < 2; ++ls)
        for (int ev = 0; ev < 2; ++ev) {
          const std::vector<int> v = step_schedule(n, T, ls, ev);
          long sum = 0;
          bool inb = true;
          for (int x : v) {
            sum += x;
            inb = inb && x >= 1 && x <= T;
          }
          EXPECT(sum == n && inb, "step_schedule(%d, %d, %d, %d) covers n within T", n, T, ls, ev);
          if (n > 0 && ls) EXPECT(v.back() == 1, "last single (%d, %d)", n, T);
          if (n > 0 && ev && n % 2 == 0) EXPECT(v.size() % 2 == 0, "even launches (%d, %d, %d)", n, T, ls);
        }
  for (int T : {2, 4, 8})
    for (int F : {1, 2, 4})
      for (int n = 0; n <= 130; ++n) {
        const std::vector<int> v = fused_schedule(n, T, F);
        long sum = 0;
        bool inb = true;
        for (size_t i = 0; i < v.size(); ++i) {
          sum += v[i];
          inb = inb && v[i] >= 1 && v[i] <= (i + 1 == v.size() ? F : T);
        }
        EXPECT(sum == n && inb, "fused_schedule(%d, %d, %d)", n, T, F);
      }
  for (int code : {4, 8, 16, 32, 116, 132, 316, 332, 4004, 4008, 2016, 4016, 8016, 4032, 8032}) {
    EXPECT(shape_known(code), "known %d", code);
    EXPECT(shape_steps(code) >= 1 && shape_rows(code) % 4 == 0, "shape %d", code);
    EXPECT(shape_steps(shape_single(code)) == 1 && shape_rows(shape_single(code)) == shape_rows(code), "single %d", code);
    EXPECT(shape_chk_steps(code) <= shape_steps(code) || shape_steps(code) == 1, "check steps %d", code);
  }
  EXPECT(group_cap_of(0) == LONG_MAX && group_cap_of(1) == 8 && group_cap_of(17) == 16, "group cap");
  // 32-bit byte offsets of a blocked kernel's region: (region rows + 1)
  // rows of the widest pitch allowed, for the plain and the check variant
  for (int code : {4004, 4008, 2016, 4016, 8016, 4032, 8032}) {
    const long H = std::max(shape_steps(code), shape_chk_steps(code) + 1);
    const long rows = shape_rows(code) + 2 * H + 1;
    EXPECT((rows * kBlockedMaxPitch + 64 + 2 * H) * 4 < (1L << 32), "region offsets of %d", code);
  }
  {
    const int32_t w[2] = {300, (int32_t)kBlockedMaxPitch}, w2[2] = {300, (int32_t)kBlockedMaxPitch + 1};
    EXPECT(blocked_pitch_ok(2, w, nullptr) && !blocked_pitch_ok(2, w2, nullptr) && blocked_pitch_ok(2, w2, w),
           "blocked pitch");
  }
  // ---- batch layouts ----
  {
    std::mt19937 rng(3);
    for (int it = 0; it < 20000; ++it) {
      const int B = 1 + (int)(rng() % 40);
      std::vector<int32_t> nx(B), ny(B), pitch(B);
      std::vector<int64_t> off(B);
      int64_t o = (int64_t)(rng() % 5);
      for (int b = 0; b < B; ++b) {
        nx[b] = 1 + (int)(rng() % 300);
        ny[b] = 1 + (int)(rng() % 300);
        pitch[b] = nx[b] + (int)(rng() % 70);
        off[b] = o;
        o += (int64_t)pitch[b] * (ny[b] - 1) + nx[b] + (int64_t)(rng() % 3);
      }
      const bool overlap = B > 1 && rng() % 4 == 0;
      if (overlap) {
        const int b = 1 + (int)(rng() % (B - 1));
        off[b] -= 1 + (int64_t)(rng() % nx[b - 1]);
      }
      const bool bad = rng() % 8 == 0;
      if (bad) nx[rng() % B] = -(int)(rng() % 3);
      long total = -1, npx = -1;
      const uot_status s = check_layout(B, nx.data(), ny.data(), pitch.data(), off.data(), &total, &npx);
      if (bad) {
        EXPECT(s == UOT_ERR_SHAPE, "non-positive width rejected");
      } else {
        bool any = false;  // a negative offset, or a span overlapping its predecessor's
        long want_px = 0, want_total = 0;
        for (int b = 0; b < B; ++b) {
          const int64_t end = off[b] + (int64_t)pitch[b] * (ny[b] - 1) + nx[b];
          any = any || off[b] < 0;
          if (b > 0) any = any || off[b] < off[b - 1] + (int64_t)pitch[b - 1] * (ny[b - 1] - 1) + nx[b - 1];
          want_px += (long)nx[b] * ny[b];
          want_total = std::max<long>(want_total, end);
        }
        EXPECT((s == UOT_ERR_SHAPE) == any, "overlap detected iff present (B %d)", B);
        if (!any) EXPECT(s == UOT_OK && npx == want_px && total == want_total, "layout sizes (B %d)", B);
      }
    }
    int32_t one = 4;
    int64_t neg = -3, huge = INT64_MAX - 2;
    long t, n;
    EXPECT(check_layout(1, &one, &one, nullptr, &neg, &t, &n) == UOT_ERR_SHAPE, "negative offset");
    EXPECT(check_layout(1, &one, &one, nullptr, &huge, &t, &n) == UOT_ERR_SHAPE, "offset overflow");
    EXPECT(check_layout(0, &one, &one, nullptr, &neg, &t, &n) == UOT_ERR_ARG, "empty batch");
  }
  if (g_fail) {
    std::printf("%d failures\n", g_fail);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
