/* Host-side code of the library under AddressSanitizer (no GPU needed):
 * pat_plan_create builds every table (sensor taps and their row lists,
 * twiddles, shift factors, kappa, PML profiles) in host memory before its
 * first device allocation, which fails on a machine without a GPU; every
 * entry point checks its arguments before touching a device.  Exit status 0
 * when every call returned the expected status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/pat.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d, expected %d\n", what, got, want);
    ++failures;
  }
}

/* m sensors on a circle of radius r (metres) */
static double* circle(int m, double r) {
  double* xy = (double*)malloc(sizeof(double) * 2 * (size_t)m);
  for (int s = 0; s < m; ++s) {
    xy[2 * s] = r * cos(2.0 * M_PI * s / m);
    xy[2 * s + 1] = r * sin(2.0 * M_PI * s / m);
  }
  return xy;
}

static void plan_case(const char* what, int nx, int ny, int K, int m, double radius_px, int pml, int want) {
  pat_grid g = {nx, ny, 50, pml, 1e-4, 1.875e-8, 1600.0, 1000.0, 2.0};
  double* xy = circle(m, radius_px * 1e-4);
  pat_plan* p = NULL;
  int st = pat_plan_create(&g, K, m, xy, &p);
  expect(what, st, want);
  if (st == PAT_OK) pat_plan_destroy(p);
  free(xy);
}

/* deterministic generator for the sweep below (64-bit LCG, top 53 bits) */
static unsigned long long lcg_state = 0x2505084820250508ULL;
static double uniform(void) {
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}
static int pick(int n) { return (int)(uniform() * n) % n; }

/* Random plans over every supported axis length (square and not), dataset
 * count, PML width and sensor set, sensors anywhere their four bilinear taps
 * stay on the grid (fractional cell-centre index in [0, n - 1), kept 1e-6
 * cells from both ends so that rounding of the position cannot decide); every
 * fourth plan on a grid whose spacing is a power of two, where the position
 * arithmetic is exact, with one sensor on the first cell centre (index 0,
 * inside).  Then the same sets with one sensor 1e-6 cells beyond either end
 * of either axis's range. */
static void random_plans(int want_ok) {
  static const int len[] = {32, 36, 40, 48, 64, 81, 84, 96, 125, 128, 160, 175, 192, 243, 256, 375, 384, 512, 768};
  const int nlen = (int)(sizeof len / sizeof len[0]);
  char what[160];
  for (int t = 0; t < 48; ++t) {
    const int nx = len[t < nlen ? t : pick(nlen)], ny = t < nlen ? nx : len[pick(nlen)];
    const int K = 1 + pick(64), m = 1 + pick(2500);
    const int pml = pick((nx < ny ? nx : ny) / 2);
    const double dx = t % 4 == 0 ? 1.0 / 8192.0 : 1e-4;
    pat_grid g = {nx, ny, 20, pml, dx, 1.875e-8, 1600.0, 1000.0, 2.0};
    double* xy = (double*)malloc(sizeof(double) * 2 * (size_t)m);
    for (int s = 0; s < m; ++s) {
      /* fractional cell-centre index f in [0, n - 1): position (f + 0.5 - n/2) dx */
      const double fx = 1e-6 + uniform() * (nx - 1 - 2e-6), fy = 1e-6 + uniform() * (ny - 1 - 2e-6);
      xy[2 * s] = (fx + 0.5 - nx / 2.0) * dx;
      xy[2 * s + 1] = (fy + 0.5 - ny / 2.0) * dx;
    }
    if (t % 4 == 0) { xy[0] = (0.5 - nx / 2.0) * dx; xy[1] = (0.5 - ny / 2.0) * dx; }   /* first cell centre, exact */
    pat_plan* p = NULL;
    snprintf(what, sizeof what, "random plan %d: %dx%d K %d m %d pml %d", t, nx, ny, K, m, pml);
    const int st = pat_plan_create(&g, K, m, xy, &p);
    expect(what, st, want_ok);
    if (st == PAT_OK) pat_plan_destroy(p);
    /* one sensor just outside, 1e-6 cells before index 0 or beyond index n - 1, on either axis */
    const int s = pick(m), side = pick(4);
    const double out_f[4] = {-1e-6, nx - 1 + 1e-6, -1e-6, ny - 1 + 1e-6};
    if (side < 2) xy[2 * s] = (out_f[side] + 0.5 - nx / 2.0) * dx;
    else xy[2 * s + 1] = (out_f[side] + 0.5 - ny / 2.0) * dx;
    snprintf(what, sizeof what, "random plan %d, sensor %d outside (side %d)", t, s, side);
    p = NULL;
    expect(what, pat_plan_create(&g, K, m, xy, &p), PAT_EINVAL);
    free(xy);
  }
}

int main(void) {
  /* valid plans: on a machine without a GPU the table upload fails (PAT_EHIP)
   * after every host table has been built */
  const int want_ok = PAT_EHIP;
  plan_case("512 K8 512 sensors", 512, 512, 8, 512, 195.0, 20, want_ok);
  plan_case("128 K3 96 sensors", 128, 128, 3, 96, 49.0, 10, want_ok);
  plan_case("84 K1 64 sensors", 84, 84, 1, 64, 30.0, 10, want_ok);
  plan_case("375 K4 2000 sensors (many per pixel)", 375, 375, 4, 2000, 150.0, 20, want_ok);
  plan_case("96x64 non-square", 96, 64, 2, 20, 20.0, 8, want_ok);
  plan_case("243 odd", 243, 243, 64, 7, 90.0, 14, want_ok);
  plan_case("32 one sensor at the centre", 32, 32, 1, 1, 0.0, 4, want_ok);
  /* sensors on pixel centres and on pixel edges of a small grid */
  {
    pat_grid g = {40, 36, 10, 4, 1e-4, 1.875e-8, 1600.0, 1000.0, 2.0};
    double xy[8] = {0.5e-4, 0.5e-4, -1.5e-4, 2.5e-4, 0.0, 0.0, 1.7e-3, -1.6e-3};
    pat_plan* p = NULL;
    expect("pixel centres and edges", pat_plan_create(&g, 2, 4, xy, &p), want_ok);
  }
  random_plans(want_ok);
  /* invalid plans */
  plan_case("sensor outside the grid", 64, 64, 1, 8, 40.0, 8, PAT_EINVAL);
  plan_case("unsupported length", 100, 100, 1, 8, 20.0, 8, PAT_EUNSUPPORTED);
  plan_case("K > 64", 64, 64, 65, 8, 20.0, 8, PAT_EUNSUPPORTED);
  plan_case("PML covers the grid", 64, 64, 1, 8, 20.0, 32, PAT_EINVAL);
  plan_case("no sensors", 64, 64, 1, 0, 20.0, 8, PAT_EINVAL);
  {
    pat_grid g = {64, 64, 10, 8, 1e-4, 1.875e-8, 1600.0, 1000.0, 2.0};
    double nan_xy[2] = {NAN, 0.0};
    pat_plan* p = NULL;
    expect("NaN sensor", pat_plan_create(&g, 1, 1, nan_xy, &p), PAT_EINVAL);
    g.dt = -1.0;
    double xy[2] = {0.0, 0.0};
    expect("negative dt", pat_plan_create(&g, 1, 1, xy, &p), PAT_EINVAL);
    expect("null grid", pat_plan_create(NULL, 1, 1, xy, &p), PAT_EINVAL);
  }
  /* argument checks of the other entry points (nothing is enqueued) */
  float dummy[4];
  const float* ptrs[1] = {dummy};
  size_t bytes = 0;
  const float* field = NULL;
  double J = 0.0;
  expect("workspace_size null", pat_workspace_size(NULL, 0, &bytes), PAT_EINVAL);
  expect("forward null", pat_forward(NULL, dummy, dummy, dummy, dummy, 4, 0, 1, NULL), PAT_EINVAL);
  expect("history null", pat_history_field(NULL, dummy, 0, &field), PAT_EINVAL);
  expect("misfit null", pat_misfit(NULL, dummy, dummy, dummy, dummy, &J, NULL), PAT_EINVAL);
  expect("adjoint null", pat_adjoint_gradient(NULL, dummy, dummy, dummy, dummy, dummy, dummy, 4, NULL), PAT_EINVAL);
  expect("project n<0", pat_project_update(-1, dummy, dummy, 1.0f, NULL, NULL, 0.0f, 1.0f, NULL), PAT_EINVAL);
  expect("prolong nchan 0", pat_prolong(0, dummy, 2, 2, dummy, 4, 4, NULL), PAT_EINVAL);
  expect("prolong_phys dx 0", pat_prolong_phys(1, dummy, 2, 2, 0.0, dummy, 4, 4, 1e-4, NULL), PAT_EINVAL);
  expect("time_interp nt 0", pat_time_interp(1, 0, 1, dummy, 1.0, dummy, 1, 1.0, NULL), PAT_EINVAL);
  expect("lbfgs null pair", pat_lbfgs_direction(4, dummy, 1, NULL, ptrs, dummy, dummy, NULL), PAT_EINVAL);
  expect("lbfgs noalloc too many pairs",
         pat_lbfgs_direction_noalloc(4, dummy, PAT_LBFGS_NOALLOC_MAX_PAIRS + 1, NULL, NULL, dummy, NULL), PAT_EINVAL);
  expect("dot n 0", pat_dot(0, dummy, dummy, &J, dummy, NULL), PAT_EINVAL);
  expect("set_tile null", pat_plan_set_tile(NULL, 0), PAT_EINVAL);
  expect("batch empty", pat_batch_gradient(0, NULL, 1, NULL), PAT_EINVAL);
  expect("ou_create empty", pat_ou_create(0, 0, 1e-4, 1e-3, NULL, NULL), PAT_EINVAL);
  if (pat_status_string(PAT_ENONFINITE) == NULL) ++failures;
  printf("host checks: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
