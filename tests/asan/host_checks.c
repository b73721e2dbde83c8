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
