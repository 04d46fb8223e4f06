/* Driver that runs every entry point of the oracle (oracle/ggdt_ref.c) on small
 * 2D and 3D inputs, including degenerate shapes (size-1 axes), several channel
 * counts, lambda values, records, the reverse pass, the checkers and the
 * incremental re-evaluation.  Built by the test with AddressSanitizer and
 * UndefinedBehaviorSanitizer (no recovery), so any out-of-bounds access, leak,
 * use after free or undefined operation ends the run with a report.  It checks
 * no values: the pinning tests do that. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ref_ggdt_f32(int, const int*, int, const float*, const float*, const float*, float, float, int, float*,
                 uint8_t*);
int ref_ggdt_f32_omp(int, const int*, int, const float*, const float*, const float*, float, float, int, float*);
int ref_ggdt_f64(int, const int*, int, const double*, const double*, const double*, double, double, int, double*,
                 uint8_t*);
int ref_pass_f32(int, const int*, int, const float*, const float*, float, int, int, float*, uint8_t*);
int ref_pass_f64(int, const int*, int, const double*, const double*, double, int, int, double*, uint8_t*);
int ref_toivanen_f32(int, const int*, int, const float*, const float*, const float*, float, float, int, int, float*);
int ref_toivanen_f64(int, const int*, int, const double*, const double*, const double*, double, double, int, int,
                     double*);
int ref_ggdt_until_converged_f32(int, const int*, int, const float*, const float*, const float*, float, float, int,
                                 float*);
int ref_ggdt_until_converged_f64(int, const int*, int, const double*, const double*, const double*, double, double,
                                 int, double*);
int ref_dijkstra_f32(int, const int*, int, const float*, const float*, const float*, float, float, float*);
int ref_dijkstra_f64(int, const int*, int, const double*, const double*, const double*, double, double, double*);
int ref_chamfer_closed_form_f64(int, const int*, const double*, const double*, double, double*);
int ref_bruteforce_paths_f64(int, const int*, int, const double*, const double*, const double*, double, double, int,
                             long, double*);
int ref_pass_bruteforce_f64(int, const int*, int, const double*, const double*, double, int, int, const double*,
                            double*);
int ref_ggdt_backward_f32(int, const int*, int, const float*, const float*, float, float, int, const uint8_t*,
                          const float*, float*, float*);
int ref_ggdt_backward_f64(int, const int*, int, const double*, const double*, double, double, int, const uint8_t*,
                          const double*, double*, double*);
int ref_ggdt_f64_trajectory(int, const int*, int, const double*, const double*, const double*, double, double, int,
                            double*, uint8_t*);
int ref_ggdt_f64_perturbed(int, const int*, int, const double*, const double*, const double*, double, double, int,
                           const double*, const uint8_t*, int, int, long, double, double*, int*);

static int failures = 0;

static void expect_ok(int rc, const char* what) {
  if (rc < 0) {
    printf("FAILED %s: status %d\n", what, rc);
    ++failures;
  }
}

/* The run-to-convergence entries return -1 when their cap is reached. */
static void expect_ok_or_cap(int rc, const char* what) {
  if (rc < -1) {
    printf("FAILED %s: status %d\n", what, rc);
    ++failures;
  }
}

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

static void run_case(int ndim, const int* dims, int C, double lam, int iters, unsigned seed) {
  long n = 1;
  for (int i = 0; i < ndim; ++i) n *= dims[i];
  const int npass = iters * 2 * ndim;
  float* img32 = malloc(sizeof(float) * n * C);
  double* img64 = malloc(sizeof(double) * n * C);
  float* m32 = malloc(sizeof(float) * n);
  double* m64 = malloc(sizeof(double) * n);
  float* o32 = malloc(sizeof(float) * n);
  double* o64 = malloc(sizeof(double) * n);
  float* g32 = malloc(sizeof(float) * n);
  double* g64 = malloc(sizeof(double) * n);
  float* gi32 = malloc(sizeof(float) * n * C);
  double* gi64 = malloc(sizeof(double) * n * C);
  double* o64b = malloc(sizeof(double) * n);
  uint8_t* rec = malloc((size_t)(npass > 0 ? npass : 1) * n);
  double* traj = malloc(sizeof(double) * (npass + 1) * n);
  float sp32[3];
  double sp64[3];
  for (int b = 0; b < 3; ++b) {
    sp32[b] = (float)(0.5 + 2.0 * urand(&seed));
    sp64[b] = sp32[b];
  }
  for (long i = 0; i < n * C; ++i) {
    img32[i] = (float)urand(&seed);
    img64[i] = img32[i];
  }
  for (long i = 0; i < n; ++i) {
    m32[i] = urand(&seed) < 0.1 ? 0.0f : (float)urand(&seed);
    m64[i] = m32[i];
    g32[i] = (float)(urand(&seed) - 0.5);
    g64[i] = g32[i];
  }
  const float v32 = 10.0f;
  const float lam32 = (float)lam;
  expect_ok(ref_ggdt_f32(ndim, dims, C, img32, m32, sp32, v32, lam32, iters, o32, rec), "ggdt_f32");
  expect_ok(ref_ggdt_backward_f32(ndim, dims, C, img32, sp32, v32, lam32, iters, rec, g32, gi32, o32),
            "backward_f32");
  expect_ok(ref_ggdt_f32_omp(ndim, dims, C, img32, m32, sp32, v32, lam32, iters, o32), "ggdt_f32_omp");
  expect_ok(ref_ggdt_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, iters, o64, rec), "ggdt_f64");
  expect_ok(ref_ggdt_backward_f64(ndim, dims, C, img64, sp64, 10.0, lam32, iters, rec, g64, gi64, o64b),
            "backward_f64");
  expect_ok(ref_ggdt_f64_trajectory(ndim, dims, C, img64, m64, sp64, 10.0, lam32, iters, traj, rec), "trajectory");
  int same = 0;
  expect_ok(ref_ggdt_f64_perturbed(ndim, dims, C, img64, m64, sp64, 10.0, lam32, iters, traj, rec, 0, 0, n / 2,
                                   1e-3, o64b, &same), "perturbed M");
  expect_ok(ref_ggdt_f64_perturbed(ndim, dims, C, img64, m64, sp64, 10.0, lam32, iters, traj, rec, 1, C - 1, n - 1,
                                   0.4, o64b, &same), "perturbed I");
  for (int a = 0; a < ndim; ++a)
    for (int s = -1; s <= 1; s += 2) {
      expect_ok(ref_pass_f32(ndim, dims, C, img32, sp32, lam32, a, s, o32, rec), "pass_f32");
      expect_ok(ref_pass_f64(ndim, dims, C, img64, sp64, lam32, a, s, o64, rec), "pass_f64");
      if (n <= 30) expect_ok(ref_pass_bruteforce_f64(ndim, dims, C, img64, sp64, lam32, a, s, o64, o64b), "chain");
    }
  expect_ok_or_cap(ref_toivanen_f32(ndim, dims, C, img32, m32, sp32, v32, lam32, 50, 1, o32), "toivanen_f32");
  expect_ok(ref_toivanen_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, iters, 0, o64), "toivanen_f64");
  expect_ok_or_cap(ref_ggdt_until_converged_f32(ndim, dims, C, img32, m32, sp32, v32, lam32, 50, o32), "converge_f32");
  expect_ok_or_cap(ref_ggdt_until_converged_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, 50, o64), "converge_f64");
  expect_ok(ref_dijkstra_f32(ndim, dims, C, img32, m32, sp32, v32, lam32, o32), "dijkstra_f32");
  expect_ok(ref_dijkstra_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, o64), "dijkstra_f64");
  expect_ok(ref_chamfer_closed_form_f64(ndim, dims, m64, sp64, 10.0, o64), "closed_form");
  if (n <= 9) expect_ok(ref_bruteforce_paths_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, 0, 50000000L, o64),
                         "paths");
  if (n <= 30) expect_ok(ref_bruteforce_paths_f64(ndim, dims, C, img64, m64, sp64, 10.0, lam32, 1, 50000000L, o64),
                         "pruned walks");
  free(img32); free(img64); free(m32); free(m64); free(o32); free(o64); free(g32); free(g64);
  free(gi32); free(gi64); free(o64b); free(rec); free(traj);
}

int main(void) {
  const int shapes[][4] = {{2, 7, 9, 0}, {2, 1, 12, 0}, {2, 13, 1, 0}, {2, 3, 4, 0}, {3, 5, 6, 7},
                           {3, 1, 6, 5}, {3, 4, 1, 9}, {3, 6, 5, 1}, {3, 2, 2, 3}, {3, 3, 3, 3}, {3, 11, 9, 10}};
  const double lams[] = {0.0, 0.35, 1.0};
  unsigned seed = 12345u;
  int cases = 0;
  for (unsigned k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
    const int ndim = shapes[k][0];
    int dims[3] = {shapes[k][1], shapes[k][2], ndim == 3 ? shapes[k][3] : 1};
    for (int C = 1; C <= 3; ++C)
      for (unsigned l = 0; l < 3; ++l) {
        run_case(ndim, dims, C, lams[l], 1 + (int)((k + C + l) % 3), seed + 7u * (unsigned)cases);
        ++cases;
      }
  }
  printf("oracle sanitizer run: %d cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
