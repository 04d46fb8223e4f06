/*
 * ORACLE — test infrastructure only.  Nothing on the product path may link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * Plain, slow, single-threaded CPU reference of the generalised geodesic
 * distance transform (GGDT) computed by directional raster-scan passes, as the
 * FastGeodis paper describes it (section "Implementation": passes that update
 * a whole row (2D) or plane (3D) in parallel from the previous row/plane; four
 * passes in 2D, six in 3D).  The paper prints no formula; the one followed here
 * is the generalised GDT of Criminisi et al. 2008 that the paper implements
 * (section "Statement of need"):
 *
 *     D0(x) = v * M(x)
 *     w(x,y) = sqrt((1 - lambda) * |x - y|_s^2 + lambda * sum_c (I_c(x) - I_c(y))^2)
 *     one pass: D(x) <- min(D(x), min over y in the previous row/plane of D(y) + w(x,y))
 *
 * Readings of points the paper leaves open:
 *  - only the 3 (2D) / 9 (3D) neighbours in the previous row/plane are used;
 *    the current value D(x) takes part in the min ("keep");
 *  - passes per iteration: for axis 0..ndim-1: ascending, then descending;
 *  - neighbours outside the grid are skipped; the first row/plane of a pass is
 *    left unchanged;
 *  - spacing is given in array-axis order;
 *  - the channel term is the plain sum of squared differences, channel order 0..C-1;
 *  - ties keep the earlier candidate (strict <), candidates in lexicographic
 *    order of the offset over the non-scan axes (ascending axis), each -1, 0, +1.
 *
 * FP32 operation sequence (one rounding per line):
 *     d_c  = I_c(x) - I_c(y)
 *     g    = d_0 * d_0;  g = fmaf(d_c, d_c, g) for c = 1..C-1
 *     q    = fmaf(lambda, g, A)      A = (float)((1 - (double)lambda) * S),
 *                                    S = sum over axes b ascending of (s_b * |dx_b|)^2 in double
 *     w    = sqrtf(q)
 *     cand = D(y) + w
 * The FP64 variant is the same sequence in double with A = (1 - lambda) * S unrounded.
 *
 * Besides the schedule this file holds independent checkers used to pin it:
 * multi-source Dijkstra, the lambda = 0 closed form, exhaustive and
 * bound-pruned path enumeration, a per-pass chain brute force and the exact
 * reverse-mode gradient of the schedule.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define REF_OK 0
#define REF_EINVAL -1
#define REF_ENOMEM -2

/* ------------------------------------------------------------------ grid */

typedef struct {
  int ndim;
  int dims[3];
  long strides[3];
  long n;
} grid_t;

static int grid_init(grid_t* g, int ndim, const int* dims) {
  if (ndim != 2 && ndim != 3) return REF_EINVAL;
  g->ndim = ndim;
  long n = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1) return REF_EINVAL;
    g->dims[i] = dims[i];
    n *= dims[i];
  }
  long s = 1;
  for (int i = ndim - 1; i >= 0; --i) {
    g->strides[i] = s;
    s *= dims[i];
  }
  g->n = n;
  return REF_OK;
}

static void unflatten(const grid_t* g, long idx, int* c) {
  for (int i = 0; i < g->ndim; ++i) {
    c[i] = (int)(idx / g->strides[i]);
    idx -= (long)c[i] * g->strides[i];
  }
}

static long flatten(const grid_t* g, const int* c) {
  long idx = 0;
  for (int i = 0; i < g->ndim; ++i) idx += (long)c[i] * g->strides[i];
  return idx;
}

static int in_grid(const grid_t* g, const int* c) {
  for (int i = 0; i < g->ndim; ++i)
    if (c[i] < 0 || c[i] >= g->dims[i]) return 0;
  return 1;
}


/* Iterator over every voxel of the plane x_a = k, other axes in row-major order. */
typedef struct {
  const grid_t* g;
  int a, o[2], no;
  int xc[3];
  int done;
} plane_it;

static void plane_first(plane_it* it, const grid_t* g, int a, int k) {
  it->g = g;
  it->a = a;
  it->no = 0;
  for (int b = 0; b < g->ndim; ++b)
    if (b != a) it->o[it->no++] = b;
  it->xc[0] = it->xc[1] = it->xc[2] = 0;
  it->xc[a] = k;
  it->done = 0;
}

static void plane_next(plane_it* it) {
  for (int i = it->no - 1; i >= 0; --i) {
    int b = it->o[i];
    if (++it->xc[b] < it->g->dims[b]) return;
    it->xc[b] = 0;
  }
  it->done = 1;
}

/* S = sum over axes b (ascending) of (s_b * |dx_b|)^2, in double. */
static double spatial_sq(int ndim, const double* spacing, const int* dx) {
  double S = 0.0;
  for (int b = 0; b < ndim; ++b) {
    double t = spacing[b] * (double)abs(dx[b]);
    S = S + t * t;
  }
  return S;
}

/* Offsets of a pass along axis a: displacement from the updated voxel x back to
 * its candidate parent y is -sign on axis a and delta_b in {-1,0,+1} on every
 * other axis.  Enumerated lexicographically over the non-scan axes (ascending
 * axis index, each component -1, 0, +1).  Returns the count, 3^(ndim-1). */
static int pass_offsets(int ndim, int a, int (*delta)[3]) {
  int other[2], no = 0;
  for (int b = 0; b < ndim; ++b)
    if (b != a) other[no++] = b;
  int count = 1;
  for (int i = 0; i < no; ++i) count *= 3;
  for (int j = 0; j < count; ++j) {
    int rem = j;
    delta[j][0] = delta[j][1] = delta[j][2] = 0;
    for (int i = no - 1; i >= 0; --i) {
      delta[j][other[i]] = rem % 3 - 1;
      rem /= 3;
    }
  }
  return count;
}

/* ----------------------------------------------------- edge cost, FP32 / FP64 */

static float edge_w_f32(const float* img, long cs, int C, long x, long y, float lam, float A) {
  float d = img[x] - img[y];
  float g = d * d;
  for (int c = 1; c < C; ++c) {
    float dc = img[(long)c * cs + x] - img[(long)c * cs + y];
    g = fmaf(dc, dc, g);
  }
  float q = fmaf(lam, g, A);
  return sqrtf(q);
}

static double edge_w_f64(const double* img, long cs, int C, long x, long y, double lam, double A) {
  double d = img[x] - img[y];
  double g = d * d;
  for (int c = 1; c < C; ++c) {
    double dc = img[(long)c * cs + x] - img[(long)c * cs + y];
    g = fma(dc, dc, g);
  }
  double q = fma(lam, g, A);
  return sqrt(q);
}

static int check_common(int ndim, const int* dims, int C, const void* image, const void* mask,
                        const void* spacing, int iterations, const void* out, grid_t* g) {
  if (!dims || !image || !mask || !spacing || !out) return REF_EINVAL;
  if (C < 1 || iterations < 0) return REF_EINVAL;
  return grid_init(g, ndim, dims);
}

/* ------------------------------------------------------------ the schedule */

/* One directional pass along axis a in direction sign (+1 / -1), in place on D.
 * rec (nullable) receives one byte per voxel: 0 = keep, 1 + j = parent through
 * offset j of pass_offsets(). */
/* Update of one voxel x (coordinates xc, on plane k of a pass along axis a):
 * the keep candidate D(x), then the parents of plane k - sign in offset order. */
static void update_voxel_f32(const grid_t* g, int C, const float* img, float lam, const float* A,
                             const int (*delta)[3], int nd, int a, int sign, int k, const int* xc,
                             float* D, uint8_t* rec) {
  long cs = g->n;
  long i = flatten(g, xc);
  float best = D[i];
  uint8_t choice = 0;
  for (int j = 0; j < nd; ++j) {
    int yc[3];
    for (int b = 0; b < g->ndim; ++b) yc[b] = xc[b] + delta[j][b];
    yc[a] = k - sign;
    if (!in_grid(g, yc)) continue;
    long y = flatten(g, yc);
    float w = edge_w_f32(img, cs, C, i, y, lam, A[j]);
    float cand = D[y] + w;
    if (cand < best) {
      best = cand;
      choice = (uint8_t)(1 + j);
    }
  }
  D[i] = best;
  if (rec) rec[i] = choice;
}

static void pass_tables_f32(const grid_t* g, const double* sp, float lam, int a, int (*delta)[3], float* A,
                            int* nd) {
  *nd = pass_offsets(g->ndim, a, delta);
  for (int j = 0; j < *nd; ++j) {
    int dx[3] = {delta[j][0], delta[j][1], delta[j][2]};
    dx[a] = 1;
    A[j] = (float)((1.0 - (double)lam) * spatial_sq(g->ndim, sp, dx));
  }
}

static void pass_f32(const grid_t* g, int C, const float* img, const double* sp, float lam,
                     int a, int sign, float* D, uint8_t* rec) {
  int delta[9][3], nd;
  float A[9];
  pass_tables_f32(g, sp, lam, a, delta, A, &nd);
  int Na = g->dims[a];
  if (rec) {
    /* the first plane in scan order is never modified */
    plane_it pf;
    for (plane_first(&pf, g, a, sign > 0 ? 0 : Na - 1); !pf.done; plane_next(&pf))
      rec[flatten(g, pf.xc)] = 0;
  }
  for (int t = 1; t < Na; ++t) {
    int k = sign > 0 ? t : Na - 1 - t;
    /* all voxels of plane k; they read plane k - sign only */
    plane_it pi;
    for (plane_first(&pi, g, a, k); !pi.done; plane_next(&pi))
      update_voxel_f32(g, C, img, lam, A, (const int (*)[3])delta, nd, a, sign, k, pi.xc, D, rec);
  }
}

/* The same pass with the voxels of each plane shared among OpenMP threads (the
 * paper's CPU parallelisation: a plane's voxels only read the previous plane, so
 * any order gives the same values). */
static void pass_f32_omp(const grid_t* g, int C, const float* img, const double* sp, float lam,
                         int a, int sign, float* D) {
  int delta[9][3], nd;
  float A[9];
  pass_tables_f32(g, sp, lam, a, delta, A, &nd);
  int Na = g->dims[a];
  int o[2] = {0, 0}, no = 0;
  for (int b = 0; b < g->ndim; ++b)
    if (b != a) o[no++] = b;
  long P = 1;
  for (int i = 0; i < no; ++i) P *= g->dims[o[i]];
  for (int t = 1; t < Na; ++t) {
    int k = sign > 0 ? t : Na - 1 - t;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < P; ++m) {
      int xc[3] = {0, 0, 0};
      long r = m;
      for (int i = no - 1; i >= 0; --i) {
        xc[o[i]] = (int)(r % g->dims[o[i]]);
        r /= g->dims[o[i]];
      }
      xc[a] = k;
      update_voxel_f32(g, C, img, lam, A, (const int (*)[3])delta, nd, a, sign, k, xc, D, NULL);
    }
  }
}

static void pass_f64(const grid_t* g, int C, const double* img, const double* sp, double lam,
                     int a, int sign, double* D, uint8_t* rec) {
  int delta[9][3];
  int nd = pass_offsets(g->ndim, a, delta);
  double A[9];
  for (int j = 0; j < nd; ++j) {
    int dx[3] = {delta[j][0], delta[j][1], delta[j][2]};
    dx[a] = 1;
    A[j] = (1.0 - lam) * spatial_sq(g->ndim, sp, dx);
  }
  int Na = g->dims[a];
  long cs = g->n;
  if (rec) {
    plane_it pf;
    for (plane_first(&pf, g, a, sign > 0 ? 0 : Na - 1); !pf.done; plane_next(&pf))
      rec[flatten(g, pf.xc)] = 0;
  }
  for (int t = 1; t < Na; ++t) {
    int k = sign > 0 ? t : Na - 1 - t;
    plane_it pi;
    for (plane_first(&pi, g, a, k); !pi.done; plane_next(&pi)) {
      const int* xc = pi.xc;
      long i = flatten(g, xc);
      double best = D[i];
      uint8_t choice = 0;
      for (int j = 0; j < nd; ++j) {
        int yc[3];
        for (int b = 0; b < g->ndim; ++b) yc[b] = xc[b] + delta[j][b];
        yc[a] = k - sign;
        if (!in_grid(g, yc)) continue;
        long y = flatten(g, yc);
        double w = edge_w_f64(img, cs, C, i, y, lam, A[j]);
        double cand = D[y] + w;
        if (cand < best) {
          best = cand;
          choice = (uint8_t)(1 + j);
        }
      }
      D[i] = best;
      if (rec) rec[i] = choice;
    }
  }
}

/* Number of directional passes in one iteration. */
int ref_passes_per_iteration(int ndim) { return 2 * ndim; }

/* Full fixed-iteration schedule, FP32.  image: (C, dims...) channel-planar;
 * mask: (dims...); spacing: ndim values in array-axis order; out: (dims...).
 * records (nullable): iterations * 2*ndim planes of n bytes, pass-major. */
int ref_ggdt_f32(int ndim, const int* dims, int C, const float* image, const float* mask,
                 const float* spacing, float v, float lam, int iterations, float* out,
                 uint8_t* records) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (rc) return rc;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  int p = 0;
  for (int it = 0; it < iterations; ++it)
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s, ++p)
        pass_f32(&g, C, image, sp, lam, a, s == 0 ? +1 : -1, out, records ? records + (long)p * g.n : NULL);
  return REF_OK;
}

/* ref_ggdt_f32 with every plane's voxels shared among OpenMP threads; same
 * result.  Returns the number of threads used, or a negative error. */
int ref_ggdt_f32_omp(int ndim, const int* dims, int C, const float* image, const float* mask,
                     const float* spacing, float v, float lam, int iterations, float* out) {
  grid_t g;
  int e = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (e) return e;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  for (int it = 0; it < iterations; ++it)
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s) pass_f32_omp(&g, C, image, sp, lam, a, s == 0 ? +1 : -1, out);
  int nt = 1;
#pragma omp parallel
  {
#pragma omp single
    nt = omp_get_num_threads();
  }
  return nt;
}

int ref_ggdt_f64(int ndim, const int* dims, int C, const double* image, const double* mask,
                 const double* spacing, double v, double lam, int iterations, double* out,
                 uint8_t* records) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (rc) return rc;
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  int p = 0;
  for (int it = 0; it < iterations; ++it)
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s, ++p)
        pass_f64(&g, C, image, spacing, lam, a, s == 0 ? +1 : -1, out, records ? records + (long)p * g.n : NULL);
  return REF_OK;
}

/* A single directional pass applied to a given D (in place), FP32 / FP64.
 * Lets a caller compose the schedule pass by pass. */
int ref_pass_f32(int ndim, const int* dims, int C, const float* image, const float* spacing,
                 float lam, int axis, int sign, float* D, uint8_t* rec) {
  grid_t g;
  if (!dims || !image || !spacing || !D || C < 1) return REF_EINVAL;
  if (grid_init(&g, ndim, dims)) return REF_EINVAL;
  if (axis < 0 || axis >= ndim || (sign != 1 && sign != -1)) return REF_EINVAL;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  pass_f32(&g, C, image, sp, lam, axis, sign, D, rec);
  return REF_OK;
}

int ref_pass_f64(int ndim, const int* dims, int C, const double* image, const double* spacing,
                 double lam, int axis, int sign, double* D, uint8_t* rec) {
  grid_t g;
  if (!dims || !image || !spacing || !D || C < 1) return REF_EINVAL;
  if (grid_init(&g, ndim, dims)) return REF_EINVAL;
  if (axis < 0 || axis >= ndim || (sign != 1 && sign != -1)) return REF_EINVAL;
  pass_f64(&g, C, image, spacing, lam, axis, sign, D, rec);
  return REF_OK;
}

/* Iterate whole iterations until one changes no voxel bitwise (at most
 * max_iterations).  Returns the number of iterations after which the state was
 * already fixed, or -1 if the cap was hit; out holds the final state. */
/* ------------------------------------------- Toivanen's sequential raster scan
 * The paper's software also ships the sequential raster-scan transform of
 * Toivanen (1996) for comparison (section "Implementation"), run on one CPU
 * thread.  Reading used here: one iteration is a forward sweep over the voxels
 * in raster order (row-major, every axis ascending) followed by a backward
 * sweep in the reverse order; a voxel takes the minimum of its own value and
 * D(y) + w(x, y) over the neighbours y of the 8/26-neighbourhood that precede it
 * in the sweep's order (4 in 2D, 13 in 3D), updating D in place, so it sees the
 * values already lowered earlier in the same sweep.  Edge costs as in the
 * passes: w = sqrt((1 - lam) |x - y|_s^2 + lam |I(x) - I(y)|^2). */

/* Offsets y - x of the neighbours preceding x in the forward raster order
 * (first non-zero component negative); the backward sweep uses their negatives. */
static int causal_offsets(int ndim, int (*off)[3]) {
  int n = 0;
  for (int dz = (ndim == 3 ? -1 : 0); dz <= (ndim == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int d[3] = {0, 0, 0};
        if (ndim == 3) {
          d[0] = dz; d[1] = dy; d[2] = dx;
        } else {
          d[0] = dy; d[1] = dx;
        }
        int first = 0;
        for (int b = 0; b < ndim && first == 0; ++b) first = d[b];
        if (first < 0) {
          off[n][0] = d[0]; off[n][1] = d[1]; off[n][2] = d[2];
          ++n;
        }
      }
  return n;
}

static void toivanen_sweep_f32(const grid_t* g, int C, const float* img, const double* sp, float lam, int dir,
                               float* D) {
  int off[13][3];
  int no = causal_offsets(g->ndim, off);
  float A[13];
  for (int j = 0; j < no; ++j) {
    int dx[3] = {abs(off[j][0]), abs(off[j][1]), abs(off[j][2])};
    A[j] = (float)((1.0 - (double)lam) * spatial_sq(g->ndim, sp, dx));
  }
  for (long t = 0; t < g->n; ++t) {
    long i = dir > 0 ? t : g->n - 1 - t;
    int xc[3] = {0, 0, 0};
    unflatten(g, i, xc);
    float best = D[i];
    for (int j = 0; j < no; ++j) {
      int yc[3];
      for (int b = 0; b < g->ndim; ++b) yc[b] = xc[b] + dir * off[j][b];
      if (!in_grid(g, yc)) continue;
      long y = flatten(g, yc);
      float cand = D[y] + edge_w_f32(img, g->n, C, i, y, lam, A[j]);
      if (cand < best) best = cand;
    }
    D[i] = best;
  }
}

static void toivanen_sweep_f64(const grid_t* g, int C, const double* img, const double* sp, double lam, int dir,
                               double* D) {
  int off[13][3];
  int no = causal_offsets(g->ndim, off);
  double A[13];
  for (int j = 0; j < no; ++j) {
    int dx[3] = {abs(off[j][0]), abs(off[j][1]), abs(off[j][2])};
    A[j] = (1.0 - lam) * spatial_sq(g->ndim, sp, dx);
  }
  for (long t = 0; t < g->n; ++t) {
    long i = dir > 0 ? t : g->n - 1 - t;
    int xc[3] = {0, 0, 0};
    unflatten(g, i, xc);
    double best = D[i];
    for (int j = 0; j < no; ++j) {
      int yc[3];
      for (int b = 0; b < g->ndim; ++b) yc[b] = xc[b] + dir * off[j][b];
      if (!in_grid(g, yc)) continue;
      long y = flatten(g, yc);
      double cand = D[y] + edge_w_f64(img, g->n, C, i, y, lam, A[j]);
      if (cand < best) best = cand;
    }
    D[i] = best;
  }
}

/* Toivanen's transform.  converge == 0: exactly `iterations` iterations,
 * returns 0.  converge != 0: iterations until one changes nothing (at most
 * `iterations`), returns the number that changed some value, or -1. */
int ref_toivanen_f32(int ndim, const int* dims, int C, const float* image, const float* mask,
                     const float* spacing, float v, float lam, int iterations, int converge, float* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (rc) return rc;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  float* prev = converge ? (float*)malloc(sizeof(float) * g.n) : NULL;
  if (converge && !prev) return REF_ENOMEM;
  int result = converge ? -1 : 0;
  for (int it = 1; it <= iterations; ++it) {
    if (prev) memcpy(prev, out, sizeof(float) * g.n);
    toivanen_sweep_f32(&g, C, image, sp, lam, +1, out);
    toivanen_sweep_f32(&g, C, image, sp, lam, -1, out);
    if (prev && memcmp(prev, out, sizeof(float) * g.n) == 0) {
      result = it - 1;
      break;
    }
  }
  free(prev);
  return result;
}

int ref_toivanen_f64(int ndim, const int* dims, int C, const double* image, const double* mask,
                     const double* spacing, double v, double lam, int iterations, int converge, double* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (rc) return rc;
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  double* prev = converge ? (double*)malloc(sizeof(double) * g.n) : NULL;
  if (converge && !prev) return REF_ENOMEM;
  int result = converge ? -1 : 0;
  for (int it = 1; it <= iterations; ++it) {
    if (prev) memcpy(prev, out, sizeof(double) * g.n);
    toivanen_sweep_f64(&g, C, image, spacing, lam, +1, out);
    toivanen_sweep_f64(&g, C, image, spacing, lam, -1, out);
    if (prev && memcmp(prev, out, sizeof(double) * g.n) == 0) {
      result = it - 1;
      break;
    }
  }
  free(prev);
  return result;
}

int ref_ggdt_until_converged_f32(int ndim, const int* dims, int C, const float* image,
                                 const float* mask, const float* spacing, float v, float lam,
                                 int max_iterations, float* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, max_iterations, out, &g);
  if (rc) return rc;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  float* prev = (float*)malloc(sizeof(float) * g.n);
  if (!prev) return REF_ENOMEM;
  int result = -1;
  for (int it = 1; it <= max_iterations; ++it) {
    memcpy(prev, out, sizeof(float) * g.n);
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s) pass_f32(&g, C, image, sp, lam, a, s == 0 ? +1 : -1, out, NULL);
    if (memcmp(prev, out, sizeof(float) * g.n) == 0) {
      result = it - 1;
      break;
    }
  }
  free(prev);
  return result;
}

int ref_ggdt_until_converged_f64(int ndim, const int* dims, int C, const double* image,
                                 const double* mask, const double* spacing, double v, double lam,
                                 int max_iterations, double* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, max_iterations, out, &g);
  if (rc) return rc;
  for (long i = 0; i < g.n; ++i) out[i] = v * mask[i];
  double* prev = (double*)malloc(sizeof(double) * g.n);
  if (!prev) return REF_ENOMEM;
  int result = -1;
  for (int it = 1; it <= max_iterations; ++it) {
    memcpy(prev, out, sizeof(double) * g.n);
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s) pass_f64(&g, C, image, spacing, lam, a, s == 0 ? +1 : -1, out, NULL);
    if (memcmp(prev, out, sizeof(double) * g.n) == 0) {
      result = it - 1;
      break;
    }
  }
  free(prev);
  return result;
}

/* ------------------------------------------------------ multi-source Dijkstra */

typedef struct {
  double key;
  long node;
} heap_item;

typedef struct {
  heap_item* a;
  long size, cap;
} heap_t;

static int heap_push(heap_t* h, double key, long node) {
  if (h->size == h->cap) {
    long nc = h->cap ? 2 * h->cap : 1024;
    heap_item* na = (heap_item*)realloc(h->a, sizeof(heap_item) * nc);
    if (!na) return REF_ENOMEM;
    h->a = na;
    h->cap = nc;
  }
  long i = h->size++;
  h->a[i].key = key;
  h->a[i].node = node;
  while (i > 0) {
    long p = (i - 1) / 2;
    if (h->a[p].key <= h->a[i].key) break;
    heap_item t = h->a[p];
    h->a[p] = h->a[i];
    h->a[i] = t;
    i = p;
  }
  return REF_OK;
}

static heap_item heap_pop(heap_t* h) {
  heap_item top = h->a[0];
  h->a[0] = h->a[--h->size];
  long i = 0;
  for (;;) {
    long l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->size && h->a[l].key < h->a[m].key) m = l;
    if (r < h->size && h->a[r].key < h->a[m].key) m = r;
    if (m == i) break;
    heap_item t = h->a[m];
    h->a[m] = h->a[i];
    h->a[i] = t;
    i = m;
  }
  return top;
}

/* Shortest paths on the 8- (2D) / 26- (3D) connected grid, every voxel a source
 * with initial cost v*M.  Edge cost is the same w as the scan uses (w is
 * symmetric); path costs are accumulated from the source towards the target,
 * one rounding per edge, in the working precision. */
int ref_dijkstra_f32(int ndim, const int* dims, int C, const float* image, const float* mask,
                     const float* spacing, float v, float lam, float* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, 0, out, &g);
  if (rc) return rc;
  double sp[3];
  for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing[b];
  int nb = 0, off[26][3];
  float A[26];
  for (int dz = (ndim == 3 ? -1 : 0); dz <= (ndim == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int d[3];
        if (ndim == 3) { d[0] = dz; d[1] = dy; d[2] = dx; }
        else { d[0] = dy; d[1] = dx; d[2] = 0; }
        if (d[0] == 0 && d[1] == 0 && d[2] == 0) continue;
        memcpy(off[nb], d, sizeof d);
        A[nb] = (float)((1.0 - (double)lam) * spatial_sq(ndim, sp, d));
        ++nb;
      }
  char* done = (char*)calloc(g.n, 1);
  heap_t h = {0, 0, 0};
  if (!done) return REF_ENOMEM;
  for (long i = 0; i < g.n; ++i) {
    out[i] = v * mask[i];
    if (heap_push(&h, (double)out[i], i)) { free(done); free(h.a); return REF_ENOMEM; }
  }
  while (h.size > 0) {
    heap_item it = heap_pop(&h);
    long u = it.node;
    if (done[u] || it.key != (double)out[u]) continue;
    done[u] = 1;
    int uc[3];
    unflatten(&g, u, uc);
    for (int j = 0; j < nb; ++j) {
      int zc[3];
      for (int b = 0; b < ndim; ++b) zc[b] = uc[b] + off[j][b];
      if (!in_grid(&g, zc)) continue;
      long z = flatten(&g, zc);
      if (done[z]) continue;
      float w = edge_w_f32(image, g.n, C, z, u, lam, A[j]);
      float cand = out[u] + w;
      if (cand < out[z]) {
        out[z] = cand;
        if (heap_push(&h, (double)cand, z)) { free(done); free(h.a); return REF_ENOMEM; }
      }
    }
  }
  free(done);
  free(h.a);
  return REF_OK;
}

int ref_dijkstra_f64(int ndim, const int* dims, int C, const double* image, const double* mask,
                     const double* spacing, double v, double lam, double* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, 0, out, &g);
  if (rc) return rc;
  int nb = 0, off[26][3];
  double A[26];
  for (int dz = (ndim == 3 ? -1 : 0); dz <= (ndim == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int d[3];
        if (ndim == 3) { d[0] = dz; d[1] = dy; d[2] = dx; }
        else { d[0] = dy; d[1] = dx; d[2] = 0; }
        if (d[0] == 0 && d[1] == 0 && d[2] == 0) continue;
        memcpy(off[nb], d, sizeof d);
        A[nb] = (1.0 - lam) * spatial_sq(ndim, spacing, d);
        ++nb;
      }
  char* done = (char*)calloc(g.n, 1);
  heap_t h = {0, 0, 0};
  if (!done) return REF_ENOMEM;
  for (long i = 0; i < g.n; ++i) {
    out[i] = v * mask[i];
    if (heap_push(&h, out[i], i)) { free(done); free(h.a); return REF_ENOMEM; }
  }
  while (h.size > 0) {
    heap_item it = heap_pop(&h);
    long u = it.node;
    if (done[u] || it.key != out[u]) continue;
    done[u] = 1;
    int uc[3];
    unflatten(&g, u, uc);
    for (int j = 0; j < nb; ++j) {
      int zc[3];
      for (int b = 0; b < ndim; ++b) zc[b] = uc[b] + off[j][b];
      if (!in_grid(&g, zc)) continue;
      long z = flatten(&g, zc);
      if (done[z]) continue;
      double w = edge_w_f64(image, g.n, C, z, u, lam, A[j]);
      double cand = out[u] + w;
      if (cand < out[z]) {
        out[z] = cand;
        if (heap_push(&h, cand, z)) { free(done); free(h.a); return REF_ENOMEM; }
      }
    }
  }
  free(done);
  free(h.a);
  return REF_OK;
}

/* ------------------------------------------------- lambda = 0 closed form */

/* With lambda = 0 the edge cost is the spacing-weighted length of a king move.
 * The cheapest king-move path for a displacement with per-axis step counts
 * sorted n1 >= n2 >= n3 (axes i1, i2, i3) uses n3 moves along all three axes,
 * n2 - n3 along {i1, i2} and n1 - n2 along i1 alone.  out(x) = min over every
 * voxel y of v*M(y) + that chain length, in FP64 (O(n^2); small grids only). */
int ref_chamfer_closed_form_f64(int ndim, const int* dims, const double* mask,
                                const double* spacing, double v, double* out) {
  grid_t g;
  if (!dims || !mask || !spacing || !out) return REF_EINVAL;
  if (grid_init(&g, ndim, dims)) return REF_EINVAL;
  for (long x = 0; x < g.n; ++x) {
    int xc[3];
    unflatten(&g, x, xc);
    double best = v * mask[x];
    for (long y = 0; y < g.n; ++y) {
      int yc[3];
      unflatten(&g, y, yc);
      int cnt[3] = {0, 0, 0}, ax[3] = {0, 1, 2};
      for (int b = 0; b < ndim; ++b) cnt[b] = abs(xc[b] - yc[b]);
      /* sort axes by count, descending */
      for (int i = 0; i < ndim; ++i)
        for (int j = i + 1; j < ndim; ++j)
          if (cnt[ax[j]] > cnt[ax[i]]) { int t = ax[i]; ax[i] = ax[j]; ax[j] = t; }
      double s1 = spacing[ax[0]] * spacing[ax[0]];
      double s2 = ndim > 1 ? spacing[ax[1]] * spacing[ax[1]] : 0.0;
      double s3 = ndim > 2 ? spacing[ax[2]] * spacing[ax[2]] : 0.0;
      double n1 = cnt[ax[0]], n2 = ndim > 1 ? cnt[ax[1]] : 0, n3 = ndim > 2 ? cnt[ax[2]] : 0;
      double len = n3 * sqrt(s1 + s2 + s3) + (n2 - n3) * sqrt(s1 + s2) + (n1 - n2) * sqrt(s1);
      double c = v * mask[y] + len;
      if (c < best) best = c;
    }
    out[x] = best;
  }
  return REF_OK;
}

/* ---------------------------------------------------- path enumeration */

typedef struct {
  const grid_t* g;
  int C;
  const double* img;
  const double* sp;
  double lam;
  double* best;
  char* on_path;
  long visits;
  long max_visits;
  int prune;
} dfs_ctx;

static double edge_between_f64(const dfs_ctx* c, long x, long y) {
  int xc[3], yc[3], d[3] = {0, 0, 0};
  unflatten(c->g, x, xc);
  unflatten(c->g, y, yc);
  for (int b = 0; b < c->g->ndim; ++b) d[b] = xc[b] - yc[b];
  double A = (1.0 - c->lam) * spatial_sq(c->g->ndim, c->sp, d);
  return edge_w_f64(c->img, c->g->n, c->C, x, y, c->lam, A);
}

/* Extend a path that currently ends at u with accumulated cost `cost` (folded
 * from the path's start).  Without pruning every simple path is visited; with
 * pruning a branch stops once its cost is no better than the best known cost
 * of its end voxel (exact for non-negative edges and monotone rounding). */
static int dfs(dfs_ctx* c, long u, double cost) {
  if (++c->visits > c->max_visits) return -1;
  if (cost < c->best[u]) c->best[u] = cost;
  int uc[3];
  unflatten(c->g, u, uc);
  int nd = c->g->ndim;
  for (int dz = (nd == 3 ? -1 : 0); dz <= (nd == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int d[3];
        if (nd == 3) { d[0] = dz; d[1] = dy; d[2] = dx; }
        else { d[0] = dy; d[1] = dx; d[2] = 0; }
        if (!d[0] && !d[1] && !d[2]) continue;
        int zc[3];
        for (int b = 0; b < nd; ++b) zc[b] = uc[b] + d[b];
        if (!in_grid(c->g, zc)) continue;
        long z = flatten(c->g, zc);
        if (c->on_path[z]) continue;
        double nc = cost + edge_between_f64(c, z, u);
        if (c->prune && nc >= c->best[z]) continue;
        c->on_path[z] = 1;
        int r = dfs(c, z, nc);
        c->on_path[z] = 0;
        if (r) return r;
      }
  return 0;
}

/* Minimum over all simple paths (prune = 0) or over all walks with
 * bound pruning (prune = 1), every voxel a start with cost v*M.  Returns -1 if
 * max_visits was exceeded. */
int ref_bruteforce_paths_f64(int ndim, const int* dims, int C, const double* image,
                             const double* mask, const double* spacing, double v, double lam,
                             int prune, long max_visits, double* out) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, 0, out, &g);
  if (rc) return rc;
  dfs_ctx c;
  c.g = &g; c.C = C; c.img = image; c.sp = spacing; c.lam = lam;
  c.best = out; c.visits = 0; c.max_visits = max_visits; c.prune = prune;
  c.on_path = (char*)calloc(g.n, 1);
  if (!c.on_path) return REF_ENOMEM;
  for (long i = 0; i < g.n; ++i) out[i] = INFINITY;
  int r = 0;
  for (long s = 0; s < g.n && !r; ++s) {
    double start = v * mask[s];
    if (prune && start >= out[s] && out[s] != INFINITY) continue;
    c.on_path[s] = 1;
    r = dfs(&c, s, start);
    c.on_path[s] = 0;
  }
  free(c.on_path);
  return r ? -1 : REF_OK;
}

/* One pass as a minimum over chains: for a target x in plane k (scan order),
 * every chain y_j -> ... -> x that visits one plane per step (planes j..k, with
 * offsets -1/0/+1 on the other axes) contributes D_in(y_j) folded with its edge
 * costs; D_out(x) = min(D_in(x), all such chains).  No sweeping: each target is
 * evaluated on its own from D_in only. */
typedef struct {
  const grid_t* g;
  int C, a, sign;
  const double* img;
  const double* sp;
  double lam;
  const double* Din;
  long chain[512];
} chain_ctx;

static void chain_eval(chain_ctx* c, int len, double* best) {
  /* chain[len-1] is the start (furthest back), chain[0] the target */
  double cost = c->Din[c->chain[len - 1]];
  for (int i = len - 1; i > 0; --i) {
    long y = c->chain[i], x = c->chain[i - 1];
    int xc[3], yc[3], d[3] = {0, 0, 0};
    unflatten(c->g, x, xc);
    unflatten(c->g, y, yc);
    for (int b = 0; b < c->g->ndim; ++b) d[b] = xc[b] - yc[b];
    double A = (1.0 - c->lam) * spatial_sq(c->g->ndim, c->sp, d);
    cost = cost + edge_w_f64(c->img, c->g->n, c->C, x, y, c->lam, A);
  }
  if (cost < *best) *best = cost;
}

static void chain_rec(chain_ctx* c, int len, double* best) {
  /* every chain of length >= 2 ending at chain[0] is a candidate */
  if (len >= 2) chain_eval(c, len, best);
  long u = c->chain[len - 1];
  int uc[3];
  unflatten(c->g, u, uc);
  int Na = c->g->dims[c->a];
  int prev = uc[c->a] - c->sign;
  if (prev < 0 || prev >= Na) return;
  int delta[9][3];
  int nd = pass_offsets(c->g->ndim, c->a, delta);
  for (int j = 0; j < nd; ++j) {
    int yc[3];
    for (int b = 0; b < c->g->ndim; ++b) yc[b] = uc[b] + delta[j][b];
    yc[c->a] = prev;
    if (!in_grid(c->g, yc)) continue;
    c->chain[len] = flatten(c->g, yc);
    chain_rec(c, len + 1, best);
  }
}

int ref_pass_bruteforce_f64(int ndim, const int* dims, int C, const double* image,
                            const double* spacing, double lam, int axis, int sign,
                            const double* D_in, double* D_out) {
  grid_t g;
  if (!dims || !image || !spacing || !D_in || !D_out || C < 1) return REF_EINVAL;
  if (grid_init(&g, ndim, dims)) return REF_EINVAL;
  if (axis < 0 || axis >= ndim || (sign != 1 && sign != -1)) return REF_EINVAL;
  if (g.dims[axis] > 500) return REF_EINVAL;
  chain_ctx c;
  c.g = &g; c.C = C; c.a = axis; c.sign = sign; c.img = image; c.sp = spacing; c.lam = lam;
  c.Din = D_in;
  for (long x = 0; x < g.n; ++x) {
    double best = D_in[x];
    c.chain[0] = x;
    chain_rec(&c, 1, &best);
    D_out[x] = best;
  }
  return REF_OK;
}

/* ------------------------------------------------ reverse-mode gradient */

/* Exact reverse of the fixed schedule given its records (one byte per voxel
 * per pass, as written by ref_ggdt_*).  L is any loss with dL/dD = grad_out.
 * Walks passes in reverse and, inside a pass, planes against the scan order.
 * For plane k (the target plane) and its predecessor plane kp:
 *   - every y in plane kp gathers, over offsets j in canonical order, from the
 *     child x = y - delta_j in plane k whose record is 1 + j:
 *         abar(y) += abar(x);  Ibar_c(y) -= coef * d_c
 *   - then every updated x in plane k (record != 0):
 *         Ibar_c(x) += coef * d_c;  abar(x) = 0
 * with d_c = I_c(x) - I_c(y), coef = (abar(x) * lambda) / w (0 when w = 0).
 * Finally dL/dM = v * abar and dL/dI = Ibar. */
#define DEFINE_BACKWARD(NAME, T, EDGE, CASTSP)                                                   \
  int NAME(int ndim, const int* dims, int C, const T* image, const T* spacing_in, T v, T lam,     \
           int iterations, const uint8_t* records, const T* grad_out, T* grad_image,             \
           T* grad_mask) {                                                                       \
    grid_t g;                                                                                    \
    if (!dims || !image || !spacing_in || !records || !grad_out || !grad_image || !grad_mask)    \
      return REF_EINVAL;                                                                         \
    if (C < 1 || iterations < 0 || grid_init(&g, ndim, dims)) return REF_EINVAL;                 \
    double sp[3];                                                                                \
    for (int b = 0; b < ndim; ++b) sp[b] = (double)spacing_in[b];                                \
    T* abar = grad_mask;                                                                         \
    for (long i = 0; i < g.n; ++i) abar[i] = grad_out[i];                                        \
    for (long i = 0; i < (long)C * g.n; ++i) grad_image[i] = (T)0;                               \
    int npass = 2 * ndim;                                                                        \
    for (int p = iterations * npass - 1; p >= 0; --p) {                                          \
      int a = (p % npass) / 2, sign = (p % 2 == 0) ? 1 : -1;                                     \
      const uint8_t* rec = records + (long)p * g.n;                                              \
      int delta[9][3];                                                                           \
      int nd = pass_offsets(ndim, a, delta);                                                     \
      T A[9];                                                                                    \
      for (int j = 0; j < nd; ++j) {                                                             \
        int dx[3] = {delta[j][0], delta[j][1], delta[j][2]};                                     \
        dx[a] = 1;                                                                               \
        A[j] = CASTSP((1.0 - (double)lam) * spatial_sq(ndim, sp, dx));                           \
      }                                                                                          \
      int Na = g.dims[a];                                                                        \
      for (int t = Na - 1; t >= 1; --t) {                                                        \
        int k = sign > 0 ? t : Na - 1 - t;                                                       \
        int kp = k - sign;                                                                       \
        plane_it py;                                                                             \
        for (plane_first(&py, &g, a, kp); !py.done; plane_next(&py)) {                           \
          const int* yc = py.xc;                                                                 \
          long y = flatten(&g, yc);                                                              \
          for (int j = 0; j < nd; ++j) {                                                         \
            int xc[3];                                                                           \
            for (int b = 0; b < ndim; ++b) xc[b] = yc[b] - delta[j][b];                          \
            xc[a] = k;                                                                           \
            if (!in_grid(&g, xc)) continue;                                                      \
            long x = flatten(&g, xc);                                                            \
            if (rec[x] != 1 + j) continue;                                                       \
            abar[y] = abar[y] + abar[x];                                                         \
            T w = EDGE(image, g.n, C, x, y, lam, A[j]);                                          \
            if (w > (T)0) {                                                                      \
              T coef = (abar[x] * lam) / w;                                                      \
              for (int c = 0; c < C; ++c) {                                                      \
                T d = image[(long)c * g.n + x] - image[(long)c * g.n + y];                       \
                grad_image[(long)c * g.n + y] = grad_image[(long)c * g.n + y] - coef * d;        \
              }                                                                                  \
            }                                                                                    \
          }                                                                                      \
        }                                                                                        \
        plane_it px;                                                                             \
        for (plane_first(&px, &g, a, k); !px.done; plane_next(&px)) {                            \
          const int* xc = px.xc;                                                                 \
          long x = flatten(&g, xc);                                                              \
          if (rec[x] == 0) continue;                                                             \
          int j = rec[x] - 1;                                                                    \
          int yc[3];                                                                             \
          for (int b = 0; b < ndim; ++b) yc[b] = xc[b] + delta[j][b];                            \
          yc[a] = kp;                                                                            \
          long y = flatten(&g, yc);                                                              \
          T w = EDGE(image, g.n, C, x, y, lam, A[j]);                                            \
          if (w > (T)0) {                                                                        \
            T coef = (abar[x] * lam) / w;                                                        \
            for (int c = 0; c < C; ++c) {                                                        \
              T d = image[(long)c * g.n + x] - image[(long)c * g.n + y];                         \
              grad_image[(long)c * g.n + x] = grad_image[(long)c * g.n + x] + coef * d;          \
            }                                                                                    \
          }                                                                                      \
          abar[x] = (T)0;                                                                        \
        }                                                                                        \
      }                                                                                          \
    }                                                                                            \
    for (long i = 0; i < g.n; ++i) grad_mask[i] = v * abar[i];                                   \
    return REF_OK;                                                                               \
  }

#define CAST_F32(x) ((float)(x))
#define CAST_F64(x) ((double)(x))
DEFINE_BACKWARD(ref_ggdt_backward_f32, float, edge_w_f32, CAST_F32)
DEFINE_BACKWARD(ref_ggdt_backward_f64, double, edge_w_f64, CAST_F64)

/* ------------------------------------- incremental FP64 re-evaluation (checker)
 * The central-difference check of the gradient evaluates the FP64 schedule on
 * many inputs that differ from one base input at a single voxel (of M, or of
 * one image channel).  In a pass, a voxel's new value and record depend only on
 * its own value before the pass, its image values, and its parents' values
 * after their own update in that pass together with their image values.  So a
 * voxel none of whose inputs differ from the base run gets the base run's value
 * and record.  ref_ggdt_f64_trajectory stores the base run's state after every
 * pass; ref_ggdt_f64_perturbed recomputes, pass by pass and plane by plane in
 * scan order, only the voxels whose inputs may differ (a bounding box that
 * holds every one of them), with the arithmetic of pass_f64, and takes every
 * other voxel from the stored state.  Its output equals ref_ggdt_f64 on the
 * perturbed input bit for bit (tested against it); it is a faster way to get
 * the same numbers, not a different computation. */

/* State of the base run: traj[p * n ..] after p passes (traj[0] = v * M),
 * p = 0 .. npass; records as ref_ggdt_f64. */
int ref_ggdt_f64_trajectory(int ndim, const int* dims, int C, const double* image, const double* mask,
                            const double* spacing, double v, double lam, int iterations, double* traj,
                            uint8_t* records) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, traj, &g);
  if (rc) return rc;
  if (!records) return REF_EINVAL;
  for (long i = 0; i < g.n; ++i) traj[i] = v * mask[i];
  int p = 0;
  for (int it = 0; it < iterations; ++it)
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s, ++p) {
        memcpy(traj + (long)(p + 1) * g.n, traj + (long)p * g.n, sizeof(double) * (size_t)g.n);
        pass_f64(&g, C, image, spacing, lam, a, s == 0 ? +1 : -1, traj + (long)(p + 1) * g.n,
                 records + (long)p * g.n);
      }
  return REF_OK;
}

typedef struct {
  int lo[3], hi[3];
  int empty;
} box_t;

static void box_add(box_t* b, int ndim, const int* c) {
  for (int i = 0; i < ndim; ++i) {
    if (b->empty || c[i] < b->lo[i]) b->lo[i] = c[i];
    if (b->empty || c[i] > b->hi[i]) b->hi[i] = c[i];
  }
  b->empty = 0;
}

/* Union of box u with box s grown by r on every axis (clipped to the grid). */
static void box_union_grown(box_t* u, const box_t* s, int r, const grid_t* g) {
  if (s->empty) return;
  int lo[3], hi[3];
  for (int i = 0; i < g->ndim; ++i) {
    lo[i] = s->lo[i] - r < 0 ? 0 : s->lo[i] - r;
    hi[i] = s->hi[i] + r > g->dims[i] - 1 ? g->dims[i] - 1 : s->hi[i] + r;
  }
  box_add(u, g->ndim, lo);
  box_add(u, g->ndim, hi);
}

static int same_bits(double x, double y) { return memcmp(&x, &y, sizeof x) == 0; }

/* The FP64 schedule on the base input with one value changed: which = 0 sets
 * M(index) to mask[index] + delta, which = 1 sets I_channel(index) to
 * image[channel * n + index] + delta.  traj and records come from
 * ref_ggdt_f64_trajectory on the base input.  out receives the final D;
 * *same_records is 1 when every record equals the base run's.  Scratch: two
 * arrays of n values, one image copy. */
int ref_ggdt_f64_perturbed(int ndim, const int* dims, int C, const double* image, const double* mask,
                           const double* spacing, double v, double lam, int iterations, const double* traj,
                           const uint8_t* records, int which, int channel, long index, double delta, double* out,
                           int* same_records) {
  grid_t g;
  int rc = check_common(ndim, dims, C, image, mask, spacing, iterations, out, &g);
  if (rc) return rc;
  if (!traj || !records || !same_records || index < 0 || index >= g.n || (which != 0 && which != 1) ||
      (which == 1 && (channel < 0 || channel >= C)))
    return REF_EINVAL;
  const long n = g.n;
  const int npass = iterations * 2 * ndim;
  double* P = (double*)malloc(sizeof(double) * (size_t)n);
  uint8_t* chg = (uint8_t*)calloc((size_t)n, 1);
  double* img = (double*)malloc(sizeof(double) * (size_t)n * (size_t)C);
  if (!P || !chg || !img) {
    free(P);
    free(chg);
    free(img);
    return REF_ENOMEM;
  }
  memcpy(img, image, sizeof(double) * (size_t)n * (size_t)C);
  int pc[3] = {0, 0, 0};
  unflatten(&g, index, pc);
  if (which == 0) {
    const double d0 = v * (mask[index] + delta);
    if (!same_bits(d0, traj[index])) {
      chg[index] = 1;
      P[index] = d0;
    }
  } else {
    img[(long)channel * n + index] = image[(long)channel * n + index] + delta;
  }
  const int img_pert = which == 1 && !same_bits(img[(long)channel * n + index], image[(long)channel * n + index]);
  int same = 1;
  int p = 0;
  for (int it = 0; it < iterations; ++it)
    for (int a = 0; a < ndim; ++a)
      for (int s = 0; s < 2; ++s, ++p) {
        const int sign = s == 0 ? +1 : -1;
        const double* before = traj + (long)p * n;
        const double* after = traj + (long)(p + 1) * n;
        const uint8_t* rec0 = records + (long)p * n;
        int delta_[9][3];
        const int nd = pass_offsets(ndim, a, delta_);
        double A[9];
        for (int j = 0; j < nd; ++j) {
          int dx[3] = {delta_[j][0], delta_[j][1], delta_[j][2]};
          dx[a] = 1;
          A[j] = (1.0 - lam) * spatial_sq(ndim, spacing, dx);
        }
        /* voxels whose value before the pass differs, and the changed image voxel */
        box_t b0 = {{0, 0, 0}, {0, 0, 0}, 1};
        for (long i = 0; i < n; ++i)
          if (chg[i]) {
            int c[3];
            unflatten(&g, i, c);
            box_add(&b0, ndim, c);
          }
        if (img_pert) box_add(&b0, ndim, pc);
        if (b0.empty) continue; /* nothing differs: the base state after this pass holds */
        const int Na = g.dims[a];
        const int k0 = sign > 0 ? 0 : Na - 1;
        /* changed voxels of the previous plane (the first plane is not modified) */
        box_t prev = {{0, 0, 0}, {0, 0, 0}, 1};
        if (b0.lo[a] <= k0 && k0 <= b0.hi[a]) {
          prev = b0;
          prev.lo[a] = prev.hi[a] = k0;
        }
        for (int t = 1; t < Na; ++t) {
          const int k = sign > 0 ? t : Na - 1 - t;
          box_t r = {{0, 0, 0}, {0, 0, 0}, 1};
          if (b0.lo[a] <= k && k <= b0.hi[a]) box_union_grown(&r, &b0, 0, &g);
          box_union_grown(&r, &prev, 1, &g);
          if (img_pert && pc[a] == k - sign) {
            box_t e = {{pc[0], pc[1], pc[2]}, {pc[0], pc[1], pc[2]}, 0};
            box_union_grown(&r, &e, 1, &g);
          }
          box_t next = {{0, 0, 0}, {0, 0, 0}, 1};
          if (!r.empty) {
            r.lo[a] = r.hi[a] = k;
            int xc[3] = {r.lo[0], r.lo[1], r.lo[2]};
            for (;;) {
              const long x = flatten(&g, xc);
              int need = chg[x] || (img_pert && x == index);
              long ys[9];
              int ok[9];
              for (int j = 0; j < nd; ++j) {
                int yc[3];
                for (int b = 0; b < ndim; ++b) yc[b] = xc[b] + delta_[j][b];
                yc[a] = k - sign;
                ok[j] = in_grid(&g, yc);
                ys[j] = ok[j] ? flatten(&g, yc) : -1;
                if (ok[j] && (chg[ys[j]] || (img_pert && ys[j] == index))) need = 1;
              }
              if (need) {
                double best = chg[x] ? P[x] : before[x];
                uint8_t choice = 0;
                for (int j = 0; j < nd; ++j) {
                  if (!ok[j]) continue;
                  const long y = ys[j];
                  const double dy = chg[y] ? P[y] : after[y];
                  const double w = edge_w_f64(img, n, C, x, y, lam, A[j]);
                  const double cand = dy + w;
                  if (cand < best) {
                    best = cand;
                    choice = (uint8_t)(1 + j);
                  }
                }
                if (choice != rec0[x]) same = 0;
                chg[x] = !same_bits(best, after[x]);
                P[x] = best;
                if (chg[x]) box_add(&next, ndim, xc);
              }
              /* next voxel of the box, row-major over the non-scan axes */
              int b = ndim - 1;
              for (; b >= 0; --b) {
                if (b == a) continue;
                if (++xc[b] <= r.hi[b]) break;
                xc[b] = r.lo[b];
              }
              if (b < 0) break;
            }
          }
          prev = next;
        }
      }
  const double* fin = traj + (long)npass * n;
  for (long i = 0; i < n; ++i) out[i] = chg[i] ? P[i] : fin[i];
  *same_records = same;
  free(P);
  free(chg);
  free(img);
  return REF_OK;
}
