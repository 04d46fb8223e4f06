// C ABI of Toivanen's raster scan on the GPU (toivanen.hip): validation, the
// causal offsets and their edge constants, and the launches.
#include <limits.h>
#include <stdlib.h>
#include <string.h>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "toivanen.h"

namespace ggdt {
namespace {

// Descriptor of the transform: a 2D image is the volume {1, H, W}; the
// offsets are those whose first non-zero component (over the array axes) is
// negative, their constants A_j = (float)((1 - lambda) * S_j) with S_j the sum
// over axes ascending of (s_b |d_b|)^2 in double, as for the passes.
int make_desc(const Problem& pr, const float* image, const float* spacing, float lam, int iterations, float* out,
              ToivDesc* d) {
  memset(d, 0, sizeof *d);
  d->image = image;
  d->D = out;
  d->N = (long long)pr.N;
  d->C = pr.C;
  d->dims[0] = pr.ndim == 3 ? pr.dims[0] : 1;
  d->dims[1] = pr.dims[pr.ndim - 2];
  d->dims[2] = pr.dims[pr.ndim - 1];
  d->lam = lam;
  d->iterations = iterations;
  const long long T = 4LL * (d->dims[0] - 1) + 2LL * (d->dims[1] - 1) + (d->dims[2] - 1) + 1;
  if (T > INT_MAX) return GGDT_ERR_UNSUPPORTED;
  d->T = (int)T;
  int n = 0;
  for (int dz = (pr.ndim == 3 ? -1 : 0); dz <= (pr.ndim == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int first = dz != 0 ? dz : (dy != 0 ? dy : dx);
        if (first >= 0) continue;
        const int o[3] = {dz, dy, dx};
        // the array axes of the offset (2D: only dy, dx)
        const int* a = pr.ndim == 3 ? o : o + 1;
        double S = 0.0;
        for (int b = 0; b < pr.ndim; ++b) {
          const double t = (double)spacing[b] * (double)abs(a[b]);
          S = S + t * t;
        }
        d->off[n][0] = dz;
        d->off[n][1] = dy;
        d->off[n][2] = dx;
        d->A[n] = (float)((1.0 - (double)lam) * S);
        ++n;
      }
  d->noff = n;
  // the edge cost's forms, chosen as for the passes: w = |I(x) - I(y)| for
  // lambda 1 and one channel, else the root, in its normal-range form where
  // the argument is known to allow it
  d->mode = (lam == 1.0f && pr.C == 1) ? kModeLam1C1 : kModeGeneral;
  d->sqrt_normal = sqrt_normal_for(d->A, n);
  return GGDT_OK;
}

int toivanen_entry(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
                   float v, float lam, int iterations, float* out, void* ws, size_t wsb, hipStream_t stream) {
  if (!image || !mask || !out || !ws || !dims) return GGDT_ERR_NULL_PTR;
  Problem pr;
  int rc = make_problem(ndim, dims, C, &pr);
  if (rc) return rc;
  rc = check_params(ndim, spacing, v, lam, iterations);
  if (rc) return rc;
  const Tuning tu{};
  if (wsb < workspace_for(pr, tu)) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr.N * 4, ni = (size_t)pr.N * pr.C * 4;
  const void* ins[3] = {image, mask, ws};
  const size_t nins[3] = {ni, nb, wsb};
  rc = check_alias(out, nb, ins, nins, 3);
  if (rc) return rc;
  ToivDesc d;
  rc = make_desc(pr, image, spacing, lam, iterations, out, &d);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  // progress words in the exchange area after the header
  const long long nwords = (long long)((workspace_for(pr, tu) - (size_t)kHeaderWords * 4) / 8);
  if ((rc = toivanen_plan(&d, nwords))) return rc;
  unsigned* words = (unsigned*)ws;
  if (launch_reset(words, (long long)(workspace_for(pr, tu) / 4), stream) != hipSuccess) return GGDT_ERR_HIP;
  if (launch_scale(mask, v, out, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  if (iterations == 0) return GGDT_OK;
  // image classification (tiny or huge values), which picks the edge cost's form on the device
  if (launch_classify(image, (long long)pr.C * pr.N, words, stream) != hipSuccess) return GGDT_ERR_HIP;
  return launch_toivanen(d, words, g_spin_limit, stream) == hipSuccess ? GGDT_OK : GGDT_ERR_HIP;
}

}  // namespace
}  // namespace ggdt

using namespace ggdt;

extern "C" {

int ggdt2d_toivanen(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
  const int dims[2] = {H, W};
  return toivanen_entry(2, dims, C, image, softmask, spacing, v, lambda, iterations, out, workspace, workspace_bytes,
                        stream);
}

int ggdt3d_toivanen(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int iterations, float* out, int C, int D, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return toivanen_entry(3, dims, C, image, softmask, spacing, v, lambda, iterations, out, workspace, workspace_bytes,
                        stream);
}

}  // extern "C"
