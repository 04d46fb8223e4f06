// C ABI of the signed distance and the geodesic symmetric filter: the forward
// schedule run on derived masks, joined by the pointwise kernels of compose.hip.
// The paper names both operations (sections "Statement of need" and
// "Implementation") without defining them; the composition implemented here is
// the one documented in ggdt.h.
#include <math.h>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "ggdt_internal.h"

namespace ggdt {
namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace: the transform's header and exchange words, then nbuf fp32
// buffers of N values, each 256-byte aligned, then (optional) the scan-major
// copies of the transform.
size_t compose_workspace(const Problem& pr, int nbuf) {
  return align256(workspace_for(pr, Tuning{})) + (size_t)nbuf * align256((size_t)pr.N * 4);
}

void* scan_major_area(const Problem& pr, int nbuf, void* ws, size_t wsb) {
  const size_t base = compose_workspace(pr, nbuf), extra = scan_major_bytes(pr);
  if (extra == 0 || wsb < base + extra) return nullptr;
  return static_cast<unsigned char*>(ws) + base;
}

float* buffer(void* ws, const Problem& pr, int i) {
  return reinterpret_cast<float*>(static_cast<unsigned char*>(ws) + align256(workspace_for(pr, Tuning{})) +
                                  (size_t)i * align256((size_t)pr.N * 4));
}

// dst = D(I; mask) - D(I; 1 - mask); tmp_a, tmp_b: N-value scratch buffers.
int enqueue_signed(const Problem& pr, const float* image, const float* mask, const float* spacing, float v,
                   float lam, int iterations, float* dst, float* tmp_a, float* tmp_b, void* ws, void* sm,
                   hipStream_t stream) {
  const Tuning tu{};
  int rc = enqueue_forward(pr, image, mask, spacing, v, lam, iterations, dst, nullptr, ws, tu, stream, kImgF32, sm);
  if (rc) return rc;
  if (launch_compose(kOpComplement, mask, nullptr, 0.0f, tmp_a, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  rc = enqueue_forward(pr, image, tmp_a, spacing, v, lam, iterations, tmp_b, nullptr, ws, tu, stream, kImgF32, sm);
  if (rc) return rc;
  if (launch_compose(kOpSub, dst, tmp_b, 0.0f, dst, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  return GGDT_OK;
}

// Shared validation; on success *pr describes the problem.
int validate(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
             float v, float lam, int iterations, const float* out, const void* ws, size_t wsb, int nbuf,
             Problem* pr) {
  if (!image || !mask || !out || !ws || !dims) return GGDT_ERR_NULL_PTR;
  int rc = make_problem(ndim, dims, C, pr);
  if (rc) return rc;
  rc = check_params(ndim, spacing, v, lam, iterations);
  if (rc) return rc;
  if (wsb < compose_workspace(*pr, nbuf)) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr->N * 4, ni = (size_t)pr->N * pr->C * 4;
  const void* ins[3] = {image, mask, ws};
  const size_t nins[3] = {ni, nb, wsb};
  rc = check_alias(out, nb, ins, nins, 3);
  if (rc) return rc;
  return check_device();
}

int signed_entry(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
                 float v, float lam, int iterations, float* out, void* ws, size_t wsb, hipStream_t stream) {
  Problem pr;
  const int rc = validate(ndim, dims, C, image, mask, spacing, v, lam, iterations, out, ws, wsb, 2, &pr);
  if (rc) return rc;
  return enqueue_signed(pr, image, mask, spacing, v, lam, iterations, out, buffer(ws, pr, 0), buffer(ws, pr, 1), ws,
                        scan_major_area(pr, 2, ws, wsb), stream);
}

int gsf_entry(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
              float theta_d, float theta_e, float v, float lam, int iterations, float* out, void* ws, size_t wsb,
              hipStream_t stream) {
  if (!(isfinite(theta_d) && theta_d >= 0.0f && isfinite(theta_e) && theta_e >= 0.0f)) return GGDT_ERR_BAD_PARAM;
  Problem pr;
  int rc = validate(ndim, dims, C, image, mask, spacing, v, lam, iterations, out, ws, wsb, 4, &pr);
  if (rc) return rc;
  float* w1 = buffer(ws, pr, 0);
  float* w2 = buffer(ws, pr, 1);
  float* w3 = buffer(ws, pr, 2);
  float* w4 = buffer(ws, pr, 3);
  void* sm = scan_major_area(pr, 4, ws, wsb);
  // S0 = S(M) -> w1
  rc = enqueue_signed(pr, image, mask, spacing, v, lam, iterations, w1, w2, w3, ws, sm, stream);
  if (rc) return rc;
  // dilated object {S0 < theta_d} -> w2; its signed distance S_d -> out
  if (launch_compose(kOpObjectMask, w1, nullptr, theta_d, w2, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  rc = enqueue_signed(pr, image, w2, spacing, v, lam, iterations, out, w3, w4, ws, sm, stream);
  if (rc) return rc;
  // eroded object {S0 < -theta_e} -> w1 (in place); its signed distance S_e -> w2
  if (launch_compose(kOpObjectMask, w1, nullptr, -theta_e, w1, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  rc = enqueue_signed(pr, image, w1, spacing, v, lam, iterations, w2, w3, w4, ws, sm, stream);
  if (rc) return rc;
  // (S_d + S_e) + (theta_e - theta_d)
  const float shift = theta_e - theta_d;
  if (launch_compose(kOpSumShift, out, w2, shift, out, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
  return GGDT_OK;
}

size_t workspace_query(int ndim, const int* dims, int C, int nbuf) {
  if (!dims) return 0;
  Problem pr;
  if (make_problem(ndim, dims, C, &pr)) return 0;
  return compose_workspace(pr, nbuf) + scan_major_bytes(pr);
}

}  // namespace
}  // namespace ggdt

using namespace ggdt;

extern "C" {

size_t ggdt_signed_workspace_bytes(int ndim, const int* dims, int C) { return workspace_query(ndim, dims, C, 2); }

size_t ggdt_gsf_workspace_bytes(int ndim, const int* dims, int C) { return workspace_query(ndim, dims, C, 4); }

int ggdt2d_signed(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                  int iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
                  hipStream_t stream) {
  const int dims[2] = {H, W};
  return signed_entry(2, dims, C, image, softmask, spacing, v, lambda, iterations, out, workspace, workspace_bytes,
                      stream);
}

int ggdt3d_signed(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                  int iterations, float* out, int C, int D, int H, int W, void* workspace, size_t workspace_bytes,
                  hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return signed_entry(3, dims, C, image, softmask, spacing, v, lambda, iterations, out, workspace, workspace_bytes,
                      stream);
}

int ggdt2d_gsf(const float* image, const float* softmask, const float* spacing, float theta_d, float theta_e,
               float v, float lambda, int iterations, float* out, int C, int H, int W, void* workspace,
               size_t workspace_bytes, hipStream_t stream) {
  const int dims[2] = {H, W};
  return gsf_entry(2, dims, C, image, softmask, spacing, theta_d, theta_e, v, lambda, iterations, out, workspace,
                   workspace_bytes, stream);
}

int ggdt3d_gsf(const float* image, const float* softmask, const float* spacing, float theta_d, float theta_e,
               float v, float lambda, int iterations, float* out, int C, int D, int H, int W, void* workspace,
               size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return gsf_entry(3, dims, C, image, softmask, spacing, theta_d, theta_e, v, lambda, iterations, out, workspace,
                   workspace_bytes, stream);
}

}  // extern "C"
