// C ABI of the backward (single instance: one launch per reversed pass;
// batched: one persistent launch, tables built by ggdt_batched_plan).
#include <math.h>
#include <string.h>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "ggdt_internal.h"

namespace ggdt {

constexpr int kMaxBwdChannels = 8;

size_t bwd_workspace_for(const Problem& pr) {
  const size_t base = workspace_for(pr, Tuning{});
  return base + ((size_t)pr.N * 4 + 255) / 256 * 256;
}

// The scan-major area of the reverse (after bwd_workspace_for): the image,
// abar twice, dL/dI (fp32 volumes) and two passes' records (byte volumes).
size_t bwd_scan_major_bytes(const Problem& pr) {
  if (pr.ndim != 3 || pr.C != 1 || pr.dims[2] < 2) return 0;
  return 4 * scan_major_vol_bytes(pr) + 2 * (((size_t)pr.N + 255) / 256 * 256);
}

// Descriptor of the reverse of forward pass p; a_in / a_out / xbuf set by the caller.
int build_bwd_pass(const Problem& pr, const float* image, const uint8_t* records, const float* spacing, float lam,
                   float* gI, int p, int K, unsigned epoch_base, BwdDesc* d) {
  PassDesc f;
  const int rc = build_pass(pr, image, nullptr, spacing, 1.0f, lam, nullptr, nullptr, p, 0, &f);
  if (rc) return rc;
  memset(d, 0, sizeof *d);
  d->image = image;
  d->rec = records + (size_t)p * pr.N;
  d->gI = gI;
  d->N = (int)pr.N;
  d->sa = f.sa;
  d->sp = f.sp;
  d->sq = f.sq;
  d->Na = f.Na;
  d->Np = f.Np;
  d->Nq = f.Nq;
  d->sign = f.sign;
  d->C = pr.C;
  d->TP = f.TP;
  d->TQ = f.TQ;
  d->K = K;
  d->ntp = f.ntp;
  d->ntq = f.ntq;
  d->nchunk = (f.Na - 1 + K - 1) / K;
  d->mode = f.mode;
  d->sqrt_normal = f.sqrt_normal;
  d->lam = lam;
  for (int j = 0; j < 9; ++j) d->A[j] = f.A[j];
  d->epoch_base = epoch_base;
  d->a_in_off = -1;
  d->a_out_off = -1;
  d->op = kOpPass;
  d->lsrc_off = d->ldst_off = d->image_off = d->rec_off = d->gi_off = -1;
  return GGDT_OK;
}

namespace {

int backward_entry(int ndim, const int* dims, int C, const float* image, const uint8_t* records,
                   const float* grad_out, const float* spacing, float v, float lam, int iterations, float* grad_image,
                   float* grad_softmask, void* ws, size_t wsb, hipStream_t stream) {
  if (!image || !records || !grad_out || !grad_image || !grad_softmask || !ws || !dims) return GGDT_ERR_NULL_PTR;
  Problem pr;
  int rc = make_problem(ndim, dims, C, &pr);
  if (rc) return rc;
  if (C > kMaxBwdChannels) return GGDT_ERR_BAD_SHAPE;
  rc = check_params(ndim, spacing, v, lam, iterations);
  if (rc) return rc;
  if (wsb < bwd_workspace_for(pr)) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr.N * 4, ni = nb * C, nrec = (size_t)iterations * 2 * ndim * pr.N;
  {
    const void* ins[5] = {image, records, grad_out, ws, grad_softmask};
    const size_t nins[5] = {ni, nrec, nb, wsb, nb};
    if ((rc = check_alias(grad_image, ni, ins, nins, 5))) return rc;
    const void* ins2[4] = {image, records, grad_out, ws};
    const size_t nins2[4] = {ni, nrec, nb, wsb};
    if ((rc = check_alias(grad_softmask, nb, ins2, nins2, 4))) return rc;
  }
  if ((rc = check_device())) return rc;
  unsigned* words = (unsigned*)ws;
  const size_t fwd_ws = workspace_for(pr, Tuning{});
  unsigned long long* xbuf = (unsigned long long*)(words + kHeaderWords);
  float* scratch = (float*)((unsigned char*)ws + fwd_ws);
  if (launch_reset(words, (long long)(fwd_ws / 4), stream) != hipSuccess) return GGDT_ERR_HIP;
  if (launch_reset((unsigned*)grad_image, (long long)pr.N * C, stream) != hipSuccess) return GGDT_ERR_HIP;
  if (iterations == 0) return launch_scale(grad_out, v, grad_softmask, pr.N, stream) == hipSuccess ? GGDT_OK : GGDT_ERR_HIP;
  if (launch_classify(image, (long long)C * pr.N, words, stream) != hipSuccess) return GGDT_ERR_HIP;
  const int P = iterations * 2 * ndim;
  // Scan-major copies (as in the forward): the reverses of the passes along
  // the last axis of a single-channel volume run on [W][D][H] copies of the
  // image (moved once), of abar and dL/dI (moved there before each pair of
  // those reverse passes and back after it) and of the pair's records.
  const size_t smb = bwd_scan_major_bytes(pr), bmin = bwd_workspace_for(pr);
  const bool sm = smb > 0 && wsb >= bmin + smb;
  const int D0 = pr.dims[0], D1 = pr.dims[1], D2 = pr.dims[ndim - 1];
  float *s_img = nullptr, *s_a = nullptr, *s_b = nullptr, *s_g = nullptr;
  uint8_t* s_r[2] = {nullptr, nullptr};
  if (sm) {
    unsigned char* base_p = (unsigned char*)ws + bmin;
    const size_t vol = scan_major_vol_bytes(pr), vol1 = ((size_t)pr.N + 255) / 256 * 256;
    s_img = (float*)base_p;
    s_a = (float*)(base_p + vol);
    s_b = (float*)(base_p + 2 * vol);
    s_g = (float*)(base_p + 3 * vol);
    s_r[0] = base_p + 4 * vol;
    s_r[1] = base_p + 4 * vol + vol1;
    if (launch_to_scan_major(image, s_img, 4, D0, D1, D2, nullptr, stream) != hipSuccess) return GGDT_ERR_HIP;
  }
  unsigned base = 0;
  const float* a_in = grad_out;
  for (int q = 0; q < P; ++q) {
    const int p = P - 1 - q;
    const int k = p % (2 * ndim);
    const bool on_copy = sm && k >= 4;
    BwdDesc d;
    PassDesc g;
    pass_geometry(pr, (p % (2 * ndim)) / 2, &g);
    const int K = bwd_chunk_for(ndim, C, g.sa == 1 && !on_copy);
    if (K <= 0) return GGDT_ERR_UNSUPPORTED;
    if ((rc = build_bwd_pass(pr, image, records, spacing, lam, grad_image, p, K, base, &d))) return rc;
    float* a_out = ((P - 1 - q) % 2 == 0) ? grad_softmask : scratch;
    d.a_in = a_in;
    d.a_out = a_out;
    d.xbuf = xbuf;
    base += (unsigned)d.nchunk + 1u;
    if (sm && k == 5) {  // first of the pair (2, -), (2, +) in reverse order
      if (launch_to_scan_major(a_in, s_a, 4, D0, D1, D2, nullptr, stream) != hipSuccess ||
          launch_to_scan_major(grad_image, s_g, 4, D0, D1, D2, nullptr, stream) != hipSuccess ||
          launch_to_scan_major(records + (size_t)p * pr.N, s_r[0], 1, D0, D1, D2, nullptr, stream) != hipSuccess ||
          launch_to_scan_major(records + (size_t)(p - 1) * pr.N, s_r[1], 1, D0, D1, D2, nullptr, stream) !=
              hipSuccess)
        return GGDT_ERR_HIP;
    }
    if (on_copy) {
      // planes (z, y) of the [W][D][H] copies: same tiles, offsets and constants
      d.sa = D0 * D1;
      d.sp = D1;
      d.sq = 1;
      d.image = s_img;
      d.rec = s_r[k == 5 ? 0 : 1];
      d.gI = s_g;
      d.a_in = k == 5 ? s_a : s_b;
      d.a_out = k == 5 ? s_b : s_a;
    }
    prof_before(stream);
    const hipError_t e = launch_bwd_pass(d, ndim, words, g_spin_limit, stream);
    prof_after(stream);
    if (e != hipSuccess) return GGDT_ERR_HIP;
    if (sm && k == 4) {  // abar and dL/dI back to the array layout
      if (launch_from_scan_major(s_a, a_out, 4, D0, D1, D2, nullptr, stream) != hipSuccess ||
          launch_from_scan_major(s_g, grad_image, 4, D0, D1, D2, nullptr, stream) != hipSuccess)
        return GGDT_ERR_HIP;
    }
    a_in = a_out;
  }
  // the last reversed pass wrote grad_softmask: dL/dM = v * abar
  return launch_scale(grad_softmask, v, grad_softmask, pr.N, stream) == hipSuccess ? GGDT_OK : GGDT_ERR_HIP;
}

}  // namespace
}  // namespace ggdt

using namespace ggdt;

extern "C" {

size_t ggdt_backward_workspace_bytes(int ndim, const int* dims, int C) {
  if (!dims) return 0;
  Problem pr;
  if (make_problem(ndim, dims, C, &pr) || C > kMaxBwdChannels) return 0;
  return bwd_workspace_for(pr) + bwd_scan_major_bytes(pr);
}

size_t ggdt_backward_workspace_min_bytes(int ndim, const int* dims, int C) {
  if (!dims) return 0;
  Problem pr;
  if (make_problem(ndim, dims, C, &pr) || C > kMaxBwdChannels) return 0;
  return bwd_workspace_for(pr);
}

int ggdt2d_backward(const float* image, const uint8_t* records, const float* grad_out, const float* spacing, float v,
                    float lambda, int iterations, float* grad_image, float* grad_softmask, int C, int H, int W,
                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
  const int dims[2] = {H, W};
  return backward_entry(2, dims, C, image, records, grad_out, spacing, v, lambda, iterations, grad_image,
                        grad_softmask, workspace, workspace_bytes, stream);
}

int ggdt3d_backward(const float* image, const uint8_t* records, const float* grad_out, const float* spacing, float v,
                    float lambda, int iterations, float* grad_image, float* grad_softmask, int C, int D, int H, int W,
                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return backward_entry(3, dims, C, image, records, grad_out, spacing, v, lambda, iterations, grad_image,
                        grad_softmask, workspace, workspace_bytes, stream);
}

}  // extern "C"
