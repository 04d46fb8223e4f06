// C ABI of the GGDT library: argument validation, per-pass parameter preparation
// (edge-constant table) and the pass schedule.  Every step of the transform runs
// in the HIP kernels; this file only prepares launches.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "ggdt_internal.h"

namespace ggdt {

unsigned long long g_spin_limit = kDefaultSpinLimit;

namespace {
hipEvent_t* g_prof_events = nullptr;
int g_prof_cap = 0;
int g_prof_used = 0;
}  // namespace

namespace {
bool g_prof_open = false;
}

void prof_before(hipStream_t stream) {
  g_prof_open = g_prof_events && g_prof_used < g_prof_cap;
  if (g_prof_open) (void)hipEventRecord(g_prof_events[2 * g_prof_used], stream);
}

void prof_after(hipStream_t stream) {
  if (g_prof_open) (void)hipEventRecord(g_prof_events[2 * g_prof_used++ + 1], stream);
  g_prof_open = false;
}

hipError_t launch_pass_profiled(const PassDesc& d, int ndim, unsigned* words, hipStream_t stream) {
  prof_before(stream);
  const hipError_t e = launch_pass(d, ndim, words, g_spin_limit, stream);
  prof_after(stream);
  return e;
}

const char* status_text(int status) {
  switch (status) {
    case GGDT_OK: return "ok";
    case GGDT_ERR_NULL_PTR: return "a required pointer is NULL";
    case GGDT_ERR_BAD_SHAPE: return "invalid shape (ndim, C or a dimension out of range, or size overflow)";
    case GGDT_ERR_BAD_PARAM: return "invalid parameter (v, lambda, spacing or iterations outside the domain)";
    case GGDT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case GGDT_ERR_HIP: return "HIP runtime error";
    case GGDT_ERR_WATCHDOG: return "an inter-workgroup wait expired (watchdog)";
    case GGDT_ERR_ALIAS: return "an output overlaps an input";
    case GGDT_ERR_UNSUPPORTED: return "unsupported request or device (needs gfx950)";
    default: return "unknown status";
  }
}

int check_device() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return GGDT_ERR_HIP;
  if (cached[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GGDT_ERR_HIP;
    cached[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  return cached[dev] == 1 ? GGDT_OK : GGDT_ERR_UNSUPPORTED;
}

int make_problem(int ndim, const int* dims, int C, Problem* pr) {
  if (ndim != 2 && ndim != 3) return GGDT_ERR_BAD_SHAPE;
  if (C < 1 || C > kMaxChannels) return GGDT_ERR_BAD_SHAPE;
  long long n = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1) return GGDT_ERR_BAD_SHAPE;
    n *= dims[i];
    if (n > 0x7fffffffLL) return GGDT_ERR_BAD_SHAPE;
  }
  if (n * C > (1LL << 40)) return GGDT_ERR_BAD_SHAPE;
  pr->ndim = ndim;
  pr->C = C;
  pr->N = n;
  for (int i = 0; i < 3; ++i) pr->dims[i] = i < ndim ? dims[i] : 1;
  return GGDT_OK;
}

int check_params(int ndim, const float* spacing, float v, float lam, int iterations) {
  if (!spacing) return GGDT_ERR_NULL_PTR;
  if (!(isfinite(v) && v >= 0.0f)) return GGDT_ERR_BAD_PARAM;
  if (!(lam >= 0.0f && lam <= 1.0f)) return GGDT_ERR_BAD_PARAM;
  if (iterations < 0) return GGDT_ERR_BAD_PARAM;
  for (int b = 0; b < ndim; ++b)
    if (!(isfinite(spacing[b]) && spacing[b] > 0.0f)) return GGDT_ERR_BAD_PARAM;
  return GGDT_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

int check_alias(const void* out, size_t nout, const void* const* ins, const size_t* nins, int nin) {
  for (int i = 0; i < nin; ++i)
    if (overlaps(out, nout, ins[i], nins[i])) return GGDT_ERR_ALIAS;
  return GGDT_OK;
}

void tile_shape(const Problem& pr, const Tuning& tu, int* TP, int* TQ) {
  (void)tu;
  if (pr.ndim == 3) {
    *TP = kTileP3;
    *TQ = kTileQ3;
  } else {
    *TP = 1;
    *TQ = kTileQ2;
  }
}

// Geometry of a pass along `axis`: p, q are the non-scan axes in ascending order.
void pass_geometry(const Problem& pr, int axis, PassDesc* d) {
  long long stride[3];
  stride[pr.ndim - 1] = 1;
  for (int b = pr.ndim - 2; b >= 0; --b) stride[b] = stride[b + 1] * pr.dims[b + 1];
  int other[2], no = 0;
  for (int b = 0; b < pr.ndim; ++b)
    if (b != axis) other[no++] = b;
  d->Na = pr.dims[axis];
  d->sa = (int)stride[axis];
  if (pr.ndim == 3) {
    d->Np = pr.dims[other[0]];
    d->sp = (int)stride[other[0]];
    d->Nq = pr.dims[other[1]];
    d->sq = (int)stride[other[1]];
  } else {
    d->Np = 1;
    d->sp = 0;
    d->Nq = pr.dims[other[0]];
    d->sq = (int)stride[other[0]];
  }
}

// Edge constants of a pass along `axis`: A_j = (float)((1 - lambda) * S_j) with
// S_j = sum over axes b ascending of (s_b * |dx_b|)^2 in double, where the offset
// j has |dx| = 1 on the scan axis and (delta_p, delta_q) on the others.
void edge_constants(const Problem& pr, int axis, const float* spacing, float lam, float* A, float* W0) {
  int other[2], no = 0;
  for (int b = 0; b < pr.ndim; ++b)
    if (b != axis) other[no++] = b;
  const int nj = pr.ndim == 3 ? 9 : 3;
  for (int j = 0; j < 9; ++j) {
    A[j] = 0.0f;
    W0[j] = 0.0f;
  }
  for (int j = 0; j < nj; ++j) {
    int dx[3] = {0, 0, 0};
    dx[axis] = 1;
    if (pr.ndim == 3) {
      dx[other[0]] = j / 3 - 1;
      dx[other[1]] = j % 3 - 1;
    } else {
      dx[other[0]] = j - 1;
    }
    double S = 0.0;
    for (int b = 0; b < pr.ndim; ++b) {
      const double t = (double)spacing[b] * (double)abs(dx[b]);
      S = S + t * t;
    }
    A[j] = (float)((1.0 - (double)lam) * S);
    W0[j] = sqrtf(A[j]);
  }
}

// When the general edge cost's root argument fmaf(lambda, g, A_j) over the n
// candidates' constants lies in the normal range that sqrt_rn_normal handles:
// always when every A_j >= 2^-96 (it is at least A_j; finite image values are
// checked on the device), and for lambda 1 (every A_j = 0, the argument is g)
// when the device finds no small or huge image value.
int sqrt_normal_for(const float* A, int n) {
  float amin = A[0], amax = A[0];
  for (int j = 1; j < n; ++j) {
    amin = A[j] < amin ? A[j] : amin;
    amax = A[j] > amax ? A[j] : amax;
  }
  if (amin >= 0x1p-96f) return kSqrtNormalUnlessHuge;
  return amax == 0.0f ? kSqrtNormalLam1 : kSqrtNormalNever;
}

int requested_mode(float lam, int C) {
  if (lam == 0.0f) return kModeLam0;
  if (lam == 1.0f && C == 1) return kModeLam1C1;
  return kModeGeneral;
}

int max_tiles(const Problem& pr, const Tuning& tu) {
  int TP, TQ;
  tile_shape(pr, tu, &TP, &TQ);
  int best = 1;
  for (int a = 0; a < pr.ndim; ++a) {
    PassDesc d;
    pass_geometry(pr, a, &d);
    const int nt = ((d.Np + TP - 1) / TP) * ((d.Nq + TQ - 1) / TQ);
    if (nt > best) best = nt;
  }
  return best;
}

// Header, then the exchange words: two parity slots of one word per tile cell.
size_t workspace_for(const Problem& pr, const Tuning& tu) {
  int TP, TQ;
  tile_shape(pr, tu, &TP, &TQ);
  const size_t xbuf = ((size_t)2 * max_tiles(pr, tu) * TP * TQ * 8 + 255) / 256 * 256;
  return (size_t)kHeaderWords * 4 + xbuf;
}

// Bytes of one scan-major fp32 volume, and of the scan-major area of a
// forward (D, then the image, then one pass's records, each 256-byte aligned)
// through which the passes along the last axis of a single-channel volume run
// as strided passes; 0 where the forward keeps those passes in place.
size_t scan_major_vol_bytes(const Problem& pr) { return ((size_t)pr.N * 4 + 255) / 256 * 256; }

size_t scan_major_bytes(const Problem& pr) {
  if (pr.ndim != 3 || pr.C != 1 || pr.dims[2] < 2) return 0;
  return 2 * scan_major_vol_bytes(pr) + ((size_t)pr.N + 255) / 256 * 256;
}

// The pass along axis 2 on the scan-major copies ([W][D][H]: the scan axis
// slowest, H contiguous).  The plane axes keep their order (p = axis 0, q =
// axis 1), so tiles, offsets j and edge constants are those of the pass on the
// C-order volume.
static void use_scan_major(const Problem& pr, const void* image_t, float* d_t, PassDesc* d) {
  d->sa = pr.dims[0] * pr.dims[1];
  d->sp = pr.dims[1];
  d->sq = 1;
  d->image = static_cast<const float*>(image_t);
  d->D = d_t;
  d->K = pass_chunk_for(pr.ndim, pr.C, d->sa == 1);
  d->nchunk = (d->Na - 1 + d->K - 1) / d->K;
}

// 2D passes of images with up to kRowMaxC channels run on the row kernel
// (one wave per 32-cell tile, chunks of 16 rows).  Its exchange area,
// ceil(Nq / 32) * 32 words per parity, fits in the tile kernel's.
static void use_row_geometry(const Problem& pr, PassDesc* d) {
  if (pr.ndim != 2 || pr.C > kRowMaxC) return;
  d->TP = 1;
  d->TQ = kRowTQ;
  d->K = kRowK;
  d->ntp = 1;
  d->ntq = (d->Nq + kRowTQ - 1) / kRowTQ;
  d->nchunk = (d->Na - 1 + kRowK - 1) / kRowK;
}

// Enqueue the whole forward schedule of one instance.
int enqueue_forward(const Problem& pr, const float* image, const float* mask, const float* spacing, float v,
                    float lam, int iterations, float* out, uint8_t* records, void* ws, const Tuning& tu,
                    hipStream_t stream, int img_fmt, void* scan_major) {
  unsigned* words = (unsigned*)ws;
  unsigned long long* xbuf = (unsigned long long*)(words + kHeaderWords);
  const long long nwords = (long long)(workspace_for(pr, tu) / 4);
  if (launch_reset(words, nwords, stream) != hipSuccess) return GGDT_ERR_HIP;
  if (iterations == 0) {
    if (launch_scale(mask, v, out, pr.N, stream) != hipSuccess) return GGDT_ERR_HIP;
    return GGDT_OK;
  }
  // The image classification decides every pass's edge-cost mode on the device.
  if (launch_classify(image, (long long)pr.C * pr.N, words, stream, img_fmt) != hipSuccess) return GGDT_ERR_HIP;
  const ScanMajor sm = scan_major_for(pr, records, scan_major);
  const int esz = img_fmt == kImgF32 ? 4 : 2;
  if (sm.on && launch_to_scan_major(image, sm.image, esz, pr.dims[0], pr.dims[1], pr.dims[2], nullptr, stream) !=
                   hipSuccess)
    return GGDT_ERR_HIP;
  unsigned base = 0;
  const int npass = iterations * 2 * pr.ndim;
  for (int p = 0; p < npass; ++p) {
    PassDesc d;
    const int rc = build_pass(pr, image, mask, spacing, v, lam, out, records, p, base, &d);
    if (rc) return rc;
    d.img_fmt = img_fmt;
    use_row_geometry(pr, &d);
    d.xbuf = xbuf;
    base += (unsigned)d.nchunk + 1u;
    const int k = p % (2 * pr.ndim);
    uint8_t* rec_c = d.rec;  // this pass's records in the array layout
    if (sm.on && k >= 4) {
      use_scan_major(pr, sm.image, sm.D, &d);
      if (rec_c) d.rec = sm.rec;  // written scan-major, moved to the array layout below
    }
    if (sm.on && k == 4 &&
        launch_to_scan_major(out, sm.D, 4, pr.dims[0], pr.dims[1], pr.dims[2], nullptr, stream) != hipSuccess)
      return GGDT_ERR_HIP;
    if (launch_pass_profiled(d, pr.ndim, words, stream) != hipSuccess) return GGDT_ERR_HIP;
    if (sm.on && k >= 4 && rec_c &&
        launch_from_scan_major(sm.rec, rec_c, 1, pr.dims[0], pr.dims[1], pr.dims[2], nullptr, stream) != hipSuccess)
      return GGDT_ERR_HIP;
    if (sm.on && k == 5 &&
        launch_from_scan_major(sm.D, out, 4, pr.dims[0], pr.dims[1], pr.dims[2], nullptr, stream) != hipSuccess)
      return GGDT_ERR_HIP;
  }
  (void)tu;
  return GGDT_OK;
}

ScanMajor scan_major_for(const Problem& pr, const uint8_t* records, void* buf) {
  ScanMajor sm{};
  (void)records;  // records of scan-major passes are staged and moved to the array layout
  if (!buf || scan_major_bytes(pr) == 0) return sm;
  sm.on = true;
  sm.D = static_cast<float*>(buf);
  sm.image = static_cast<unsigned char*>(buf) + scan_major_vol_bytes(pr);
  sm.rec = static_cast<uint8_t*>(buf) + 2 * scan_major_vol_bytes(pr);
  return sm;
}

int build_pass(const Problem& pr, const float* image, const float* mask, const float* spacing, float v, float lam,
               float* out, uint8_t* records, int p, unsigned epoch_base, PassDesc* d) {
  const int a = (p % (2 * pr.ndim)) / 2;
  const int TP = pr.ndim == 3 ? kTileP3 : 1;
  const int TQ = pr.ndim == 3 ? kTileQ3 : kTileQ2;
  memset(d, 0, sizeof *d);
  pass_geometry(pr, a, d);
  edge_constants(pr, a, spacing, lam, d->A, d->W0);
  const int K = pass_chunk_for(pr.ndim, pr.C, d->sa == 1);
  if (K <= 0) return GGDT_ERR_UNSUPPORTED;
  d->image = image;
  d->mask = mask;
  d->D = out;
  d->xbuf = nullptr;
  d->N = (int)pr.N;
  d->C = pr.C;
  d->TP = TP;
  d->TQ = TQ;
  d->K = K;
  d->ntp = (d->Np + TP - 1) / TP;
  d->ntq = (d->Nq + TQ - 1) / TQ;
  d->nchunk = (d->Na - 1 + K - 1) / K;
  d->mode = requested_mode(lam, pr.C);
  d->v = v;
  d->lam = lam;
  d->sign = (p % 2 == 0) ? 1 : -1;
  d->init = p == 0 ? 1 : 0;
  d->rec = records ? records + (size_t)p * pr.N : nullptr;
  d->epoch_base = epoch_base;
  d->sqrt_normal = sqrt_normal_for(d->A, pr.ndim == 3 ? 9 : 3);
  d->op = kOpPass;
  d->esz = 4;
  d->image_off = d->d_off = d->rec_off = -1;
  return GGDT_OK;
}

// Convergence mode: up to max_iterations whole iterations, each followed by the
// iteration-end kernel; passes after a no-change iteration return at once.
// Iterations are enqueued in blocks (4, 4, 8, 16, ... iterations); after each
// block the stream is synchronised and the done word read, so that at most one
// block of no-op iterations follows the fixed point.
int converge_entry(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
                   float v, float lam, int max_iterations, float* out, void* ws, size_t wsb, hipStream_t stream) {
  if (!image || !mask || !out || !ws || !dims) return GGDT_ERR_NULL_PTR;
  Problem pr;
  int rc = make_problem(ndim, dims, C, &pr);
  if (rc) return rc;
  rc = check_params(ndim, spacing, v, lam, max_iterations);
  if (rc) return rc;
  const Tuning tu{};
  if (wsb < workspace_for(pr, tu)) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr.N * 4, ni = (size_t)pr.N * pr.C * 4;
  const void* ins[3] = {image, mask, ws};
  const size_t nins[3] = {ni, nb, wsb};
  rc = check_alias(out, nb, ins, nins, 3);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  unsigned* words = (unsigned*)ws;
  unsigned long long* xbuf = (unsigned long long*)(words + kHeaderWords);
  if (launch_reset(words, (long long)(workspace_for(pr, tu) / 4), stream) != hipSuccess) return GGDT_ERR_HIP;
  if (max_iterations == 0) return launch_scale(mask, v, out, pr.N, stream) == hipSuccess ? GGDT_OK : GGDT_ERR_HIP;
  if (launch_classify(image, (long long)pr.C * pr.N, words, stream) != hipSuccess) return GGDT_ERR_HIP;
  const ScanMajor sm = scan_major_for(pr, nullptr, scan_major_in(pr, tu, ws, wsb));
  if (sm.on && launch_to_scan_major(image, sm.image, 4, pr.dims[0], pr.dims[1], pr.dims[2], nullptr, stream) !=
                   hipSuccess)
    return GGDT_ERR_HIP;
  unsigned base = 0;
  const int per = 2 * pr.ndim;
  int block = 4;
  for (int it = 1; it <= max_iterations;) {
    const int last = it + block - 1 < max_iterations ? it + block - 1 : max_iterations;
    for (; it <= last; ++it) {
      for (int k = 0; k < per; ++k) {
        PassDesc d;
        rc = build_pass(pr, image, mask, spacing, v, lam, out, nullptr, (it - 1) * per + k, base, &d);
        if (rc) return rc;
        use_row_geometry(pr, &d);
        d.xbuf = xbuf;
        d.converge = 1;
        base += (unsigned)d.nchunk + 1u;
        // the layout changes do nothing once the done word is set, as the passes
        if (sm.on && k >= 4) use_scan_major(pr, sm.image, sm.D, &d);
        if (sm.on && k == 4 &&
            launch_to_scan_major(out, sm.D, 4, pr.dims[0], pr.dims[1], pr.dims[2], words + kWordDone, stream) !=
                hipSuccess)
          return GGDT_ERR_HIP;
        if (launch_pass_profiled(d, pr.ndim, words, stream) != hipSuccess) return GGDT_ERR_HIP;
        if (sm.on && k == 5 &&
            launch_from_scan_major(sm.D, out, 4, pr.dims[0], pr.dims[1], pr.dims[2], words + kWordDone, stream) !=
                hipSuccess)
          return GGDT_ERR_HIP;
      }
      if (launch_iteration_end(words, it, stream) != hipSuccess) return GGDT_ERR_HIP;
    }
    if (it > max_iterations) break;
    unsigned w[kWordDone + 1] = {0};
    if (hipMemcpyAsync(w, words, sizeof w, hipMemcpyDeviceToHost, stream) != hipSuccess) return GGDT_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GGDT_ERR_HIP;
    if (w[kWordDone] || w[kWordAbort]) break;
    if (it > 5) block *= 2;
  }
  return GGDT_OK;
}

int forward_entry(int ndim, const int* dims, int C, const float* image, const float* mask, const float* spacing,
                  float v, float lam, int iterations, float* out, uint8_t* records, bool want_records, void* ws,
                  size_t wsb, hipStream_t stream, int img_fmt = kImgF32) {
  if (!image || !mask || !out || !ws || !dims) return GGDT_ERR_NULL_PTR;
  if (want_records && !records) return GGDT_ERR_NULL_PTR;
  Problem pr;
  int rc = make_problem(ndim, dims, C, &pr);
  if (rc) return rc;
  rc = check_params(ndim, spacing, v, lam, iterations);
  if (rc) return rc;
  if (img_fmt != kImgF32) {
    if (img_fmt != kImgBF16 && img_fmt != kImgF16) return GGDT_ERR_BAD_PARAM;
    // kernels that read 16-bit images: single-channel volumes, images of up to kRowMaxC channels
    if ((ndim == 3 && C != 1) || (ndim == 2 && C > kRowMaxC) || want_records) return GGDT_ERR_UNSUPPORTED;
  }
  const Tuning tu{};
  if (wsb < workspace_for(pr, tu)) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr.N * 4, ni = (size_t)pr.N * pr.C * (img_fmt == kImgF32 ? 4 : 2);
  const size_t nrec = want_records ? (size_t)iterations * 2 * ndim * pr.N : 0;
  const void* ins[3] = {image, mask, ws};
  const size_t nins[3] = {ni, nb, wsb};
  rc = check_alias(out, nb, ins, nins, 3);
  if (rc) return rc;
  if (want_records) {
    const void* ins2[4] = {image, mask, ws, out};
    const size_t nins2[4] = {ni, nb, wsb, nb};
    rc = check_alias(records, nrec, ins2, nins2, 4);
    if (rc) return rc;
  }
  rc = check_device();
  if (rc) return rc;
  return enqueue_forward(pr, image, mask, spacing, v, lam, iterations, out, want_records ? records : nullptr, ws,
                         tu, stream, img_fmt, scan_major_in(pr, tu, ws, wsb));
}

void* scan_major_in(const Problem& pr, const Tuning& tu, void* ws, size_t wsb) {
  const size_t base = workspace_for(pr, tu), extra = scan_major_bytes(pr);
  if (extra == 0 || wsb < base + extra) return nullptr;
  return static_cast<unsigned char*>(ws) + base;
}

}  // namespace ggdt

using namespace ggdt;

extern "C" {

const char* ggdt_strerror(int status) { return status_text(status); }

size_t ggdt_workspace_bytes(int ndim, const int* dims, int C) {
  if (!dims) return 0;
  Problem pr;
  if (make_problem(ndim, dims, C, &pr)) return 0;
  return workspace_for(pr, Tuning{}) + scan_major_bytes(pr);
}

size_t ggdt_workspace_min_bytes(int ndim, const int* dims, int C) {
  if (!dims) return 0;
  Problem pr;
  if (make_problem(ndim, dims, C, &pr)) return 0;
  return workspace_for(pr, Tuning{});
}

size_t ggdt_records_bytes(int ndim, const int* dims, int iterations) {
  if (!dims || iterations < 0) return 0;
  Problem pr;
  if (make_problem(ndim, dims, 1, &pr)) return 0;
  return (size_t)iterations * 2 * ndim * (size_t)pr.N;
}

int ggdt2d(const float* image, const float* softmask, const float* spacing, float v, float lambda, int iterations,
           float* out, int C, int H, int W, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  const int dims[2] = {H, W};
  return forward_entry(2, dims, C, image, softmask, spacing, v, lambda, iterations, out, nullptr, false, workspace,
                       workspace_bytes, stream);
}

int ggdt3d(const float* image, const float* softmask, const float* spacing, float v, float lambda, int iterations,
           float* out, int C, int D, int H, int W, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return forward_entry(3, dims, C, image, softmask, spacing, v, lambda, iterations, out, nullptr, false, workspace,
                       workspace_bytes, stream);
}

int ggdt2d_half(const uint16_t* image, int format, const float* softmask, const float* spacing, float v,
                float lambda, int iterations, float* out, int C, int H, int W, void* workspace,
                size_t workspace_bytes, hipStream_t stream) {
  const int dims[2] = {H, W};
  if (format != GGDT_IMAGE_BF16 && format != GGDT_IMAGE_F16) return GGDT_ERR_BAD_PARAM;
  return forward_entry(2, dims, C, reinterpret_cast<const float*>(image), softmask, spacing, v, lambda, iterations,
                       out, nullptr, false, workspace, workspace_bytes, stream,
                       format == GGDT_IMAGE_BF16 ? kImgBF16 : kImgF16);
}

int ggdt3d_half(const uint16_t* image, int format, const float* softmask, const float* spacing, float v,
                float lambda, int iterations, float* out, int C, int D, int H, int W, void* workspace,
                size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  if (format != GGDT_IMAGE_BF16 && format != GGDT_IMAGE_F16) return GGDT_ERR_BAD_PARAM;
  return forward_entry(3, dims, C, reinterpret_cast<const float*>(image), softmask, spacing, v, lambda, iterations,
                       out, nullptr, false, workspace, workspace_bytes, stream,
                       format == GGDT_IMAGE_BF16 ? kImgBF16 : kImgF16);
}

int ggdt2d_forward_rec(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                       int iterations, float* out, uint8_t* records, int C, int H, int W, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  const int dims[2] = {H, W};
  return forward_entry(2, dims, C, image, softmask, spacing, v, lambda, iterations, out, records, true, workspace,
                       workspace_bytes, stream);
}

int ggdt3d_forward_rec(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                       int iterations, float* out, uint8_t* records, int C, int D, int H, int W, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return forward_entry(3, dims, C, image, softmask, spacing, v, lambda, iterations, out, records, true, workspace,
                       workspace_bytes, stream);
}

int ggdt2d_converge(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int max_iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
  const int dims[2] = {H, W};
  return converge_entry(2, dims, C, image, softmask, spacing, v, lambda, max_iterations, out, workspace,
                        workspace_bytes, stream);
}

int ggdt3d_converge(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int max_iterations, float* out, int C, int D, int H, int W, void* workspace,
                    size_t workspace_bytes, hipStream_t stream) {
  const int dims[3] = {D, H, W};
  return converge_entry(3, dims, C, image, softmask, spacing, v, lambda, max_iterations, out, workspace,
                        workspace_bytes, stream);
}

int ggdt_workspace_iterations(const void* workspace, hipStream_t stream, int* iterations) {
  if (!workspace || !iterations) return GGDT_ERR_NULL_PTR;
  if (hipStreamSynchronize(stream) != hipSuccess) return GGDT_ERR_HIP;
  unsigned w[kWordIters + 1] = {0};
  if (hipMemcpy(w, workspace, sizeof w, hipMemcpyDeviceToHost) != hipSuccess) return GGDT_ERR_HIP;
  if (w[kWordAbort]) return GGDT_ERR_WATCHDOG;
  *iterations = w[kWordDone] ? (int)w[kWordIters] : -1;
  return GGDT_OK;
}

int ggdt_workspace_status(const void* workspace, hipStream_t stream) {
  if (!workspace) return GGDT_ERR_NULL_PTR;
  if (hipStreamSynchronize(stream) != hipSuccess) return GGDT_ERR_HIP;
  unsigned word = 0;
  if (hipMemcpy(&word, workspace, sizeof word, hipMemcpyDeviceToHost) != hipSuccess) return GGDT_ERR_HIP;
  return word ? GGDT_ERR_WATCHDOG : GGDT_OK;
}

void ggdt_set_spin_limit(unsigned long long polls) { g_spin_limit = polls ? polls : kDefaultSpinLimit; }

static void profile_free() {
  if (g_prof_events) {
    for (int i = 0; i < 2 * g_prof_cap; ++i) hipEventDestroy(g_prof_events[i]);
    free(g_prof_events);
  }
  g_prof_events = nullptr;
  g_prof_cap = 0;
  g_prof_used = 0;
}

int ggdt_profile_begin(int n) {
  profile_free();
  if (n <= 0) return GGDT_ERR_BAD_PARAM;
  hipEvent_t* ev = (hipEvent_t*)calloc((size_t)2 * n, sizeof(hipEvent_t));
  if (!ev) return GGDT_ERR_HIP;
  for (int i = 0; i < 2 * n; ++i) {
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(ev[j]);
      free(ev);
      return GGDT_ERR_HIP;
    }
  }
  g_prof_events = ev;
  g_prof_cap = n;
  g_prof_used = 0;
  return GGDT_OK;
}

int ggdt_profile_end(float* ms, int capacity) {
  if (!g_prof_events) return 0;
  const int used = g_prof_used;
  int rc = used;
  for (int i = 0; i < used; ++i) {
    if (hipEventSynchronize(g_prof_events[2 * i + 1]) != hipSuccess) {
      rc = GGDT_ERR_HIP;
      break;
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, g_prof_events[2 * i], g_prof_events[2 * i + 1]) != hipSuccess) {
      rc = GGDT_ERR_HIP;
      break;
    }
    if (ms && i < capacity) ms[i] = t;
  }
  profile_free();
  return rc;
}

}  // extern "C"
