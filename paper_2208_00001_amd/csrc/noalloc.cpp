// The 3D forward for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid it): the
// caller passes inputs and the output only, and the inter-workgroup scratch
// that ggdt3d takes as a workspace lives in a fixed device array instead.
//
// The array is file-scope device memory of GGDT_NOALLOC_SCRATCH_BYTES, one
// copy per GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): on the first call on a device, with that device current, its
// device address is looked up once and kept per device, and that address goes
// to the kernels exactly like a caller's workspace.  Every call on a GPU shares
// that GPU's array: the schedule clears the header and the exchange words it
// uses with a reset kernel first (no memset), and calls that overlap in time
// on one GPU race.
#include <mutex>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "ggdt_internal.h"

namespace ggdt {

constexpr size_t kScratchBytes = GGDT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's scratch array (looked up once per device).
int scratch_address(void** addr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GGDT_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GGDT_ERR_HIP;
    g_scratch_addr[dev] = p;
  }
  *addr = g_scratch_addr[dev];
  return GGDT_OK;
}

}  // namespace
}  // namespace ggdt

using namespace ggdt;

extern "C" int ggdt3d_noalloc(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                              int iterations, float* out, int C, int D, int H, int W, hipStream_t stream) {
  if (!image || !softmask || !out) return GGDT_ERR_NULL_PTR;
  const int dims[3] = {D, H, W};
  Problem pr;
  int rc = make_problem(3, dims, C, &pr);
  if (rc) return rc;
  rc = check_params(3, spacing, v, lambda, iterations);
  if (rc) return rc;
  const Tuning tu{};
  if (workspace_for(pr, tu) > kScratchBytes) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  const size_t nb = (size_t)pr.N * 4, ni = (size_t)pr.N * pr.C * 4;
  const void* ins[2] = {image, softmask};
  const size_t nins[2] = {ni, nb};
  rc = check_alias(out, nb, ins, nins, 2);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return enqueue_forward(pr, image, softmask, spacing, v, lambda, iterations, out, nullptr, ws, tu, stream);
}
