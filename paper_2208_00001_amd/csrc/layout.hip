// Layout changes of a volume: a batched 2D transpose through LDS.
//
// A pass along the contiguous memory axis of a C-order volume reads each
// voxel's planes as consecutive elements of one memory row, which the plane
// kernels can only gather by short runs.  The forward schedule therefore runs
// the two passes along the last axis of a single-channel volume on a copy laid
// out [W][D][H] (the scan axis slowest, H contiguous), where they are ordinary
// strided passes, and moves D into and out of that layout once per iteration.
// Moving values is exact, so the passes see the same numbers.
#include "ggdt_internal.h"
#include "layout.h"

namespace ggdt {
namespace {

using namespace dev;

// One workgroup of 256 threads per 64 x 64 tile.  When `skip` is set (the
// fixed-point mode's done word), the launch does nothing.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                        TransposeShape sh, int tiles_c, int tiles_r,
                                                        const unsigned* skip) {
  __shared__ T tile[kTr * (kTr + 1)];
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
  const long long id = blockIdx.x;
  const long long per_b = (long long)tiles_c * tiles_r;
  const long long b = id / per_b;
  const int t = (int)(id - b * per_b);
  transpose_tile<T, 256>(src, dst, tile, sh.R, sh.Cc, sh.srs, sh.sbs, sh.drs, sh.dbs, b, (t / tiles_c) * kTr,
                         (t % tiles_c) * kTr);
}

template <typename T>
hipError_t launch_t(const void* src, void* dst, const TransposeShape& sh, const unsigned* skip, hipStream_t stream) {
  const int tc = (sh.Cc + kTr - 1) / kTr, tr = (sh.R + kTr - 1) / kTr;
  const long long blocks = (long long)tc * tr * sh.B;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, stream, (const T*)src, (T*)dst, sh,
                     tc, tr, skip);
  return hipGetLastError();
}

hipError_t launch_layout(bool to_scan_major, const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                         const unsigned* skip, hipStream_t stream) {
  const TransposeShape sh = transpose_shape(to_scan_major, D0, D1, D2);
  if (elem_bytes == 4) return launch_t<float>(src, dst, sh, skip, stream);
  if (elem_bytes == 2) return launch_t<uint16_t>(src, dst, sh, skip, stream);
  if (elem_bytes == 1) return launch_t<uint8_t>(src, dst, sh, skip, stream);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_to_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                const unsigned* skip, hipStream_t stream) {
  return launch_layout(true, src, dst, elem_bytes, D0, D1, D2, skip, stream);
}

hipError_t launch_from_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                  const unsigned* skip, hipStream_t stream) {
  return launch_layout(false, src, dst, elem_bytes, D0, D1, D2, skip, stream);
}

}  // namespace ggdt
