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

namespace ggdt {
namespace {

constexpr int kTr = 64;  // tile side (one wave-wide row)

// dst[b][c][r] = src[b][r][c] for r < R, c < Cc, b < B: element (b, r, c) of
// src is at b*sbs + r*srs + c, element (b, c, r) of dst at b*dbs + c*drs + r.
// One workgroup of 256 threads moves a 64 x 64 tile: rows are read and written
// as whole 64-element runs; the LDS tile has one element of padding per row so
// that the column reads fall in distinct banks.  When `skip` is set (the
// fixed-point mode's done word), the launch does nothing.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, T* __restrict__ dst, int R,
                                                        int Cc, long long srs, long long sbs, long long drs,
                                                        long long dbs, int tiles_c, int tiles_r,
                                                        const unsigned* skip) {
  __shared__ T tile[kTr][kTr + 1];
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
  const long long id = blockIdx.x;
  const long long per_b = (long long)tiles_c * tiles_r;
  const long long b = id / per_b;
  const int t = (int)(id - b * per_b);
  const int r0 = (t / tiles_c) * kTr, c0 = (t % tiles_c) * kTr;
  const int tx = threadIdx.x & (kTr - 1), ty = threadIdx.x / kTr;
  const T* s = src + b * sbs;
  T* d = dst + b * dbs;
#pragma unroll
  for (int i = ty; i < kTr; i += 256 / kTr) {
    const int r = r0 + i, c = c0 + tx;
    if (r < R && c < Cc) tile[i][tx] = s[(long long)r * srs + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = ty; i < kTr; i += 256 / kTr) {
    const int c = c0 + i, r = r0 + tx;
    if (r < R && c < Cc) d[(long long)c * drs + r] = tile[tx][i];
  }
}

template <typename T>
hipError_t launch_t(const void* src, void* dst, int R, int Cc, int B, long long srs, long long sbs, long long drs,
                    long long dbs, const unsigned* skip, hipStream_t stream) {
  const int tc = (Cc + kTr - 1) / kTr, tr = (R + kTr - 1) / kTr;
  const long long blocks = (long long)tc * tr * B;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, stream, (const T*)src, (T*)dst, R,
                     Cc, srs, sbs, drs, dbs, tc, tr, skip);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_to_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                const unsigned* skip, hipStream_t stream) {
  // src [D0][D1][D2] -> dst [D2][D0][D1]: per z, the (y, x) slice transposed
  // into rows x of stride D0*D1 at offset z*D1.
  const long long s1 = D1, s12 = (long long)D1 * D2, s01 = (long long)D0 * D1;
  if (elem_bytes == 4) return launch_t<float>(src, dst, D1, D2, D0, D2, s12, s01, s1, skip, stream);
  if (elem_bytes == 2) return launch_t<uint16_t>(src, dst, D1, D2, D0, D2, s12, s01, s1, skip, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_from_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                  const unsigned* skip, hipStream_t stream) {
  // src [D2][D0][D1] -> dst [D0][D1][D2]: per z, the (x, y) slice at offset
  // z*D1 with row stride D0*D1 transposed into the (y, x) slice of dst.
  const long long s1 = D1, s12 = (long long)D1 * D2, s01 = (long long)D0 * D1;
  if (elem_bytes == 4) return launch_t<float>(src, dst, D2, D1, D0, s01, s1, D2, s12, skip, stream);
  if (elem_bytes == 2) return launch_t<uint16_t>(src, dst, D2, D1, D0, s01, s1, D2, s12, skip, stream);
  return hipErrorInvalidValue;
}

}  // namespace ggdt
