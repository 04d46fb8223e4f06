// Layout changes of a volume, device side: 64 x 64 tiles of a batched 2D
// transpose, dst[b][c][r] = src[b][r][c] (element (b, r, c) of src at
// b*sbs + r*srs + c, element (b, c, r) of dst at b*dbs + c*drs + r, r < R,
// c < Cc), moved through an LDS tile with one element of padding per row so
// that the column reads fall in distinct banks.  Called by every thread of a
// workgroup of NT threads (NT a multiple of 64); `tile` holds 64 x 65 elements.
#pragma once

#include <hip/hip_runtime.h>

namespace ggdt {
namespace dev {

constexpr int kTr = 64;
constexpr int kTrTileElems = kTr * (kTr + 1);  // elements of one LDS tile

// The two halves of a tile move: rows of src into the LDS tile, and rows of
// the transposed tile into dst; a workgroup barrier must separate them.
template <typename T, int NT>
__device__ __forceinline__ void transpose_load(const T* __restrict__ src, T* tile, int R, int Cc, long long srs,
                                               long long sbs, long long b, int r0, int c0) {
  static_assert(NT % kTr == 0, "whole 64-lane rows");
  const int tx = threadIdx.x & (kTr - 1), ty = threadIdx.x / kTr;
  const T* s = src + b * sbs;
#pragma unroll
  for (int i = ty; i < kTr; i += NT / kTr) {
    const int r = r0 + i, c = c0 + tx;
    if (r < R && c < Cc) tile[i * (kTr + 1) + tx] = s[(long long)r * srs + c];
  }
}

template <typename T, int NT>
__device__ __forceinline__ void transpose_store(T* __restrict__ dst, const T* tile, int R, int Cc, long long drs,
                                                long long dbs, long long b, int r0, int c0) {
  const int tx = threadIdx.x & (kTr - 1), ty = threadIdx.x / kTr;
  T* d = dst + b * dbs;
#pragma unroll
  for (int i = ty; i < kTr; i += NT / kTr) {
    const int c = c0 + i, r = r0 + tx;
    if (r < R && c < Cc) d[(long long)c * drs + r] = tile[tx * (kTr + 1) + i];
  }
}

template <typename T, int NT>
__device__ __forceinline__ void transpose_tile(const T* __restrict__ src, T* __restrict__ dst, T* tile, int R, int Cc,
                                               long long srs, long long sbs, long long drs, long long dbs,
                                               long long b, int r0, int c0) {
  transpose_load<T, NT>(src, tile, R, Cc, srs, sbs, b, r0, c0);
  __syncthreads();
  transpose_store<T, NT>(dst, tile, R, Cc, drs, dbs, b, r0, c0);
}

// Transpose parameters of the two layout changes of a [D0][D1][D2] volume:
// to_scan_major: [D0][D1][D2] -> [D2][D0][D1] (per z, the (y, x) slice into
// rows x of stride D0*D1 at offset z*D1); back: the inverse.
struct TransposeShape {
  int R, Cc, B;
  long long srs, sbs, drs, dbs;
};
__host__ __device__ inline TransposeShape transpose_shape(bool to_scan_major, int D0, int D1, int D2) {
  const long long s1 = D1, s12 = (long long)D1 * D2, s01 = (long long)D0 * D1;
  if (to_scan_major) return TransposeShape{D1, D2, D0, D2, s12, s01, s1};
  return TransposeShape{D2, D1, D0, s01, s1, D2, s12};
}

}  // namespace dev
}  // namespace ggdt
