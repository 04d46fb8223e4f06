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

// A whole layout change spread over the G workgroups of a persistent launch
// (this one is number wg), by rounds of KT consecutive tiles.  Every load of a
// round is issued before any LDS write (unconditionally, from addresses
// clamped into the volume; LDS slots of clamped loads are never read back), so
// a round waits for one memory round trip.  `tiles` holds KT LDS tiles.
template <typename T, int NT, int KT>
__device__ void layout_rounds(const T* src_p, T* dst_p, const TransposeShape& sh, T* tiles, int wg, int G) {
  constexpr int RPT = kTr / (NT / kTr);  // rows of a tile per thread
  const int tx = threadIdx.x & (kTr - 1), ty = threadIdx.x / kTr;
  // tiles are numbered b-major, then tile row, then tile column (fewer than
  // 2^31: the volume has fewer elements); a round's tiles are consecutive, so
  // their coordinates follow from the first one's by counting
  const int tc = (sh.Cc + kTr - 1) / kTr, tr = (sh.R + kTr - 1) / kTr;
  const int per_b = tc * tr, total = per_b * sh.B;
  const __attribute__((address_space(1))) T* src = (const __attribute__((address_space(1))) T*)src_p;
  __attribute__((address_space(1))) T* dst = (__attribute__((address_space(1))) T*)dst_p;
  for (int id0 = wg * KT; id0 < total; id0 += G * KT) {
    const int n = total - id0 < KT ? total - id0 : KT;
    int b[KT], r0[KT], c0[KT];
    {
      int bb = id0 / per_b;
      const int rem = id0 - bb * per_b;
      int trw = rem / tc, tcl = rem - trw * tc;
#pragma unroll
      for (int u = 0; u < KT; ++u) {
        b[u] = bb;
        r0[u] = trw * kTr;
        c0[u] = tcl * kTr;
        if (++tcl == tc) {
          tcl = 0;
          if (++trw == tr) {
            trw = 0;
            ++bb;
          }
        }
      }
    }
    T v[KT][RPT];
#pragma unroll
    for (int u = 0; u < KT; ++u) {
      const int bu = u < n ? b[u] : b[0];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = min(r0[u] + ty + k * (NT / kTr), sh.R - 1), c = min(c0[u] + tx, sh.Cc - 1);
        v[u][k] = src[bu * sh.sbs + (long long)r * sh.srs + c];
      }
    }
#pragma unroll
    for (int u = 0; u < KT; ++u)
#pragma unroll
      for (int k = 0; k < RPT; ++k) tiles[u * kTrTileElems + (ty + k * (NT / kTr)) * (kTr + 1) + tx] = v[u][k];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KT; ++u) {
      if (u >= n) break;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = ty + k * (NT / kTr);
        const int c = c0[u] + i, r = r0[u] + tx;
        if (r < sh.R && c < sh.Cc)
          dst[b[u] * sh.dbs + (long long)c * sh.drs + r] = tiles[u * kTrTileElems + tx * (kTr + 1) + i];
      }
    }
    __syncthreads();  // the tiles are refilled by the next round
  }
}

}  // namespace dev
}  // namespace ggdt
