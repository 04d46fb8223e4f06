// Device code of one 3D directional pass with one thread per cell of the tile
// box (single-channel images).
//
// Same decomposition as run_pass in pass_device.h: the plane is cut into
// 16 x 16 tiles owned by workgroups, the scan axis into chunks of K = 8 steps,
// and each chunk recomputes a halo that shrinks by one voxel per plane, so that
// neighbours are consulted only between chunks, through epoch-tagged exchange
// words.  The mapping differs: a workgroup of 1024 threads covers the tile's
// 32 x 32 box (the tile grown by K on each side) with one thread per box cell,
// fixed for the whole pass.  A thread holds its cell's image and D_old values
// for the chunk's planes in registers, loaded straight from global memory; the
// only LDS traffic is the previous plane's (D, I) pairs, read at fixed offsets.
// At step i of a chunk the cells within Chebyshev distance kk - 1 - i of the
// tile compute; the others idle.
#pragma once

#include "pass_device.h"

namespace ggdt {
namespace dev {

constexpr int kCellTP = 16, kCellTQ = 16, kCellK = 8;
constexpr int kCellBQ = kCellTQ + 2 * kCellK;          // 32: box row length
constexpr int kCellThreads = kCellBQ * kCellBQ;         // 1024: one thread per box cell

template <int MODE>
__device__ __forceinline__ float cell_edge(const PassDesc& g, int j, float ix, float iy) {
  if (MODE == kModeLam0) return g.W0[j];
  const float d = ix - iy;
  if (MODE == kModeLam1C1) return fabsf(d);
  return sqrtf(fmaf(g.lam, d * d, g.A[j]));
}

// One pass of one single-channel 3D instance by workgroup `wg` of G (blockDim
// = 1024).  `pair` holds 2 x 1024 float2 of LDS.  False if a bounded wait gave up.
template <int MODE, bool REC>
__device__ __forceinline__ bool run_pass_cell(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                              unsigned long long limit, float2* pair, int wg, int G) {
  constexpr int TP = kCellTP, TQ = kCellTQ, K = kCellK, BQ = kCellBQ, NB = kCellThreads;
  const PassDesc g = *gp;
  const int tid = threadIdx.x;
  const int br = tid / BQ, bc = tid - br * BQ;
  // Chebyshev distance of the box cell outside the tile (0 for the tile's own cells)
  const int e = max(max(max(K - br, br - (K + TP - 1)), max(K - bc, bc - (K + TQ - 1))), 0);
  const int own_slot = (br - K) * TQ + (bc - K);  // valid when e == 0
  const int ntiles = g.ntp * g.ntq;
  const int Na = g.Na, Np = g.Np, Nq = g.Nq;
  constexpr bool USE_I = MODE != kModeLam0;
  float2* const P0 = pair;
  float2* const P1 = pair + NB;

  // First plane in scan order (never changed by the pass): written when the
  // pass initialises D, recorded as "keep" when records are asked for.
  if (g.init || REC) {
    const int kf = g.sign > 0 ? 0 : Na - 1;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int pp = tp * TP - K + br, qq = tq * TQ - K + bc;
      if (e == 0 && pp < Np && qq < Nq) {
        const int x = kf * g.sa + pp * g.sp + qq * g.sq;
        if (g.init) g.D[x] = g.v * g.mask[x];
        if (REC && g.rec) g.rec[x] = 0;
      }
    }
  }

  const float* const dsrc0 = g.init ? g.mask : g.D;
  for (int c = 0; c < g.nchunk; ++c) {
    const int t0 = 1 + c * K;  // scan position of the chunk's first computed plane
    const int kk = min(K, Na - t0);
    const unsigned epoch_in = g.epoch_base + (unsigned)c;
    const unsigned epoch_out = epoch_in + 1u;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int pp = p0 - K + br, qq = q0 - K + bc;
      const bool in = pp >= 0 && pp < Np && qq >= 0 && qq < Nq;
      const int xpq = in ? pp * g.sp + qq * g.sq : 0;
      // memory index of plane j of the chunk (scan position t0 - 1 + j)
      auto xof = [&](int j) {
        const int t = t0 - 1 + j;
        return (g.sign > 0 ? t : Na - 1 - t) * g.sa + xpq;
      };

      // 1. This cell's image and D_old on the planes where it is needed: plane
      // j is used by the cells within distance kk - j of the tile.
      float ix[K + 1], dd[K + 1];
#pragma unroll
      for (int j = 0; j <= K; ++j) {
        const bool need = in && j <= kk && e <= kk - j;
        ix[j] = 0.0f;
        dd[j] = 0.0f;
        if (need) {
          const int x = xof(j);
          if (USE_I) ix[j] = g.image[x];
          if (j >= 1 || c == 0) dd[j] = dsrc0[x];
        }
      }

      // 2. Plane 0 of the chunk: the pass's first plane in chunk 0, else the
      // values the previous chunk published (this tile's and its neighbours').
      float d0 = __builtin_inff();
      int fail = 0;
      if (in && e <= kk) {
        if (c == 0) {
          d0 = g.init ? g.v * dd[0] : dd[0];
        } else {
          const int otp = pp / TP, otq = qq / TQ;
          const int slot = (pp - otp * TP) * TQ + (qq - otq * TQ);
          const unsigned long long* a =
              xbuf + (size_t)((c - 1) & 1) * ntiles * (TP * TQ) + (size_t)(otp * g.ntq + otq) * (TP * TQ) + slot;
          unsigned long long wv = ld64_relaxed(a);
          unsigned long long polls = 0;
          while ((unsigned)(wv >> 32) != epoch_in) {
            if (ld_relaxed(words + kWordAbort) != 0u) {
              fail = 1;
              break;
            }
            if (++polls > limit) {
              __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              fail = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            wv = ld64_relaxed(a);
          }
          d0 = __uint_as_float((unsigned)wv);
        }
      }
      // Cells outside the volume hold +inf in both planes, so candidates through
      // them never win and the candidate loop needs no bounds checks.
      P0[tid] = make_float2(d0, ix[0]);
      if (!in) P1[tid] = make_float2(__builtin_inff(), 0.0f);
      if (__syncthreads_or(fail)) return false;

      // 3. The chunk's planes.
      float2* Pp = P0;
      float2* Pc = P1;
      unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)tile * (TP * TQ);
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if (i >= kk) break;
        if (in && e <= kk - 1 - i) {
          const float ixj = ix[i + 1];
          float best = g.init ? g.v * dd[i + 1] : dd[i + 1];
          int choice = 0;
#pragma unroll
          for (int dp = -1; dp <= 1; ++dp) {
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) {
              const int j = (dp + 1) * 3 + dq + 1;
              const float2 y = Pp[tid + dp * BQ + dq];
              const float cand = y.x + cell_edge<MODE>(g, j, ixj, y.y);
              if (REC) {
                if (cand < best) {
                  best = cand;
                  choice = 1 + j;
                }
              } else {
                best = fminf(best, cand);
              }
            }
          }
          Pc[tid] = make_float2(best, ixj);
          if (e == 0) {
            const int x = xof(i + 1);
            g.D[x] = best;
            if (REC && g.rec) g.rec[x] = (uint8_t)choice;
            if (i == kk - 1) st64_relaxed(xout + own_slot, ((unsigned long long)epoch_out << 32) | __float_as_uint(best));
          }
        }
        lds_barrier();
        float2* t = Pp;
        Pp = Pc;
        Pc = t;
      }
    }
  }
  return true;
}

// Requested mode RMODE falls back to the general formula when the image
// classification word rules the fast edge cost out.
template <int RMODE, bool REC>
__device__ __forceinline__ bool run_pass_cell_mode(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                   const unsigned* cls_word, unsigned long long limit, float2* pair,
                                                   int wg, int G) {
  if (RMODE == kModeGeneral) return run_pass_cell<kModeGeneral, REC>(gp, xbuf, words, limit, pair, wg, G);
  const unsigned cls = ld_relaxed(cls_word);
  const bool fast = (RMODE == kModeLam0) ? (cls & kClassHuge) == 0u : cls == 0u;
  if (fast) return run_pass_cell<RMODE, REC>(gp, xbuf, words, limit, pair, wg, G);
  return run_pass_cell<kModeGeneral, REC>(gp, xbuf, words, limit, pair, wg, G);
}

}  // namespace dev
}  // namespace ggdt
