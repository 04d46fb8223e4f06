// Directional pass of a 2D image with one wavefront per tile: a row of the pass
// is updated in parallel from the previous row (FastGeodis paper, section
// "Implementation"), each lane owning one cell of the tile's row grown by K on
// both sides.  Neighbours in the previous row are the adjacent lanes, moved with
// whole-wave DPP shifts, so a step needs no barrier, no LDS and no index
// arithmetic: the serial chain of rows runs at the latency of a few VALU
// instructions per row instead of a workgroup barrier per row.
//
// Chunks of K rows use the same overlapped tiling and epoch exchange as the
// other pass kernels: the halo shrinks by one cell per row, and the tile's last
// row of a chunk is published as 64-bit exchange words (epoch << 32 | bits).
// The next chunk's rows are loaded into registers while the current chunk runs.
#pragma once

#include "pass_device.h"

namespace ggdt {
namespace dev {

static_assert(kRowLanes == 64 && kRowTQ == kRowLanes - 2 * kRowK, "row tile: one wave, K halo cells per side");

// Value of the lane to the left (lane - 1) / right (lane + 1), 0 past the
// wave's ends (lanes 0 and 63 are halo cells that never take part in a step).
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}

// Edge cost through offset j from the registers of x (ix) and of its parent (iy).
template <int MODE, int NCH>
__device__ __forceinline__ float row_edge(const PassDesc& g, int j, const float* ix, const float* iy) {
  if (MODE == kModeLam0) return g.W0[j];
  const float d0 = ix[0] - iy[0];
  if (MODE == kModeLam1C1) return fabsf(d0);
  float s = d0 * d0;
#pragma unroll
  for (int c = 1; c < NCH; ++c) {
    const float dc = ix[c] - iy[c];
    s = fmaf(dc, dc, s);
  }
  return general_root<MODE>(fmaf(g.lam, s, g.A[j]));
}

// One 2D pass of an image with NCH channels (the image is not read when MODE is
// kModeLam0), run by workgroup `wg` of G single-wave workgroups.
template <int MODE, int NCH, bool REC, int FMT = kImgF32>
__device__ __forceinline__ bool run_pass_row(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                             unsigned long long limit, int wg, int G) {
  constexpr int K = kRowK, TQ = kRowTQ;
  constexpr bool USE_I = MODE != kModeLam0;
  constexpr int NI = USE_I ? NCH : 1;
  const PassDesc g = *gp;
  const auto gImage = image_of<FMT>(g.image);  // read widened to fp32
  const gmem<const float> gMask = to_gmem(g.mask);
  const gmem<float> gD = to_gmem(g.D);
  const gmem<uint8_t> gRec = to_gmem(g.rec);
  const int lane = threadIdx.x;
  // distance of the lane's cell outside the tile (0 for the tile's own cells)
  const int e = max(max(K - lane, lane - (K + TQ - 1)), 0);
  const int own = lane - K;  // the cell's slot in the tile when e == 0
  const int ntiles = g.ntq;
  if (wg >= ntiles) return true;
  const int Na = g.Na, Nq = g.Nq;
  const long long cstride = g.N;

  // First row in scan order (never changed by the pass).
  if (g.init || REC) {
    const int kf = g.sign > 0 ? 0 : Na - 1;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int q = tile * TQ + own;
      if (e == 0 && q < Nq) {
        const int x = kf * g.sa + q * g.sq;
        if (g.init) gD[x] = g.v * gMask[x];
        if (REC && g.rec) gRec[x] = 0;
      }
    }
  }

  const gmem<const float> dsrc0 = g.init ? gMask : (gmem<const float>)gD;
  const float vscale = g.init ? g.v : 1.0f;
  const int nmine = (ntiles - wg + G - 1) / G;  // >= 1 since wg < ntiles
  const int nitems = g.nchunk * nmine;
  struct Item {
    int c, tile, t0, kk, q, xq;
    bool in;
  };
  auto item_of = [&](int n) {
    Item it;
    it.c = n / nmine;
    it.tile = wg + (n - it.c * nmine) * G;
    it.t0 = 1 + it.c * K;
    it.kk = min(K, Na - it.t0);
    it.q = it.tile * TQ - K + lane;
    it.in = it.q >= 0 && it.q < Nq;
    it.xq = it.in ? it.q * g.sq : 0;
    return it;
  };
  // memory index of row j of an item's chunk (scan position t0 - 1 + j)
  auto xof = [&](const Item& it, int j) {
    const int t = it.t0 - 1 + j;
    return (g.sign > 0 ? t : Na - 1 - t) * g.sa + it.xq;
  };

  // Row j of an item is used by the cells within distance kk - j of the tile.
  // Every lane loads every row (an unneeded one from a clamped, in-bounds
  // address) and keeps the value only where it is needed: no branch.  Row j
  // lies sign * sa elements after row j - 1.
  float nd[K + 1], nx[K + 1][NI];
  // A 16-bit image's raw bits and the last row the lane needs: widened and
  // selected where consumed, so that no load of the prefetch is waited for.
  unsigned nxr[K + 1][NI];
  int nlast = -1;
  auto fetch = [&](const Item& it) {
    const int x0 = xof(it, 0);
    const int step = g.sign * g.sa;
    const int last = it.in ? it.kk - e : -1;  // the lane needs rows 0 .. last
    nlast = last;
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      const bool need = j <= last;
      int x = need ? x0 + j * step : 0;
      // opaque to the optimiser, which would otherwise turn the clamped load
      // and the select back into a branch per row
      __asm__ volatile("" : "+v"(x));
      const float dv = dsrc0[x];
      nd[j] = (need && (j >= 1 || it.c == 0)) ? dv : 0.0f;
      if (USE_I) {
#pragma unroll
        for (int c = 0; c < NI; ++c) {
          if constexpr (FMT == kImgF32) {
            const float iv = gImage[c * cstride + x];
            nx[j][c] = need ? iv : 0.0f;
          } else {
            nxr[j][c] = gImage[c * cstride + x];
          }
        }
      } else {
        nx[j][0] = 0.0f;
      }
    }
  };

  int chg = 0;  // an own cell was lowered (convergence mode)
  Item cur = item_of(0);
  fetch(cur);
  for (int n = 0; n < nitems; ++n) {
    const int c = cur.c, kk = cur.kk;
    const unsigned epoch_in = g.epoch_base + (unsigned)c;  // published by chunk c - 1
    const unsigned epoch_out = epoch_in + 1u;
    const bool has_next = n + 1 < nitems;
    const Item nxt = item_of(has_next ? n + 1 : n);
    float dd[K + 1], ix[K + 1][NI];
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      dd[j] = nd[j] * vscale;  // the initialising pass reads the mask: D_old = v * M
#pragma unroll
      for (int ch = 0; ch < NI; ++ch) {
        if constexpr (FMT == kImgF32 || !USE_I)
          ix[j][ch] = nx[j][ch];
        else
          ix[j][ch] = j <= nlast ? widen<FMT>((uint16_t)nxr[j][ch]) : 0.0f;
      }
    }

    // Row 0 of the chunk: the pass's first row in chunk 0, else the values the
    // previous chunk published (this tile's and its neighbours').  Cells outside
    // the image hold +inf, so candidates through them never win.
    float dcur = __builtin_inff();
    int fail = 0;
    if (cur.in && e <= kk) {
      if (c == 0) {
        dcur = dd[0];
      } else {
        // the owner's slot of cell q is q itself: tile q / TQ, slot q % TQ
        const unsigned long long* a = xbuf + (size_t)((c - 1) & 1) * ntiles * TQ + cur.q;
        unsigned long long wv = ld64_relaxed(a);
        unsigned long long polls = 0;
        while ((unsigned)(wv >> 32) != epoch_in) {
          if ((++polls & 31u) == 0u) {
            if (ld_relaxed(words + kWordAbort) != 0u) {
              fail = 1;
              break;
            }
            if (polls > limit) {
              __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              fail = 1;
              break;
            }
          }
          __builtin_amdgcn_s_sleep(1);
          wv = ld64_relaxed(a);
        }
        dcur = __uint_as_float((unsigned)wv);
      }
    }
    if (__any(fail)) return false;
    // the next item's rows load while this item's rows are advanced
    if (has_next) fetch(nxt);

    float icur[NI];
#pragma unroll
    for (int ch = 0; ch < NI; ++ch) icur[ch] = ix[0][ch];
    // The steps, branch-free: every lane computes, lanes outside the image keep
    // +inf.  A lane of the shrinking cone (e <= kk - 1 - i) reads only lanes
    // that were in the cone at the previous row, so values computed outside
    // the cone are never used.  Full chunks run without a trip-count guard; the
    // last one keeps a fixed trip count with a uniform guard (the loop holds
    // the convergent lane shifts, which keep it from being unrolled around an
    // early exit).
    float res[K];
    int rch[K];
    auto step = [&](int i) {
      // the previous row's neighbours, offsets j = 0 (q - 1), 1 (q), 2 (q + 1)
      float dy[3], iy[3][NI];
      dy[0] = from_left(dcur);
      dy[1] = dcur;
      dy[2] = from_right(dcur);
#pragma unroll
      for (int ch = 0; ch < NI; ++ch) {
        iy[0][ch] = from_left(icur[ch]);
        iy[1][ch] = icur[ch];
        iy[2][ch] = from_right(icur[ch]);
      }
      float best = dd[i + 1];
      int choice = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float cand = dy[j] + row_edge<MODE, NI>(g, j, ix[i + 1], iy[j]);
        if (REC) {
          choice = cand < best ? 1 + j : choice;
          best = cand < best ? cand : best;
        } else {
          best = fminf(best, cand);
        }
      }
      res[i] = best;
      rch[i] = choice;
      dcur = cur.in ? best : __builtin_inff();
#pragma unroll
      for (int ch = 0; ch < NI; ++ch) icur[ch] = ix[i + 1][ch];
    };
    if (kk == K) {
#pragma unroll
      for (int i = 0; i < K; ++i) step(i);
    } else {
#pragma unroll
      for (int i = 0; i < K; ++i)
        if (i < kk) step(i);
    }
    // The tile's own cells: the exchange word of the chunk's last row first
    // (the neighbours wait for it), then the rows.
    if (cur.in && e == 0) {
      unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * TQ + (size_t)cur.tile * TQ;
      float last = res[0];
#pragma unroll
      for (int i = 1; i < K; ++i) last = i < kk ? res[i] : last;
      st64_relaxed(xout + own, ((unsigned long long)epoch_out << 32) | __float_as_uint(last));
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if (i < kk) {
          const int x = xof(cur, i + 1);
          chg |= res[i] < dd[i + 1];
          gD[x] = res[i];
          if (REC && g.rec) gRec[x] = (uint8_t)rch[i];
        }
      }
    }
    cur = nxt;
  }
  if (g.converge && __any(chg) && lane == 0)
    __hip_atomic_store(words + kWordChanged, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Requested mode RMODE falls back to the general formula when the image
// classification word rules the fast edge cost out.
template <int RMODE, int NCH, bool REC, int FMT = kImgF32>
__device__ __forceinline__ bool run_pass_row_mode(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                  const unsigned* cls_word, unsigned long long limit, int wg, int G) {
  if (RMODE == kModeGeneral) {
    if (general_n_ok(gp->sqrt_normal, cls_word))
      return run_pass_row<kModeGeneralN, NCH, REC, FMT>(gp, xbuf, words, limit, wg, G);
    return run_pass_row<kModeGeneral, NCH, REC, FMT>(gp, xbuf, words, limit, wg, G);
  }
  const bool fast = fast_mode_ok(RMODE, ld_relaxed(cls_word));
  if (fast) return run_pass_row<RMODE, NCH, REC, FMT>(gp, xbuf, words, limit, wg, G);
  return run_pass_row<kModeGeneral, NCH, REC, FMT>(gp, xbuf, words, limit, wg, G);
}

}  // namespace dev
}  // namespace ggdt
