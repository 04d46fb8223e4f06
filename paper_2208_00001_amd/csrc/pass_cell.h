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
// Scan-contiguous layout: per box cell a run of kCellSC consecutive memory
// positions along the scan axis (K + 1 planes and up to 3 alignment slots,
// starting at a multiple of 4), and the own cells' results at an odd stride.
constexpr int kCellSC = 4 * ((kCellK + 4 + 3) / 4);    // 12
constexpr int kCellSCR = kCellK + 1;                     // 9
constexpr int kCellStage = kCellThreads * kCellSC;       // floats of one staged array

// The same box of 1024 cells also holds a 24 x 24 tile with K = 4 (batched
// launches may choose it): 1.27 computed cells per voxel update instead of
// 2.15, for twice the exchanges.
template <int TT, int KC>
struct CellGeom {
  static constexpr int TP = TT, TQ = TT, K = KC;
  static constexpr int BQ = TT + 2 * KC;
  static constexpr int NB = BQ * BQ;
  static constexpr int SC = 4 * ((KC + 4 + 3) / 4);
  static constexpr int SCR = KC + 1;
  static constexpr int STAGE = NB * SC;
  static constexpr int RES = TT * TT * SCR;
  static_assert(NB == kCellThreads, "one thread per cell of a 32 x 32 box");
};
using CellGeomWide = CellGeom<24, 4>;
constexpr int kCellWideTP = CellGeomWide::TP, kCellWideK = CellGeomWide::K;
// largest staged array and result buffer over the geometries
constexpr int kCellStageMax = kCellStage > CellGeomWide::STAGE ? kCellStage : CellGeomWide::STAGE;
constexpr int kCellResMax = kCellTP * kCellTQ * kCellSCR > CellGeomWide::RES ? kCellTP * kCellTQ * kCellSCR
                                                                                : CellGeomWide::RES;

template <int MODE>
__device__ __forceinline__ float cell_edge(const PassDesc& g, int j, float ix, float iy) {
  if (MODE == kModeLam0) return g.W0[j];
  const float d = ix - iy;
  if (MODE == kModeLam1C1) return fabsf(d);
  return general_root<MODE>(fmaf(g.lam, d * d, g.A[j]));
}

// One pass of one single-channel 3D instance by workgroup `wg` of G (blockDim
// = 1024), `lds` laid out as cell_lds_bytes(SCANC) describes.  SCANC: the scan
// axis is the contiguous memory axis; a thread's planes are then consecutive
// floats, and are gathered through LDS by 16-byte runs instead of one load per
// lane and plane.  False if a bounded wait gave up.
// Workgroup barrier for the step loop: this wave's LDS accesses are complete
// (lgkmcnt(0)) and the compiler moves no memory access across it.  Unlike a
// release fence it does not wait for global stores or for global->LDS copies
// in flight, which target other LDS arrays and are waited for where read.
__device__ __forceinline__ void step_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt and expcnt at their maxima, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// LDS of the pass, as separate arrays: the global->LDS copies of the next item
// then provably do not alias the pair planes, and the steps need not wait for
// them to land.
struct CellLds {
  float2* pair;  // 2 x kCellThreads
  float* stD;    // kCellStage (scan-contiguous layout only)
  float* stI;    // kCellStage
  float* res;    // kCellTP * kCellTQ * kCellSCR
  int* fail;     // one word: item number + 1 of a bounded wait that gave up
};

// Bytes of one dynamic LDS area holding every array of CellLds, for either
// geometry.
constexpr size_t kCellLdsBytes = sizeof(float2) * 2 * kCellThreads +
                                 sizeof(float) * ((size_t)2 * kCellStageMax + (size_t)kCellResMax) + sizeof(int);

// CellLds carved from one dynamic LDS area of kCellLdsBytes (launches that
// share the area with other paths).
__device__ __forceinline__ CellLds carve_cell_lds(float* lds) {
  CellLds l;
  l.pair = reinterpret_cast<float2*>(lds);
  l.stD = lds + 4 * kCellThreads;
  l.stI = l.stD + kCellStageMax;
  l.res = l.stI + kCellStageMax;
  l.fail = reinterpret_cast<int*>(l.res + kCellResMax);
  return l;
}

template <bool SCANC, int MODE, bool REC, int TT = kCellTP, int KC = kCellK, int FMT = kImgF32>
__device__ __forceinline__ bool run_pass_cell(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                              unsigned long long limit, const CellLds& lds, int wg, int G) {
  using Geo = CellGeom<TT, KC>;
  constexpr int TP = Geo::TP, TQ = Geo::TQ, K = Geo::K, BQ = Geo::BQ, NB = Geo::NB;
  constexpr int SC = Geo::SC, SCR = Geo::SCR, STAGE = Geo::STAGE;
  const PassDesc g = resolve_offsets(*gp, words);
  // global-memory views of the descriptor's arrays (the image in its storage format)
  const gmem<const float> gImage = to_gmem(g.image);           // fp32 image
  const gmem<const uint16_t> gImage16 = image_of<kImgBF16>(g.image);  // 16-bit image (FMT != kImgF32)
  // the same, two positions per 32-bit word (even element offsets)
  const gmem<const unsigned> gImage2 = (gmem<const unsigned>)(const unsigned*)(const void*)g.image;
  const gmem<const float> gMask = to_gmem(g.mask);
  const gmem<float> gD = to_gmem(g.D);
  const gmem<uint8_t> gRec = to_gmem(g.rec);
  const int tid = threadIdx.x;
  const int br = tid / BQ, bc = tid - br * BQ;
  // Chebyshev distance of the box cell outside the tile (0 for the tile's own cells)
  const int e = max(max(max(K - br, br - (K + TP - 1)), max(K - bc, bc - (K + TQ - 1))), 0);
  const int own_slot = (br - K) * TQ + (bc - K);  // valid when e == 0
  const int ntiles = g.ntp * g.ntq;
  // A batched instance may hold more workgroups than this pass has tiles.
  if (wg >= ntiles) return true;
  const int Na = g.Na, Np = g.Np, Nq = g.Nq;
  constexpr bool USE_I = MODE != kModeLam0;
  float2* const P0 = lds.pair;
  float2* const P1 = P0 + NB;
  float* const StD = lds.stD;
  float* const StI = lds.stI;
  float* const Res = lds.res;
  const int wave0 = tid & ~63;
  // 16-byte runs need every run start 16-byte aligned
  const bool vec4s = SCANC && (Na & 3) == 0 && (g.sp & 3) == 0 && (g.sq & 3) == 0;
  // A 16-bit image is staged by 16-byte groups of 8 positions (runs of SC16
  // positions from a multiple of 8) when every run start is 16-byte aligned,
  // else as 32-bit pairs of positions when it is 4-byte aligned, else it is
  // loaded into registers.
  constexpr int SC16 = 8 * ((K + 8 + 7) / 8);
  const bool vec8h = SCANC && FMT != kImgF32 && (Na & 7) == 0 && (g.sp & 7) == 0 && (g.sq & 7) == 0;
  const bool pairs16 =
      SCANC && FMT != kImgF32 && !vec8h && (Na & 1) == 0 && (g.sp & 1) == 0 && (g.sq & 1) == 0;
  const uint16_t* const StI16 = reinterpret_cast<const uint16_t*>(lds.stI);

  // First plane in scan order (never changed by the pass): written when the
  // pass initialises D, recorded as "keep" when records are asked for.
  if (g.init || REC) {
    const int kf = g.sign > 0 ? 0 : Na - 1;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int pp = tp * TP - K + br, qq = tq * TQ - K + bc;
      if (e == 0 && pp < Np && qq < Nq) {
        const int x = kf * g.sa + pp * g.sp + qq * g.sq;
        if (g.init) gD[x] = g.v * gMask[x];
        if (REC && g.rec) gRec[x] = 0;
      }
    }
  }

  if (tid == 0) *lds.fail = 0;  // read only after a barrier
  const gmem<const float> dsrc0 = g.init ? gMask : (gmem<const float>)gD;
  const float vscale = g.init ? g.v : 1.0f;
  // Work items in order: chunk-major, then this workgroup's tiles.  The next
  // item's image and D_old are fetched while the current item's planes are
  // advanced (into registers, or into the LDS staging area once the current
  // item has copied its values out of it).
  const int nmine = (ntiles - wg + G - 1) / G;  // >= 1 since wg < ntiles
  const int nitems = g.nchunk * nmine;
  struct Item {
    int c, t0, kk, tile, p0, q0, pp, qq, xpq;
    bool in;
  };
  auto item_of = [&](int n) {
    Item it;
    it.c = n / nmine;
    it.tile = wg + (n - it.c * nmine) * G;
    it.t0 = 1 + it.c * K;  // scan position of the chunk's first computed plane
    it.kk = min(K, Na - it.t0);
    const int tp = it.tile / g.ntq, tq = it.tile - tp * g.ntq;
    it.p0 = tp * TP;
    it.q0 = tq * TQ;
    it.pp = it.p0 - K + br;
    it.qq = it.q0 - K + bc;
    it.in = it.pp >= 0 && it.pp < Np && it.qq >= 0 && it.qq < Nq;
    it.xpq = it.in ? it.pp * g.sp + it.qq * g.sq : 0;
    return it;
  };
  // memory index of plane j of an item's chunk (scan position t0 - 1 + j)
  auto xof = [&](const Item& it, int j) {
    const int t = it.t0 - 1 + j;
    return (g.sign > 0 ? t : Na - 1 - t) * g.sa + it.xpq;
  };
  // Slot of plane j in a cell's staged run (scan-contiguous layout): the run
  // holds memory positions kb .. kb + SC - 1, kb the chunk's lowest position
  // rounded down to a multiple of 4.
  auto run_start = [&](const Item& it) {
    const int kmin = g.sign > 0 ? it.t0 - 1 : Na - it.t0 - it.kk;
    return kmin & ~3;
  };
  auto slot_base = [&](const Item& it, int kb) { return g.sign > 0 ? it.t0 - 1 - kb : Na - it.t0 - kb; };

  // Plane j of an item is used by the cells within distance kk - j of the tile.
  float nx[K + 1], nd[K + 1];
  // A 16-bit image's raw bits: widened where consumed, so that no load of the
  // prefetch is waited for when it is issued.
  unsigned nxr[K + 1];
  auto fetch_regs = [&](const Item& it) {
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      const bool need = it.in && j <= it.kk && e <= it.kk - j;
      nx[j] = 0.0f;
      nxr[j] = 0u;
      nd[j] = 0.0f;
      if (need) {
        const int x = xof(it, j);
        if (USE_I) {
          if constexpr (FMT == kImgF32)
            nx[j] = gImage[x];
          else
            nxr[j] = gImage16[x];
        }
        if (j >= 1 || it.c == 0) nd[j] = dsrc0[x];
      }
    }
  };
  // A 16-bit image in the scan-contiguous layout goes to registers (2-byte
  // loads along the cell's run), D_old through the LDS staging.
  auto fetch_img16 = [&](const Item& it) {
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      const bool need = it.in && j <= it.kk && e <= it.kk - j;
      nxr[j] = 0u;
      if (need) nxr[j] = gImage16[xof(it, j)];
    }
  };
  auto stage = [&](const Item& it) {
    const int kb = run_start(it);
    // the thread index, opaque to the optimiser: the staging index math is
    // recomputed per item instead of being hoisted and held in registers
    int stid = tid;
    __asm__ volatile("" : "+v"(stid));
    if (vec4s) {
      constexpr int GPC = SC / 4;  // 16-byte groups per cell
      constexpr int NG = STAGE / 4;
#pragma unroll
      for (int g0 = 0; g0 < NG; g0 += NB) {
        const int gi = g0 + stid;
        const int lx = gi / GPC, gg = gi - lx * GPC;
        const int cbr = lx / BQ, cbc = lx - cbr * BQ;
        const int cpp = it.p0 - K + cbr, cqq = it.q0 - K + cbc;
        const int ce = max(max(max(K - cbr, cbr - (K + TP - 1)), max(K - cbc, cbc - (K + TQ - 1))), 0);
        const int k0 = kb + 4 * gg;
        const bool ok = k0 + 3 <= Na - 1 && cpp >= 0 && cpp < Np && cqq >= 0 && cqq < Nq;
        // planes j held by this group, and the highest plane this cell needs
        const int jlo = g.sign > 0 ? k0 - (it.t0 - 1) : (Na - it.t0) - (k0 + 3);
        const int jtop = min(jlo + 3, it.kk - ce);
        if (ok) {
          const int x = k0 + cpp * g.sp + cqq * g.sq;
          if (max(jlo, it.c == 0 ? 0 : 1) <= jtop)
            __builtin_amdgcn_global_load_lds(dsrc0 + x, StD + 4 * (g0 + wave0), 16, 0, 0);
          if (FMT == kImgF32 && USE_I && max(jlo, 0) <= jtop)
            __builtin_amdgcn_global_load_lds(gImage + x, StI + 4 * (g0 + wave0), 16, 0, 0);
        }
      }
    } else {
#pragma unroll 1
      for (int f0 = 0; f0 < STAGE; f0 += NB) {
        const int f = f0 + stid;
        const int lx = f / SC, sl = f - lx * SC;
        const int cbr = lx / BQ, cbc = lx - cbr * BQ;
        const int cpp = it.p0 - K + cbr, cqq = it.q0 - K + cbc;
        const int ce = max(max(max(K - cbr, cbr - (K + TP - 1)), max(K - cbc, cbc - (K + TQ - 1))), 0);
        const int k = kb + sl;
        const int j = g.sign > 0 ? k - (it.t0 - 1) : (Na - it.t0) - k;
        const bool ok = j >= 0 && j <= it.kk && ce <= it.kk - j && cpp >= 0 && cpp < Np && cqq >= 0 && cqq < Nq;
        if (ok) {
          const int x = k + cpp * g.sp + cqq * g.sq;
          if (j >= 1 || it.c == 0) __builtin_amdgcn_global_load_lds(dsrc0 + x, StD + f0 + wave0, 4, 0, 0);
          if (FMT == kImgF32 && USE_I) __builtin_amdgcn_global_load_lds(gImage + x, StI + f0 + wave0, 4, 0, 0);
        }
      }
    }
    // A 16-bit image in 32-bit words of two positions: the run of a cell is SC / 2
    // words, so the staged 16-bit elements keep the fp32 layout's indices.
    if constexpr (FMT != kImgF32 && USE_I) {
      if (vec8h) {
        constexpr int GPC = SC16 / 8;  // 16-byte groups per cell
        constexpr int NG = NB * GPC;
        const int kmin = g.sign > 0 ? it.t0 - 1 : Na - it.t0 - it.kk;
        const int kb16 = kmin & ~7;
#pragma unroll
        for (int g0 = 0; g0 < NG; g0 += NB) {
          const int gi = g0 + stid;
          const int lx = gi / GPC, gg = gi - lx * GPC;
          const int cbr = lx / BQ, cbc = lx - cbr * BQ;
          const int cpp = it.p0 - K + cbr, cqq = it.q0 - K + cbc;
          const int ce = max(max(max(K - cbr, cbr - (K + TP - 1)), max(K - cbc, cbc - (K + TQ - 1))), 0);
          const int k0 = kb16 + 8 * gg;
          const bool ok = k0 + 7 <= Na - 1 && cpp >= 0 && cpp < Np && cqq >= 0 && cqq < Nq;
          const int jlo = g.sign > 0 ? k0 - (it.t0 - 1) : (Na - it.t0) - (k0 + 7);
          const int jtop = min(jlo + 7, it.kk - ce);
          if (ok && max(jlo, 0) <= jtop)
            __builtin_amdgcn_global_load_lds(gImage16 + (k0 + cpp * g.sp + cqq * g.sq), lds.stI + 4 * (g0 + wave0),
                                             16, 0, 0);
        }
      }
      if (pairs16) {
        constexpr int GPC = SC / 2;  // words per cell
        constexpr int NG = NB * GPC;
#pragma unroll
        for (int g0 = 0; g0 < NG; g0 += NB) {
          const int gi = g0 + stid;
          const int lx = gi / GPC, gg = gi - lx * GPC;
          const int cbr = lx / BQ, cbc = lx - cbr * BQ;
          const int cpp = it.p0 - K + cbr, cqq = it.q0 - K + cbc;
          const int ce = max(max(max(K - cbr, cbr - (K + TP - 1)), max(K - cbc, cbc - (K + TQ - 1))), 0);
          const int k0 = kb + 2 * gg;
          const bool ok = k0 + 1 <= Na - 1 && cpp >= 0 && cpp < Np && cqq >= 0 && cqq < Nq;
          // planes j held by this word, and the highest plane this cell needs
          const int jlo = g.sign > 0 ? k0 - (it.t0 - 1) : (Na - it.t0) - (k0 + 1);
          const int jtop = min(jlo + 1, it.kk - ce);
          if (ok && max(jlo, 0) <= jtop) {
            const int x = k0 + cpp * g.sp + cqq * g.sq;  // even
            __builtin_amdgcn_global_load_lds(gImage2 + (x >> 1), lds.stI + (g0 + wave0), 4, 0, 0);
          }
        }
      }
    }
  };

  int chg = 0;  // an own cell of this workgroup was lowered (convergence mode)
  Item cur = item_of(0);
  if (SCANC) {
    stage(cur);
    if constexpr (FMT != kImgF32 && USE_I) {
      if (!pairs16 && !vec8h) fetch_img16(cur);
    }
  } else {
    fetch_regs(cur);
  }
  for (int n = 0; n < nitems; ++n) {
    const int c = cur.c, kk = cur.kk;
    const unsigned epoch_in = g.epoch_base + (unsigned)c;  // published by chunk c - 1
    const unsigned epoch_out = epoch_in + 1u;
    const bool has_next = n + 1 < nitems;
    const Item nxt = item_of(has_next ? n + 1 : n);

    // 1. This item's image and D_old.
    float ix[K + 1], dd[K + 1];
    if (SCANC) {
      __builtin_amdgcn_s_waitcnt(0);  // the global->LDS copies have landed
      __syncthreads();
      const int sbase = slot_base(cur, run_start(cur));
      // slot of plane 0 in a 16-bit run of SC16 positions from a multiple of 8
      const int sbase16 = slot_base(cur, (g.sign > 0 ? cur.t0 - 1 : Na - cur.t0 - cur.kk) & ~7);
#pragma unroll
      for (int j = 0; j <= K; ++j) {
        const bool need = cur.in && j <= kk && e <= kk - j;
        const int sl = tid * SC + sbase + g.sign * j;
        if constexpr (FMT == kImgF32)
          ix[j] = (USE_I && need) ? StI[sl] : 0.0f;
        else
          ix[j] = (USE_I && need) ? widen<FMT>(vec8h ? StI16[tid * SC16 + sbase16 + g.sign * j]
                                                    : (pairs16 ? StI16[sl] : (uint16_t)nxr[j]))
                                  : 0.0f;
        dd[j] = (need && (j >= 1 || c == 0)) ? StD[sl] : 0.0f;
      }
    } else {
#pragma unroll
      for (int j = 0; j <= K; ++j) {
        if constexpr (FMT == kImgF32)
          ix[j] = nx[j];
        else
          ix[j] = widen<FMT>((uint16_t)nxr[j]);
        dd[j] = nd[j];
      }
    }
    // The initialising pass reads the mask: D_old = v * M (1 * x == x otherwise).
#pragma unroll
    for (int j = 0; j <= K; ++j) dd[j] *= vscale;

    // 2. Plane 0 of the chunk: the pass's first plane in chunk 0, else the
    // values the previous chunk published (this tile's and its neighbours').
    float d0 = __builtin_inff();
    int fail = 0;
    if (cur.in && e <= kk) {
      if (c == 0) {
        d0 = dd[0];
      } else {
        const int otp = cur.pp / TP, otq = cur.qq / TQ;
        const int slot = (cur.pp - otp * TP) * TQ + (cur.qq - otq * TQ);
        const unsigned long long* a =
            xbuf + (size_t)((c - 1) & 1) * ntiles * (TP * TQ) + (size_t)(otp * g.ntq + otq) * (TP * TQ) + slot;
        unsigned long long wv = ld64_relaxed(a);
        unsigned long long polls = 0;
        while ((unsigned)(wv >> 32) != epoch_in) {
          // the abort word costs a memory round trip: look at it every 32 polls
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
        d0 = __uint_as_float((unsigned)wv);
      }
    }
    // Cells outside the volume hold +inf in both planes, so candidates through
    // them never win and the candidate loop needs no bounds checks.
    P0[tid] = make_float2(d0, ix[0]);
    if (!cur.in) P1[tid] = make_float2(__builtin_inff(), 0.0f);
    if (fail) *lds.fail = n + 1;
    step_barrier();
    if (*lds.fail == n + 1) return false;
    // Fetch the next item's registers now: the loads overlap the steps, and
    // nothing before this point waits on them.  (The scan-contiguous staging is
    // refilled after the steps instead: global->LDS copies in flight slow the
    // step loop down by more than their latency costs when exposed.)
    if (!SCANC && has_next) fetch_regs(nxt);
    if constexpr (SCANC && FMT != kImgF32 && USE_I) {
      if (has_next && !pairs16 && !vec8h) fetch_img16(nxt);
    }

    // 3. The chunk's planes.
    float2* Pp = P0;
    float2* Pc = P1;
    unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)cur.tile * (TP * TQ);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i >= kk) break;
      if (cur.in && e <= kk - 1 - i) {
        const float ixj = ix[i + 1];
        float best = dd[i + 1];
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
          chg |= best < dd[i + 1];
          const int x = xof(cur, i + 1);
          // per-step stores spread over the steps' barrier stalls; the
          // scan-contiguous layout stages its results for run-wise writes
          if (SCANC)
            Res[own_slot * SCR + i] = best;
          else
            gD[x] = best;
          if (REC && g.rec) gRec[x] = (uint8_t)choice;
          if (i == kk - 1) st64_relaxed(xout + own_slot, ((unsigned long long)epoch_out << 32) | __float_as_uint(best));
        }
      }
      step_barrier();
      float2* t = Pp;
      Pp = Pc;
      Pc = t;
    }

    // 4. Scan-contiguous results: each own cell's kk planes as one run of
    // consecutive memory positions, K lanes per cell.  TP * TQ * K need not be
    // a multiple of the workgroup (24 x 24 x 4 = 2304): the last round is partial.
    if (SCANC) {
#pragma unroll
      for (int f0 = 0; f0 < TP * TQ * K; f0 += NB) {
        const int f = f0 + tid;
        const int own = f / K, i = f - own * K;
        const int opp = cur.p0 + own / TQ, oqq = cur.q0 + (own - (own / TQ) * TQ);
        if (f < TP * TQ * K && i < kk && opp < Np && oqq < Nq) {
          const int t = cur.t0 + i;
          gD[(g.sign > 0 ? t : Na - 1 - t) + opp * g.sp + oqq * g.sq] = Res[own * SCR + i];
        }
      }
      // Res is rewritten only after the next item's staging barrier.
      if (has_next) stage(nxt);
    }
    cur = nxt;
  }
  if (g.converge && __syncthreads_or(chg) && tid == 0)
    __hip_atomic_store(words + kWordChanged, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Requested mode RMODE falls back to the general formula when the image
// classification word rules the fast edge cost out.
template <bool SCANC, int RMODE, bool REC, int TT = kCellTP, int KC = kCellK, int FMT = kImgF32>
__device__ __forceinline__ bool run_pass_cell_mode(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                   const unsigned* cls_word, unsigned long long limit,
                                                   const CellLds& lds, int wg, int G) {
  if (RMODE == kModeGeneral) {
    if (general_n_ok(gp->sqrt_normal, cls_word))
      return run_pass_cell<SCANC, kModeGeneralN, REC, TT, KC, FMT>(gp, xbuf, words, limit, lds, wg, G);
    return run_pass_cell<SCANC, kModeGeneral, REC, TT, KC, FMT>(gp, xbuf, words, limit, lds, wg, G);
  }
  const bool fast = fast_mode_ok(RMODE, ld_relaxed(cls_word));
  if (fast) return run_pass_cell<SCANC, RMODE, REC, TT, KC, FMT>(gp, xbuf, words, limit, lds, wg, G);
  return run_pass_cell<SCANC, kModeGeneral, REC, TT, KC, FMT>(gp, xbuf, words, limit, lds, wg, G);
}

// Layout and requested mode chosen at run time (batched launches).
template <bool REC, int TT = kCellTP, int KC = kCellK>
__device__ __forceinline__ bool run_pass_cell_rt(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                 const unsigned* cls_word, int mode, unsigned long long limit,
                                                 const CellLds& lds, int wg, int G) {
  if (gp->sa == 1) {
    if (mode == kModeLam0)
      return run_pass_cell_mode<true, kModeLam0, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
    if (mode == kModeLam1C1)
      return run_pass_cell_mode<true, kModeLam1C1, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
    return run_pass_cell_mode<true, kModeGeneral, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
  }
  if (mode == kModeLam0)
    return run_pass_cell_mode<false, kModeLam0, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
  if (mode == kModeLam1C1)
    return run_pass_cell_mode<false, kModeLam1C1, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
  return run_pass_cell_mode<false, kModeGeneral, REC, TT, KC>(gp, xbuf, words, cls_word, limit, lds, wg, G);
}

}  // namespace dev
}  // namespace ggdt
