// Device code of the reverse of one single-channel 3D directional pass with one
// thread per cell of the tile box (the backward counterpart of pass_cell.h).
//
// The arithmetic and its order per voxel are those of run_bwd_pass
// (backward_device.h): for a parent plane Y of a child plane X,
//   abar(y) = abar_in(y) + sum over children x_j with record 1 + j (j ascending) of abar(x_j)
//   Ibar(y) -= coef(x_j) * (I(x_j) - I(y)) for the same children, j ascending
//   Ibar(y) += coef(y) * (I(y) - I(y'))     when y has a parent y'
//   abar_out(y) = record(y) ? 0 : abar(y)
// with the same overlapped tiling: 16 x 16 tiles, chunks of K = 8 planes, a
// halo shrinking by one voxel per plane, and epoch-tagged exchange words for the
// chunk's last parent plane.  A workgroup of 1024 threads covers the tile's
// 32 x 32 box, one thread per cell for the whole pass.  A thread keeps its
// cell's abar_in, image, records and (own cells) Ibar for the chunk's planes in
// registers, fetched one work item ahead; per step it reads its children's
// (abar, I, coefficient, record) from LDS, and its parent's image.
//
// coef(x_j) = (abar(x_j) * lambda) / w(x_j, y) is the coefficient of the child's
// own parent edge, which the child computes anyway for its own Ibar term; each
// cell within distance 1 of the tile (the only cells whose coefficient an own
// cell uses) computes it once and publishes it, so the parents' child terms
// need no root or division.  The same operands give the same bits.
#pragma once

#include "backward_device.h"
#include "pass_cell.h"

namespace ggdt {
namespace dev {

// LDS of the reverse pass: two planes of (abar, record bits), two of (I,
// coefficient) (read by own cells only), two image planes (a step's grandparent
// plane), one fail word.
constexpr size_t kBwdCellLdsBytes = sizeof(float2) * 4 * kCellThreads + sizeof(float) * 2 * kCellThreads +
                                    sizeof(int);
// record bits of a published cell: the record (0 or 1 + j), and kCoefValid
// when its parent edge has w > 0 (its coefficient then enters the parent's Ibar)
constexpr int kCoefValid = 0x100;

template <int MODE>
__device__ __forceinline__ float bwd_cell_edge(const BwdDesc& g, int j, float ix, float iy) {
  const float d = ix - iy;
  if (MODE == kModeLam1C1) return fabsf(d);
  return general_root<MODE>(fmaf(g.lam, d * d, g.A[j]));
}

// Same, offset j known only at run time.
template <int MODE>
__device__ __forceinline__ float bwd_cell_edge_rt(const BwdDesc& g, int j, float ix, float iy) {
  const float d = ix - iy;
  if (MODE == kModeLam1C1) return fabsf(d);
  return general_root<MODE>(fmaf(g.lam, d * d, spatial_term(g, j)));
}

template <int MODE>
__device__ __forceinline__ bool run_bwd_pass_cell(const BwdDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                  unsigned long long limit, float* lds, int wg, int G) {
  constexpr int TP = kCellTP, TQ = kCellTQ, K = kCellK, BQ = kCellBQ, NB = kCellThreads;
  BwdDesc g = *gp;
  if (g.a_in_off >= 0) g.a_in = reinterpret_cast<const float*>(reinterpret_cast<unsigned char*>(words) + g.a_in_off);
  if (g.a_out_off >= 0) g.a_out = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(words) + g.a_out_off);
  if (g.image_off >= 0) g.image = reinterpret_cast<const float*>(reinterpret_cast<unsigned char*>(words) + g.image_off);
  if (g.rec_off >= 0) g.rec = reinterpret_cast<const uint8_t*>(reinterpret_cast<unsigned char*>(words) + g.rec_off);
  if (g.gi_off >= 0) g.gI = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(words) + g.gi_off);
  // global-memory views of the descriptor's arrays
  const gmem<const float> gImage = to_gmem(g.image);
  const gmem<const uint8_t> gRec = to_gmem(g.rec);
  const gmem<const float> gAin = to_gmem(g.a_in);
  const gmem<float> gAout = to_gmem(g.a_out);
  const gmem<float> gGI = to_gmem(g.gI);
  const int tid = threadIdx.x;
  const int br = tid / BQ, bc = tid - br * BQ;
  const int e = max(max(max(K - br, br - (K + TP - 1)), max(K - bc, bc - (K + TQ - 1))), 0);
  const int own_slot = (br - K) * TQ + (bc - K);  // valid when e == 0
  const int ntiles = g.ntp * g.ntq;
  if (wg >= ntiles) return true;  // a batched instance may hold more workgroups than tiles
  const int Na = g.Na, Np = g.Np, Nq = g.Nq;
  constexpr bool USE_I = MODE != kModeLam0;
  float2* const S0 = reinterpret_cast<float2*>(lds);  // (abar, record bits)
  float2* const S1 = S0 + NB;
  float2* const V0 = S1 + NB;  // (I, coefficient)
  float2* const V1 = V0 + NB;
  float* const J0 = reinterpret_cast<float*>(V1 + NB);
  float* const J1 = J0 + NB;
  int* const failw = reinterpret_cast<int*>(J1 + NB);
  if (tid == 0) *failw = 0;  // read only after a barrier

  // Last plane of the forward scan (never a parent plane): its own terms.
  {
    const int kl = g.sign > 0 ? Na - 1 : 0;
    const int kpar = kl - g.sign;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int pp = tp * TP - K + br, qq = tq * TQ - K + bc;
      if (e != 0 || pp >= Np || qq >= Nq) continue;
      const int x = kl * g.sa + pp * g.sp + qq * g.sq;
      const float a = gAin[x];
      const int rc = gRec[x];
      const int j = rc - 1;
      const int dp = j / 3 - 1, dq = j % 3 - 1;
      // a parent outside the grid only comes from records of another schedule: skip it
      const bool par_ok = rc >= 1 && rc <= 9 && Na > 1 && pp + dp >= 0 && pp + dp < Np && qq + dq >= 0 &&
                          qq + dq < Nq;
      if (USE_I && par_ok) {
        const int y = kpar * g.sa + (pp + dp) * g.sp + (qq + dq) * g.sq;
        const float ix = gImage[x], iy = gImage[y];
        const float w = bwd_cell_edge_rt<MODE>(g, j, ix, iy);
        if (w > 0.0f) {
          const float coef = (a * g.lam) / w;
          gGI[x] = gGI[x] + coef * (ix - iy);
        }
      }
      gAout[x] = rc != 0 ? 0.0f : a;
    }
  }

  // Work items: chunk-major, then this workgroup's tiles; the next item's
  // values are fetched while the current item's planes are walked.
  const int nmine = (ntiles - wg + G - 1) / G;
  const int nitems = g.nchunk * nmine;
  struct Item {
    int c, T0, kk, mtop, tile, p0, q0, pp, qq, xpq;
    bool in;
  };
  auto item_of = [&](int n) {
    Item it;
    it.c = n / nmine;
    it.tile = wg + (n - it.c * nmine) * G;
    it.T0 = Na - 1 - it.c * K;  // scan position of the chunk's first child plane (m = 0)
    it.kk = min(K, it.T0);
    it.mtop = min(it.kk + 1, it.T0);
    const int tp = it.tile / g.ntq, tq = it.tile - tp * g.ntq;
    it.p0 = tp * TP;
    it.q0 = tq * TQ;
    it.pp = it.p0 - K + br;
    it.qq = it.q0 - K + bc;
    it.in = it.pp >= 0 && it.pp < Np && it.qq >= 0 && it.qq < Nq;
    it.xpq = it.in ? it.pp * g.sp + it.qq * g.sq : 0;
    return it;
  };
  // memory index of plane m of an item (scan position T0 - m)
  auto xof = [&](const Item& it, int m) {
    const int t = it.T0 - m;
    return (g.sign > 0 ? t : Na - 1 - t) * g.sa + it.xpq;
  };
  // Plane m as a child (step m) and as a parent (step m - 1) is used by the
  // cells within distance kk - m; the parent edges of the cells within distance
  // 1 read images one plane further, at distance 2.
  // Records of planes 0..K: fetched one byte per register, kept four to a
  // register for the item being walked.
  constexpr int NRW = (K + 1 + 3) / 4;
  float nA[K + 2], nI[K + 2];
  int nR[K + 1];  // record bytes, unpacked here so that their loads need no early wait
  // (inlined: called twice, and a call would put the captured arrays in memory)
  auto fetch = [&](const Item& it) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m <= K + 1; ++m) {
      const bool in_m = it.in && m <= it.mtop;
      const bool need = in_m && e <= it.kk - m;
      nA[m] = 0.0f;
      nI[m] = 0.0f;
      if (m <= K) nR[m] = 0;
      if (in_m) {
        const int x = xof(it, m);
        if (m <= K && need && m <= it.kk) {
          if (m >= 1 || it.c == 0) nA[m] = gAin[x];
          nR[m] = gRec[x];
        }
        if (USE_I && (need || e <= 2)) nI[m] = gImage[x];
      }
    }
  };
  auto rec_of = [](const unsigned* r, int m) { return (int)((r[m >> 2] >> (8 * (m & 3))) & 0xffu); };

  Item cur = item_of(0);
  fetch(cur);
  for (int n = 0; n < nitems; ++n) {
    const int c = cur.c, kk = cur.kk;
    const unsigned epoch_in = g.epoch_base + (unsigned)c;
    const unsigned epoch_out = epoch_in + 1u;
    const bool has_next = n + 1 < nitems;
    const Item nxt = item_of(has_next ? n + 1 : n);
    float ain[K + 2], ix[K + 2], gi[K + 2];
    unsigned rec[NRW];
#pragma unroll
    for (int m = 0; m <= K + 1; ++m) {
      ain[m] = nA[m];
      ix[m] = nI[m];
      // own Ibar of the parent planes: loaded here, one item later than the
      // rest, so that it costs no registers during the previous item's steps;
      // the exchange wait below covers its latency
      gi[m] = 0.0f;
      if (USE_I && e == 0 && cur.in && m >= 1 && m <= kk) gi[m] = gGI[xof(cur, m)];
    }
#pragma unroll
    for (int w = 0; w < NRW; ++w) rec[w] = 0u;
#pragma unroll
    for (int m = 0; m <= K; ++m) rec[m >> 2] |= (unsigned)nR[m] << (8 * (m & 3));

    // Plane 0 of the chunk: abar_in of the pass's last plane in chunk 0, else
    // the state the previous chunk published (this tile's and its neighbours').
    float s0 = 0.0f;
    int fail = 0;
    if (cur.in && e <= kk) {
      if (c == 0) {
        s0 = ain[0];
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
        s0 = __uint_as_float((unsigned)wv);
      }
    }
    // The parent plane's image for plane 0's parent edges.
    J1[tid] = ix[1];
    if (fail) *failw = n + 1;
    step_barrier();
    if (*failw == n + 1) return false;
    // Plane 0 as children of step 0: coefficients of their parent edges (the
    // same operands as where the previous chunk's owner, or the prologue,
    // computed them).  Cells outside the volume publish zeros: never a child.
    {
      const int r0 = cur.in ? rec_of(rec, 0) : 0;
      float cf = 0.0f;
      int valid = 0;
      if (USE_I && cur.in && e <= 1 && r0 != 0) {
        const int jj = r0 - 1;
        const float iyp = J1[tid + (jj / 3 - 1) * BQ + (jj % 3 - 1)];
        const float w = bwd_cell_edge_rt<MODE>(g, jj, ix[0], iyp);
        if (w > 0.0f) {
          cf = (s0 * g.lam) / w;
          valid = kCoefValid;
        }
      }
      S0[tid] = make_float2(s0, __int_as_float(r0 | valid));
      V0[tid] = make_float2(ix[0], cf);
      J0[tid] = ix[2];
      if (!cur.in) S1[tid] = make_float2(0.0f, __int_as_float(0));
    }
    step_barrier();
    if (has_next) fetch(nxt);

    // Parent planes m = i + 1 for i = 0 .. kk - 1.
    float2* Sc = S0;
    float2* Sn = S1;
    float2* Vc = V0;
    float2* Vn = V1;
    float* Jc = J0;
    float* Jn = J1;
    unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)cur.tile * (TP * TQ);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i >= kk) break;
      if (cur.in && e <= kk - 1 - i) {
        const float iy = ix[i + 1];
        const int ry = rec_of(rec, i + 1);
        float a = ain[i + 1];
        float2 ch[9];  // children x_j = y - delta_j: (abar, record bits)
#pragma unroll
        for (int j = 0; j < 9; ++j) ch[j] = Sc[tid - (j / 3 - 1) * BQ - (j % 3 - 1)];
#pragma unroll
        for (int j = 0; j < 9; ++j)
          if ((__float_as_int(ch[j].y) & 0xff) == 1 + j) a = a + ch[j].x;
        // this cell's parent edge (cells within distance 1 of the tile)
        float cf = 0.0f, iyp = 0.0f;
        int valid = 0;
        if (USE_I && e <= 1 && ry != 0 && i + 2 <= cur.mtop) {
          const int jj = ry - 1;
          iyp = Jc[tid + (jj / 3 - 1) * BQ + (jj % 3 - 1)];  // parent y' = y + delta_jj
          const float w = bwd_cell_edge_rt<MODE>(g, jj, iy, iyp);
          if (w > 0.0f) {
            cf = (a * g.lam) / w;
            valid = kCoefValid;
          }
        }
        if (e == 0) {
          const int x = xof(cur, i + 1);
          if (USE_I) {
            float gy = gi[i + 1];
            float2 v[9];  // (I(x_j), coef(x_j)), read together; applied where the record matches
#pragma unroll
            for (int j = 0; j < 9; ++j) v[j] = Vc[tid - (j / 3 - 1) * BQ - (j % 3 - 1)];
#pragma unroll
            for (int j = 0; j < 9; ++j) {
              const float t = gy - v[j].y * (v[j].x - iy);
              gy = (__float_as_int(ch[j].y) & 0x1ff) == (kCoefValid | (1 + j)) ? t : gy;
            }
            if (valid) gy = gy + cf * (iy - iyp);
            gGI[x] = gy;
          }
          gAout[x] = ry != 0 ? 0.0f : a;
          if (i == kk - 1) st64_relaxed(xout + own_slot, ((unsigned long long)epoch_out << 32) | __float_as_uint(a));
        }
        Sn[tid] = make_float2(a, __int_as_float(ry | valid));
        Vn[tid] = make_float2(iy, cf);
        if (i + 3 <= K + 1) Jn[tid] = ix[i + 3 <= K + 1 ? i + 3 : K + 1];  // grandparent plane of step i + 1
      }
      step_barrier();
      float2* ts = Sc;
      Sc = Sn;
      Sn = ts;
      float2* tv = Vc;
      Vc = Vn;
      Vn = tv;
      float* tj = Jc;
      Jc = Jn;
      Jn = tj;
    }
    cur = nxt;
  }
  return true;
}

__device__ __forceinline__ bool run_bwd_pass_cell_mode(const BwdDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                       const unsigned* cls_word, unsigned long long limit,
                                                       float* lds, int wg, int G) {
  const int mode = gp->mode;
  if (mode == kModeLam0) return run_bwd_pass_cell<kModeLam0>(gp, xbuf, words, limit, lds, wg, G);
  if (mode == kModeLam1C1 && fast_mode_ok(kModeLam1C1, ld_relaxed(cls_word)))
    return run_bwd_pass_cell<kModeLam1C1>(gp, xbuf, words, limit, lds, wg, G);
  if (mode == kModeGeneral && general_n_ok(gp->sqrt_normal, cls_word))
    return run_bwd_pass_cell<kModeGeneralN>(gp, xbuf, words, limit, lds, wg, G);
  return run_bwd_pass_cell<kModeGeneral>(gp, xbuf, words, limit, lds, wg, G);
}

}  // namespace dev
}  // namespace ggdt
