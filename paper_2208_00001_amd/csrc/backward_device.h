// Device code of the reverse of one directional pass (the backward of the
// recorded forward schedule).
//
// A forward pass along axis a, direction s, set D(x) = D(y) + w(x, y) for every
// x whose record names a parent y in the previous plane (record 0: x kept its
// value).  Its reverse walks the planes against the scan order.  For the
// parent plane Y of a child plane X:
//   abar(y) += abar(x_j)                      for each child x_j = y - delta_j in X
//                                             whose record is 1 + j, j ascending
//   Ibar(y) -= coef(x_j) * (I(x_j) - I(y))    for the same children, j ascending,
//              coef = (abar(x_j) * lambda) / w(x_j, y)   (0 when w = 0)
//   Ibar(y) += coef(y) * (I(y) - I(y'))       when y itself has a parent y'
//   abar_out(y) = record(y) ? 0 : abar(y)
// The plane-to-plane recurrence has the same 3x3 cone as the forward pass, so
// the same overlapped tiling is used: chunks of K planes, a tile grown by K whose
// halo shrinks by one voxel per plane, and 64-bit (epoch, value) exchange words
// for the state (abar of the chunk's last parent plane, before zeroing).
// abar is read from one buffer and written to another (a sum cannot tolerate
// reading a neighbour's already-updated value); Ibar is only touched by the
// tile that owns the voxel.
#pragma once

#include "pass_device.h"

namespace ggdt {
namespace dev {

template <int NDIM, int TP, int TQ, int K, bool SCANC>
struct BLayout {
  static constexpr int BQ = TQ + 2 * K;
  static constexpr int BP = NDIM == 3 ? TP + 2 * K : 1;
  static constexpr int NB = BP * BQ;
  static constexpr int P = K + 2;                   // staged planes m = 0 .. K+1
  static constexpr int SC = 4 * ((P + 3 + 3) / 4);  // cell-major run (P planes + up to 3 alignment slots)
  static constexpr int STAGE = SCANC ? NB * SC : NB * P;
  static constexpr int OWN = TP * TQ;
  // state ping-pong, staged abar_in and image (C), own Ibar (K planes x C), records (bytes)
  static constexpr size_t bytes(int C) {
    return sizeof(float) * (size_t)(2 * NB + STAGE * (1 + C) + OWN * K * C) + (size_t)STAGE;
  }
};

__device__ __forceinline__ float pick(bool c, float x, float y) { return c ? x : y; }

// A[j] for a j known only at run time (taken from a record), by an unrolled
// select of values: indexing the array directly (or selecting between array
// elements as lvalues) would move the descriptor copy to private scratch memory.
__device__ __forceinline__ float spatial_term(const BwdDesc& g, int j) {
  float a = g.A[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) a = pick(j == k, g.A[k], a);
  return a;
}

// Edge cost w(x, y) through offset j, from the staged image (x and y addresses
// of channel 0; channels are `cstride` apart).
template <int MODE>
__device__ __forceinline__ float bwd_edge(const BwdDesc& g, int j, const float* sx, const float* sy, int cstride) {
  const float d0 = sx[0] - sy[0];
  if (MODE == kModeLam1C1) return fabsf(d0);
  float s = d0 * d0;
  for (int c = 1; c < g.C; ++c) {
    const float dc = sx[c * cstride] - sy[c * cstride];
    s = fmaf(dc, dc, s);
  }
  return general_root<MODE>(fmaf(g.lam, s, spatial_term(g, j)));
}

template <int NDIM, int TP, int TQ, int K, bool SCANC, int MODE, int NT = kThreads>
__device__ __forceinline__ bool run_bwd_pass(const BwdDesc* gp, unsigned long long* xbuf, unsigned* words,
                                             unsigned long long limit, float* lds, int wg, int G) {
  using L = BLayout<NDIM, TP, TQ, K, SCANC>;
  constexpr int BQ = L::BQ, NB = L::NB, SC = L::SC, STAGE = L::STAGE, OWN = L::OWN;
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
  const int wave0 = tid & ~63;
  float* const Sbuf0 = lds;
  float* const Sbuf1 = lds + NB;
  float* const StA = lds + 2 * NB;
  float* const StI = StA + STAGE;
  float* const StG = StI + STAGE * g.C;
  unsigned char* const StR = reinterpret_cast<unsigned char*>(StG + OWN * K * g.C);
  const int ntiles = g.ntp * g.ntq;
  const int Np = g.Np, Nq = g.Nq, Na = g.Na;
  constexpr bool USE_I = MODE != kModeLam0;
  const int nch = USE_I ? ((MODE == kModeGeneral || MODE == kModeGeneralN) ? g.C : 1) : 0;

  // Last plane of the forward scan (never a parent plane): its own terms.
  {
    const int kl = g.sign > 0 ? Na - 1 : 0;
    const int kpar = kl - g.sign;  // parent plane (exists when Na > 1)
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int rp = min(TP, Np - p0), rq = min(TQ, Nq - q0);
      for (int f = tid; f < rp * rq; f += NT) {
        const int r = f / rq, cq = f - r * rq;
        const int pp = p0 + r, qq = q0 + cq;
        const int x = kl * g.sa + pp * g.sp + qq * g.sq;
        const float a = gAin[x];
        const int rc = gRec[x];
        const int j = rc - 1;
        const int dp = NDIM == 3 ? j / 3 - 1 : 0, dq = (NDIM == 3 ? j % 3 : j) - 1;
        // a parent outside the grid only comes from records of another schedule: skip it
        const bool par_ok = rc >= 1 && rc <= (NDIM == 3 ? 9 : 3) && Na > 1 && pp + dp >= 0 && pp + dp < Np &&
                            qq + dq >= 0 && qq + dq < Nq;
        if (USE_I && par_ok) {
          const int y = kpar * g.sa + (pp + dp) * g.sp + (qq + dq) * g.sq;
          const float d0 = gImage[x] - gImage[y];
          float w;
          if (MODE == kModeLam1C1) {
            w = fabsf(d0);
          } else {
            float s = d0 * d0;
            for (int c = 1; c < g.C; ++c) {
              const float dc = gImage[(long long)c * g.N + x] - gImage[(long long)c * g.N + y];
              s = fmaf(dc, dc, s);
            }
            w = general_root<MODE>(fmaf(g.lam, s, spatial_term(g, j)));
          }
          if (w > 0.0f) {
            const float coef = (a * g.lam) / w;
            for (int c = 0; c < g.C; ++c) {
              const float dc = gImage[(long long)c * g.N + x] - gImage[(long long)c * g.N + y];
              gGI[(long long)c * g.N + x] = gGI[(long long)c * g.N + x] + coef * dc;
            }
          }
        }
        gAout[x] = rc != 0 ? 0.0f : a;
      }
    }
  }

  for (int c = 0; c < g.nchunk; ++c) {
    // Chunk c walks scan positions T0, T0-1, ..., T1 as child planes.
    const int T0 = Na - 1 - c * K;
    const int kk = min(K, T0);
    const unsigned epoch_in = g.epoch_base + (unsigned)c;
    const unsigned epoch_out = epoch_in + 1u;
    // staged plane m is scan position T0 - m (m = 0 .. kk+1; the last may not exist)
    const int mtop = min(kk + 1, T0);
    const int kmin = g.sign > 0 ? T0 - mtop : Na - 1 - T0;
    const int kb = kmin & ~3;
    const int sbase = g.sign > 0 ? T0 - kb : Na - 1 - T0 - kb;
    const int sstep = -g.sign;
    auto sidx = [&](int m, int lx) { return SCANC ? lx * SC + sbase + sstep * m : m * NB + lx; };
    auto kof = [&](int m) { const int t = T0 - m; return g.sign > 0 ? t : Na - 1 - t; };

    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int bp0 = (NDIM == 3) ? p0 - K : 0;
      const int bq0 = q0 - K;
      // the thread index, opaque to the optimiser: per-thread index math of the
      // unrolled staging loops below is then recomputed per tile instead of being
      // hoisted out of the chunk loop and held in registers for the whole pass
      int tid = threadIdx.x;
      __asm__ volatile("" : "+v"(tid));

      // 1. abar_in (m = 1..kk, and m = 0 in chunk 0) and the image (m = 0..mtop)
      // into LDS; expansion of plane m is kk - m (image: at least 1).
      for (int f0 = 0; f0 < STAGE; f0 += NT) {
        const int f = f0 + tid;
        int m, lx, k;
        if (SCANC) {
          lx = f / SC;
          const int sl = f - lx * SC;
          k = kb + sl;
          const int t = g.sign > 0 ? k : Na - 1 - k;
          m = T0 - t;
        } else {
          m = f / NB;
          lx = f - m * NB;
          k = kof(m);
        }
        const int br = lx / BQ, bc = lx - br * BQ;
        const int pp = bp0 + br, qq = bq0 + bc;
        const bool in = f < STAGE && m >= 0 && m <= mtop && k >= 0 && k < Na && qq >= 0 && qq < Nq &&
                        (NDIM == 2 || (pp >= 0 && pp < Np));
        const int e = in ? outside<NDIM, TP, TQ>(pp, qq, p0, q0) : 0;
        const int x = in ? k * g.sa + pp * g.sp + qq * g.sq : 0;
        if (in && m <= kk && (m >= 1 || c == 0) && e <= kk - m)
          __builtin_amdgcn_global_load_lds(gAin + x, StA + f0 + wave0, 4, 0, 0);
        if (in && e <= max(kk - m, 1))
          for (int ch = 0; ch < nch; ++ch)
            __builtin_amdgcn_global_load_lds(gImage + (long long)ch * g.N + x, StI + ch * STAGE + f0 + wave0, 4, 0,
                                             0);
      }
      // records (m = 0..kk) through registers, in batches of RB byte loads
      // issued together before their LDS stores (the batch bounds the registers
      // held); out-of-plane and unneeded cells read as 0 ("kept").
      constexpr int NR = (STAGE + NT - 1) / NT;
      constexpr int RB = NR < 8 ? NR : 8;
      for (int n0 = 0; n0 < NR; n0 += RB) {
        unsigned rv[RB];
#pragma unroll
        for (int n1 = 0; n1 < RB; ++n1) {
          const int f = (n0 + n1) * NT + tid;
          int m, lx, k;
          if (SCANC) {
            lx = f / SC;
            const int sl = f - lx * SC;
            k = kb + sl;
            const int t = g.sign > 0 ? k : Na - 1 - k;
            m = T0 - t;
          } else {
            m = f / NB;
            lx = f - m * NB;
            k = kof(m);
          }
          const int br = lx / BQ, bc = lx - br * BQ;
          const int pp = bp0 + br, qq = bq0 + bc;
          const bool in = f < STAGE && m >= 0 && m <= kk && k >= 0 && k < Na && qq >= 0 && qq < Nq &&
                          (NDIM == 2 || (pp >= 0 && pp < Np)) && outside<NDIM, TP, TQ>(pp, qq, p0, q0) <= kk - m;
          rv[n1] = in ? (unsigned)gRec[k * g.sa + pp * g.sp + qq * g.sq] : 0u;
        }
#pragma unroll
        for (int n1 = 0; n1 < RB; ++n1) {
          const int f = (n0 + n1) * NT + tid;
          if (f < STAGE) StR[f] = (unsigned char)rv[n1];
        }
      }
      // own Ibar of the parent planes m = 1..kk
      if (USE_I) {
        for (int f0 = 0; f0 < K * OWN; f0 += NT) {
          const int f = f0 + tid;
          const int mm = f / OWN, own = f - mm * OWN;
          const int r = (NDIM == 3) ? own / TQ : 0, cq = own - r * TQ;
          const int pp = p0 + r, qq = q0 + cq;
          if (mm < kk && pp < Np && qq < Nq) {
            const int x = kof(mm + 1) * g.sa + pp * g.sp + qq * g.sq;
            for (int ch = 0; ch < g.C; ++ch)
              __builtin_amdgcn_global_load_lds(gGI + (long long)ch * g.N + x, StG + ch * K * OWN + f0 + wave0, 4, 0,
                                               0);
          }
        }
      }

      // 2. the state on child plane m = 0: exchange words of chunk c - 1.
      constexpr int MAXB = (NB + NT - 1) / NT;
      unsigned long long wv[MAXB];
      int lxs[MAXB];
#pragma unroll
      for (int n = 0; n < MAXB; ++n) lxs[n] = -1;
      if (c > 0) {
        const unsigned long long* xin = xbuf + (size_t)((c - 1) & 1) * ntiles * (TP * TQ);
#pragma unroll
        for (int n = 0; n < MAXB; ++n) {
          const int lx = tid + n * NT;
          const int br = lx / BQ, bc = lx - br * BQ;
          const int pp = bp0 + br, qq = bq0 + bc;
          bool ok = lx < NB && qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
          ok = ok && outside<NDIM, TP, TQ>(pp, qq, p0, q0) <= kk;
          if (ok) {
            lxs[n] = lx;
            const int otp = (NDIM == 3) ? pp / TP : 0, otq = qq / TQ;
            const int slot = (NDIM == 3 ? (pp - otp * TP) * TQ : 0) + (qq - otq * TQ);
            wv[n] = ld64_relaxed(xin + (size_t)(otp * g.ntq + otq) * (TP * TQ) + slot);
          }
        }
        int fail = 0;
#pragma unroll
        for (int n = 0; n < MAXB; ++n) {
          if (lxs[n] < 0 || (unsigned)(wv[n] >> 32) == epoch_in || fail) continue;
          const int lx = lxs[n];
          const int br = lx / BQ, bc = lx - br * BQ;
          const int pp = bp0 + br, qq = bq0 + bc;
          const int otp = (NDIM == 3) ? pp / TP : 0, otq = qq / TQ;
          const int slot = (NDIM == 3 ? (pp - otp * TP) * TQ : 0) + (qq - otq * TQ);
          const unsigned long long* a = xin + (size_t)(otp * g.ntq + otq) * (TP * TQ) + slot;
          unsigned long long polls = 0;
          while ((unsigned)(wv[n] >> 32) != epoch_in) {
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
            wv[n] = ld64_relaxed(a);
          }
        }
        if (__syncthreads_or(fail)) return false;
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
#pragma unroll
      for (int n = 0; n < MAXB; ++n) {
        const int lx = tid + n * NT;
        if (lx >= NB) break;
        float s = 0.0f;
        if (c > 0) {
          if (lxs[n] >= 0) s = __uint_as_float((unsigned)wv[n]);
        } else {
          s = StA[sidx(0, lx)];
        }
        Sbuf0[lx] = s;
      }
      lds_barrier();

      // 3. parent planes m = i + 1 for i = 0 .. kk-1
      float* Sp = Sbuf0;
      float* Sc = Sbuf1;
      unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)tile * (TP * TQ);
      for (int i = 0; i < kk; ++i) {
        const int ky = kof(i + 1);
        const int h = kk - 1 - i;
        const int lp = (NDIM == 3) ? max(0, p0 - h) : 0;
        const int hp = (NDIM == 3) ? min(Np, p0 + TP + h) : 1;
        const int lq = max(0, q0 - h), hq = min(Nq, q0 + TQ + h);
        const int rq = hq - lq, cnt = (hp - lp) * rq;
        const float inv_rq = 1.0f / (float)rq;
        for (int f = tid; f < cnt; f += NT) {
          int r, cq;
          if (NDIM == 3) {
            r = (int)(((float)f + 0.5f) * inv_rq);
            cq = f - r * rq;
          } else {
            r = 0;
            cq = f;
          }
          const int pp = lp + r, qq = lq + cq;
          const int ly = (pp - bp0) * BQ + (qq - bq0);
          float a = StA[sidx(i + 1, ly)];
          float sj[9];
          int rj[9];
#pragma unroll
          for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp)
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) {
              const int j = (NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1;
              const int lxc = ly - dp * BQ - dq;  // child x_j = y - delta_j
              rj[j] = StR[sidx(i, lxc)];
              sj[j] = Sp[lxc];
            }
#pragma unroll
          for (int j = 0; j < (NDIM == 3 ? 9 : 3); ++j)
            if (rj[j] == 1 + j) a = a + sj[j];
          Sc[ly] = a;
          if (pp >= p0 && pp < p0 + TP && qq >= q0 && qq < q0 + TQ) {
            const int own = (NDIM == 3 ? (pp - p0) * TQ : 0) + (qq - q0);
            const int y = ky * g.sa + pp * g.sp + qq * g.sq;
            const int ry = StR[sidx(i + 1, ly)];
            if (USE_I) {
              float* gy = StG + i * OWN + own;  // channel c at gy[c * K * OWN]
              const float* syI = StI + sidx(i + 1, ly);
#pragma unroll
              for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp)
#pragma unroll
                for (int dq = -1; dq <= 1; ++dq) {
                  const int j = (NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1;
                  if (rj[j] != 1 + j) continue;
                  const int lxc = ly - dp * BQ - dq;
                  const float* sxI = StI + sidx(i, lxc);
                  const float w = bwd_edge<MODE>(g, j, sxI, syI, STAGE);
                  if (w > 0.0f) {
                    const float coef = (sj[j] * g.lam) / w;
                    for (int ch = 0; ch < g.C; ++ch) {
                      const float d = sxI[ch * STAGE] - syI[ch * STAGE];
                      gy[ch * K * OWN] = gy[ch * K * OWN] - coef * d;
                    }
                  }
                }
              if (ry != 0 && i + 2 <= mtop) {
                const int j = ry - 1;
                const int dp = NDIM == 3 ? j / 3 - 1 : 0, dq = (NDIM == 3 ? j % 3 : j) - 1;
                const float* spI = StI + sidx(i + 2, ly + dp * BQ + dq);  // parent y' = y + delta_j
                const float w = bwd_edge<MODE>(g, j, syI, spI, STAGE);
                if (w > 0.0f) {
                  const float coef = (a * g.lam) / w;
                  for (int ch = 0; ch < g.C; ++ch) {
                    const float d = syI[ch * STAGE] - spI[ch * STAGE];
                    gy[ch * K * OWN] = gy[ch * K * OWN] + coef * d;
                  }
                }
              }
              for (int ch = 0; ch < g.C; ++ch) gGI[(long long)ch * g.N + y] = gy[ch * K * OWN];
            }
            gAout[y] = ry != 0 ? 0.0f : a;
            if (i == kk - 1)
              st64_relaxed(xout + own, ((unsigned long long)epoch_out << 32) | __float_as_uint(a));
          }
        }
        lds_barrier();
        float* t = Sp;
        Sp = Sc;
        Sc = t;
      }
    }
  }
  return true;
}

template <int NDIM, int TP, int TQ, int K, bool SCANC, int NT = kThreads>
__device__ __forceinline__ bool run_bwd_pass_mode(const BwdDesc* gp, unsigned long long* xbuf, unsigned* words,
                                                  const unsigned* cls_word, unsigned long long limit, float* lds,
                                                  int wg, int G) {
  const int mode = gp->mode;
  if (mode == kModeLam0) return run_bwd_pass<NDIM, TP, TQ, K, SCANC, kModeLam0, NT>(gp, xbuf, words, limit, lds, wg, G);
  if (mode == kModeLam1C1 && fast_mode_ok(kModeLam1C1, ld_relaxed(cls_word)))
    return run_bwd_pass<NDIM, TP, TQ, K, SCANC, kModeLam1C1, NT>(gp, xbuf, words, limit, lds, wg, G);
  if (mode == kModeGeneral && general_n_ok(gp->sqrt_normal, cls_word))
    return run_bwd_pass<NDIM, TP, TQ, K, SCANC, kModeGeneralN, NT>(gp, xbuf, words, limit, lds, wg, G);
  return run_bwd_pass<NDIM, TP, TQ, K, SCANC, kModeGeneral, NT>(gp, xbuf, words, limit, lds, wg, G);
}

}  // namespace dev
}  // namespace ggdt
