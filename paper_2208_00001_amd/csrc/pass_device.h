// Device code of one directional pass (shared by the single-instance and the
// batched kernels).
//
// One launch runs one directional pass (FastGeodis paper, section
// "Implementation": a row (2D) or plane (3D) is updated in parallel from the
// previous one, so values propagate along the pass direction).  The launch is
// persistent along the scan axis: the plane is cut into TP x TQ tiles, each tile
// owned by one workgroup, and the scan axis into chunks of K steps.
//
// Per chunk a workgroup
//   1. copies the chunk's image and D_old planes on its tile grown by K (only the
//      cells the shrinking halo needs) straight from global memory into LDS;
//   2. reads the plane finished by the previous chunk on the grown tile from the
//      exchange words its neighbours (and itself) published;
//   3. advances the chunk's planes with one workgroup barrier per plane,
//      recomputing a halo that shrinks by one voxel per plane, so that no other
//      workgroup is consulted inside the chunk;
//   4. publishes its last plane as exchange words.
//
// Exchange words are 64-bit (epoch << 32 | value bits), written and read with
// device-scope relaxed atomics.  A word is valid when its epoch matches, so no
// fence or separate flag is needed.  Slots alternate with the chunk parity: a
// neighbour cannot run two chunks ahead of a reader, so it never overwrites a
// slot that is still to be read.
//
// Halo voxels read D_old from memory that the owning neighbour may be
// overwriting in the same chunk.  Either value gives the same result: the
// neighbour writes min(D_old, candidates) and this workgroup takes min(read
// value, the same candidates), so the halo value it recomputes is identical bit
// for bit.
#pragma once

#include "ggdt_internal.h"
#include "sqrt_fix.h"

namespace ggdt {
namespace dev {


// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Give every
// XCD a contiguous range of logical ids so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, r = b >> 3;
  const int base = G >> 3, extra = G & 7;
  return x * base + min(x, extra) + r;
}

// A pointer into global memory, typed as such.  Pointers read out of a
// descriptor table in memory (the batched launches) carry no address space,
// and accesses through them compile to generic FLAT instructions; those also
// count against the LDS wait counter, so every LDS barrier would then wait for
// the global stores in flight.
template <class T>
using gmem = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gmem<T> to_gmem(T* p) {
  return (gmem<T>)p;
}

// Element type of an image format and its exact widening to fp32.
template <int FMT>
struct ImgElem {
  using T = float;
};
template <>
struct ImgElem<kImgBF16> {
  using T = uint16_t;
};
template <>
struct ImgElem<kImgF16> {
  using T = uint16_t;
};
template <int FMT>
__device__ __forceinline__ float widen(typename ImgElem<FMT>::T v) {
  if constexpr (FMT == kImgBF16) return __uint_as_float((unsigned)v << 16);
  else if constexpr (FMT == kImgF16) return (float)__builtin_bit_cast(_Float16, v);
  else return v;
}
// The image of a pass descriptor as an array of its storage format.
template <int FMT>
__device__ __forceinline__ gmem<const typename ImgElem<FMT>::T> image_of(const float* image) {
  return (gmem<const typename ImgElem<FMT>::T>)(const typename ImgElem<FMT>::T*)(const void*)image;
}

__device__ __forceinline__ unsigned ld_relaxed(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld64_relaxed(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st64_relaxed(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier that orders LDS only.  Steps inside a chunk exchange values
// through LDS; their global stores are read by nobody in the workgroup, so the
// barrier must not wait for them (a full __syncthreads would put a store round
// trip on every step of the serial scan).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Distance of (pp, qq) outside the tile [p0, p0+TP) x [q0, q0+TQ) (Chebyshev, 0 inside).
template <int NDIM, int TP, int TQ>
__device__ __forceinline__ int outside(int pp, int qq, int p0, int q0) {
  const int dq = max(max(q0 - qq, qq - (q0 + TQ - 1)), 0);
  if (NDIM == 2) return dq;
  const int dp = max(max(p0 - pp, pp - (p0 + TP - 1)), 0);
  return max(dp, dq);
}

// Correctly rounded square root of x in [2^-96, FLT_MAX]: the hardware root
// (within one ulp) corrected to the nearest (sqrt_round_fix).  In this range it
// returns the bits of sqrtf as built here (the correctly rounded lowering
// scales only arguments below 2^-96 and special-cases only zero and infinity).
__device__ __forceinline__ float sqrt_rn_normal(float x) { return sqrt_round_fix(x, __builtin_amdgcn_sqrtf(x)); }

// sqrtf(x) for the general modes.
template <int MODE>
__device__ __forceinline__ float general_root(float x) {
  return MODE == kModeGeneralN ? sqrt_rn_normal(x) : sqrtf(x);
}

// A descriptor whose arrays lie in the workspace (batched launches: the
// scan-major copies) gives them as byte offsets from the workspace base,
// `words`; the pointers are filled in here.
__device__ __forceinline__ PassDesc resolve_offsets(PassDesc g, unsigned* words) {
  unsigned char* ws = reinterpret_cast<unsigned char*>(words);
  if (g.image_off >= 0) g.image = reinterpret_cast<const float*>(ws + g.image_off);
  if (g.d_off >= 0) g.D = reinterpret_cast<float*>(ws + g.d_off);
  if (g.rec_off >= 0) g.rec = reinterpret_cast<uint8_t*>(ws + g.rec_off);
  return g;
}

// Mode for a pass whose requested mode RMODE is the general one: the
// normal-range root when the spatial terms keep the argument at least 2^-96
// and no image value is huge, or when they are all 0 (lambda 1: the argument
// is g, a sum of squared channel differences) and no value is small or huge:
// every non-zero difference is then at least 2^-47, so g is 0 (whose root
// kModeGeneralN also gives exactly) or in [2^-94, 2^126].
__device__ __forceinline__ bool general_n_ok(int sqrt_normal, const unsigned* cls_word) {
  const unsigned cls = ld_relaxed(cls_word);
  if (sqrt_normal == kSqrtNormalUnlessHuge) return (cls & kClassHuge) == 0u;
  if (sqrt_normal == kSqrtNormalLam1) return (cls & (kClassHuge | kClassSmall)) == 0u;
  return false;
}

// The fast modes' condition on the classification: w = |I(x) - I(y)| (lambda 1,
// one channel) needs no tiny and no huge value; w = sqrtf(A_j) (lambda 0) no
// huge value.
__device__ __forceinline__ bool fast_mode_ok(int mode, unsigned cls) {
  return mode == kModeLam0 ? (cls & kClassHuge) == 0u : (cls & (kClassTiny | kClassHuge)) == 0u;
}

template <int MODE>
__device__ __forceinline__ float edge_cost(const PassDesc& g, int j, float ix0, float iy0, const float* sx,
                                           const float* sy, int cstride) {
  if (MODE == kModeLam0) {
    return g.W0[j];
  } else if (MODE == kModeLam1C1) {
    return fabsf(ix0 - iy0);
  } else {
    const float d0 = ix0 - iy0;
    float s = d0 * d0;
    for (int c = 1; c < g.C; ++c) {
      const float dc = sx[c * cstride] - sy[c * cstride];
      s = fmaf(dc, dc, s);
    }
    return general_root<MODE>(fmaf(g.lam, s, g.A[j]));
  }
}

// One directional pass of one instance, run by workgroup `wg` of the G
// workgroups given to the instance.  Returns false if a bounded wait gave up.
template <int NDIM, int TP, int TQ, int K, bool SCANC, int MODE, bool REC, int NT = kThreads>
__device__ __forceinline__ bool run_pass(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                         unsigned long long limit, float* lds, int wg, int G) {
  const PassDesc g = resolve_offsets(*gp, words);  // uniform copy: no aliasing with the stores below
  // global-memory views of the descriptor's arrays
  const gmem<const float> gImage = to_gmem(g.image);
  const gmem<const float> gMask = to_gmem(g.mask);
  const gmem<float> gD = to_gmem(g.D);
  const gmem<uint8_t> gRec = to_gmem(g.rec);
  using L = Layout<NDIM, TP, TQ, K, SCANC>;
  constexpr int BQ = L::BQ, NB = L::NB, SC = L::SC, SCR = L::SCR, STAGE = L::STAGE;
  const int tid = threadIdx.x;
  const int wave0 = tid & ~63;
  // Previous/current plane as (D, I(channel 0)) pairs: one 8-byte LDS read per neighbour.
  float2* const Pbuf0 = reinterpret_cast<float2*>(lds);
  float2* const Pbuf1 = Pbuf0 + NB;
  float* const StD = lds + 4 * NB;
  float* const StI = StD + STAGE;  // C arrays of STAGE floats
  float* const Res = StI + STAGE * g.C;
  const int ntiles = g.ntp * g.ntq;
  const int Np = g.Np, Nq = g.Nq, Na = g.Na;
  const bool use_img = MODE != kModeLam0;
  const int nch = (MODE == kModeGeneral || MODE == kModeGeneralN) ? g.C : (use_img ? 1 : 0);
  // 16-byte global->LDS copies need q contiguous and every row start 16-byte aligned.
  const bool vec4 = g.sq == 1 && (g.Nq & 3) == 0 && (g.sp & 3) == 0 && (g.sa & 3) == 0;
  // The same for the scan-contiguous layout: aligned runs along the scan axis.
  const bool vec4s = g.sa == 1 && (Na & 3) == 0 && (g.sp & 3) == 0 && (g.sq & 3) == 0;


  // First plane in scan order: never changed by the pass.  Written once when the
  // pass also initialises D, recorded as "keep" when records are asked for.
  if (g.init || REC) {
    const int kf = g.sign > 0 ? 0 : Na - 1;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int rp = min(TP, Np - p0), rq = min(TQ, Nq - q0);
      for (int f = tid; f < rp * rq; f += NT) {
        const int r = f / rq, cq = f - r * rq;
        const int x = kf * g.sa + (p0 + r) * g.sp + (q0 + cq) * g.sq;
        if (g.init) gD[x] = g.v * gMask[x];
        if (REC && g.rec) gRec[x] = 0;
      }
    }
  }

  int chg = 0;  // an own cell of this workgroup was lowered (convergence mode)
  for (int c = 0; c < g.nchunk; ++c) {
    const int t0 = 1 + c * K;
    const int kk = min(K, Na - t0);
    const unsigned epoch_in = g.epoch_base + (unsigned)c;  // published by chunk c - 1
    const unsigned epoch_out = epoch_in + 1u;
    // Cell-major staging: memory positions kb .. kb + SC - 1 along the scan axis,
    // kb the lowest position of the chunk's planes rounded down to a multiple of 4.
    // Plane j (scan position t0 - 1 + j) sits in slot sbase + sign * j.
    const int kmin = g.sign > 0 ? t0 - 1 : Na - t0 - kk;
    const int kb = kmin & ~3;
    const int sbase = g.sign > 0 ? t0 - 1 - kb : Na - t0 - kb;
    auto sidx = [&](int j, int lx) { return SCANC ? lx * SC + sbase + g.sign * j : j * NB + lx; };
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int bp0 = (NDIM == 3) ? p0 - K : 0;
      const int bq0 = q0 - K;
      // the thread index, opaque to the optimiser: per-thread index math of the
      // unrolled loops below is recomputed per tile instead of being hoisted
      // out of the chunk loop and held in registers for the whole pass
      int tid = threadIdx.x;
      __asm__ volatile("" : "+v"(tid));

      // 1. Global -> LDS copies of the chunk's planes.  Plane j is scan position
      // t0 - 1 + j.  Cell needed iff its distance outside the tile is <= kk - j.
      // D_old (or the mask, for the initialising pass) for planes j >= 1, and
      // plane 0 too in chunk 0 (the pass's unchanged first plane); the image for
      // all planes.
      {
        const gmem<const float> dsrc = g.init ? gMask : (gmem<const float>)gD;
        if (!SCANC && vec4) {
          // 16-byte groups of 4 cells along q (the contiguous axis): groups never
          // straddle the plane edge because q0 - K and Nq are multiples of 4.
          constexpr int NG = STAGE / 4;
          for (int g0 = 0; g0 < NG; g0 += NT) {
            const int gi = g0 + tid;
            const int j = gi / (NB / 4);
            const int lx = 4 * (gi - j * (NB / 4));
            const int br = lx / BQ, bc = lx - br * BQ;
            const int pp = bp0 + br, qq = bq0 + bc;
            bool ok = gi < NG && j <= kk && qq >= 0 && qq + 3 < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
            ok = ok && min(outside<NDIM, TP, TQ>(pp, qq, p0, q0), outside<NDIM, TP, TQ>(pp, qq + 3, p0, q0)) <= kk - j;
            if (ok) {
              const int t = t0 - 1 + j;
              const int k = g.sign > 0 ? t : Na - 1 - t;
              const int x = k * g.sa + pp * g.sp + qq;
              if (j >= 1 || c == 0) __builtin_amdgcn_global_load_lds(dsrc + x, StD + 4 * (g0 + wave0), 16, 0, 0);
              for (int ch = 0; ch < nch; ++ch)
                __builtin_amdgcn_global_load_lds(gImage + (long long)ch * g.N + x, StI + ch * STAGE + 4 * (g0 + wave0),
                                                 16, 0, 0);
            }
          }
        } else if (SCANC && vec4s) {
          // Cell-major 16-byte groups of 4 consecutive scan positions; with Na a
          // multiple of 4 a group is either wholly inside the axis or wholly past
          // its end.
          constexpr int GPC = SC / 4;  // groups per cell
          constexpr int NG = STAGE / 4;
          for (int g0 = 0; g0 < NG; g0 += NT) {
            const int gi = g0 + tid;
            const int lx = gi / GPC, gg = gi - lx * GPC;
            const int br = lx / BQ, bc = lx - br * BQ;
            const int pp = bp0 + br, qq = bq0 + bc;
            const int k0 = kb + 4 * gg;
            bool ok = gi < NG && k0 + 3 <= Na - 1 && qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
            // planes j held by this group
            const int jlo = g.sign > 0 ? k0 - (t0 - 1) : (Na - t0) - (k0 + 3);
            const int jhi = jlo + 3;
            const int jtop = min(jhi, kk - outside<NDIM, TP, TQ>(pp, qq, p0, q0));
            if (ok) {
              const int x = k0 + pp * g.sp + qq * g.sq;
              if (max(jlo, c == 0 ? 0 : 1) <= jtop)
                __builtin_amdgcn_global_load_lds(dsrc + x, StD + 4 * (g0 + wave0), 16, 0, 0);
              if (max(jlo, 0) <= jtop)
                for (int ch = 0; ch < nch; ++ch)
                  __builtin_amdgcn_global_load_lds(gImage + (long long)ch * g.N + x,
                                                   StI + ch * STAGE + 4 * (g0 + wave0), 16, 0, 0);
            }
          }
        } else {
          for (int f0 = 0; f0 < STAGE; f0 += NT) {
            const int f = f0 + tid;
            int j, lx, k;
            if (SCANC) {
              lx = f / SC;
              const int sl = f - lx * SC;
              k = kb + sl;
              j = g.sign > 0 ? k - (t0 - 1) : (Na - t0) - k;
            } else {
              j = f / NB;
              lx = f - j * NB;
              const int t = t0 - 1 + j;
              k = g.sign > 0 ? t : Na - 1 - t;
            }
            const int br = lx / BQ, bc = lx - br * BQ;
            const int pp = bp0 + br, qq = bq0 + bc;
            bool ok = f < STAGE && j >= 0 && j <= kk && qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
            ok = ok && outside<NDIM, TP, TQ>(pp, qq, p0, q0) <= kk - j;
            if (ok) {
              const int x = k * g.sa + pp * g.sp + qq * g.sq;
              if (j >= 1 || c == 0) __builtin_amdgcn_global_load_lds(dsrc + x, StD + f0 + wave0, 4, 0, 0);
              for (int ch = 0; ch < nch; ++ch)
                __builtin_amdgcn_global_load_lds(gImage + (long long)ch * g.N + x, StI + ch * STAGE + f0 + wave0, 4,
                                                 0, 0);
            }
          }
        }
      }

      // 2. The plane before the chunk on the tile grown by kk: exchange words of
      // the previous chunk (chunk 0: the staged first plane of the pass).
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
          lxs[n] = ok ? lx : -1;
          if (ok) {
            const int otp = (NDIM == 3) ? pp / TP : 0, otq = qq / TQ;
            const int slot = (NDIM == 3 ? (pp - otp * TP) * TQ : 0) + (qq - otq * TQ);
            wv[n] = ld64_relaxed(xin + (size_t)(otp * g.ntq + otq) * (TP * TQ) + slot);
          }
        }
        int fail = 0;
#pragma unroll
        for (int n = 0; n < MAXB; ++n) {
          if (lxs[n] < 0) continue;
          const int lx = lxs[n];
          if ((unsigned)(wv[n] >> 32) != epoch_in && !fail) {
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
        }
        if (__syncthreads_or(fail)) return false;
      }
      __builtin_amdgcn_s_waitcnt(0);  // the global->LDS copies have landed
      __syncthreads();
      // Pair plane 0: (D, I) of the border plane; cells outside the plane hold
      // +inf, so a candidate through them never wins and the candidate loop
      // needs no bounds checks.
#pragma unroll
      for (int n = 0; n < MAXB; ++n) {
        const int lx = tid + n * NT;
        if (lx >= NB) break;
        const int br = lx / BQ, bc = lx - br * BQ;
        const int pp = bp0 + br, qq = bq0 + bc;
        const bool in = qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
        float d = __builtin_inff();
        if (in) {
          if (c > 0) {
            if (lxs[n] >= 0) d = __uint_as_float((unsigned)wv[n]);
          } else {
            const float m = StD[sidx(0, lx)];
            d = g.init ? g.v * m : m;
          }
        }
        Pbuf0[lx] = make_float2(d, use_img ? StI[sidx(0, lx)] : 0.0f);
        Pbuf1[lx] = make_float2(__builtin_inff(), 0.0f);
      }
      lds_barrier();

      // 3. Advance the chunk's planes.
      float2* Pp = Pbuf0;
      float2* Pc = Pbuf1;
      unsigned long long* xout = xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)tile * (TP * TQ);
      for (int i = 0; i < kk; ++i) {
        const int t = t0 + i;
        const int k = g.sign > 0 ? t : Na - 1 - t;
        const int h = kk - 1 - i;
        const int lp = (NDIM == 3) ? max(0, p0 - h) : 0;
        const int hp = (NDIM == 3) ? min(Np, p0 + TP + h) : 1;
        const int lq = max(0, q0 - h), hq = min(Nq, q0 + TQ + h);
        const int rq = hq - lq, cnt = (hp - lp) * rq;
        const float inv_rq = 1.0f / (float)rq;
        // Up to U cells per thread in one block: all their LDS reads are issued
        // before any is consumed, so a plane costs about one LDS round trip.
        constexpr int U = (NB + NT - 1) / NT;
        const int nu = (cnt + NT - 1) / NT;  // uniform
        int lxs[U], pps[U], qqs[U];
        float dold[U], ix0[U];
        float2 nb[U][9];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u >= nu) break;
          const int f0 = tid + u * NT;
          const int f = f0 < cnt ? f0 : cnt - 1;
          int r, cq;
          if (NDIM == 3) {
            r = (int)(((float)f + 0.5f) * inv_rq);
            cq = f - r * rq;
          } else {
            r = 0;
            cq = f;
          }
          pps[u] = lp + r;
          qqs[u] = lq + cq;
          const int lx = (pps[u] - bp0) * BQ + (qqs[u] - bq0);
          lxs[u] = lx;
          dold[u] = StD[sidx(i + 1, lx)];
          ix0[u] = use_img ? StI[sidx(i + 1, lx)] : 0.0f;
#pragma unroll
          for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp)
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) nb[u][(NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1] = Pp[lx + dp * BQ + dq];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u >= nu) break;
          if (tid + u * NT >= cnt) continue;
          const int lx = lxs[u], pp = pps[u], qq = qqs[u];
          float best = g.init ? g.v * dold[u] : dold[u];
          const float before = best;
          int choice = 0;
          const float* sx = StI + sidx(i + 1, lx);
          const float* sy = StI + sidx(i, lx);
#pragma unroll
          for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp) {
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) {
              const int j = (NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1;
              const int off = dp * BQ + dq;
              const float w = edge_cost<MODE>(g, j, ix0[u], nb[u][j].y, sx, sy + (SCANC ? off * SC : off), STAGE);
              const float cand = nb[u][j].x + w;
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
          Pc[lx] = make_float2(best, ix0[u]);
          if (pp >= p0 && pp < p0 + TP && qq >= q0 && qq < q0 + TQ) {
            chg |= best < before;
            const int own = (NDIM == 3 ? (pp - p0) * TQ : 0) + (qq - q0);
            const int x = k * g.sa + pp * g.sp + qq * g.sq;
            if (SCANC)
              Res[own * SCR + i] = best;
            else
              gD[x] = best;
            if (REC && g.rec) gRec[x] = (uint8_t)choice;
            if (i == kk - 1)
              st64_relaxed(xout + own, ((unsigned long long)epoch_out << 32) | __float_as_uint(best));
          }
        }
        lds_barrier();
        float2* tP = Pp;
        Pp = Pc;
        Pc = tP;
      }

      // 4. Cell-major results: write each cell's run of scan positions.
      if (SCANC) {
        const int rp = (NDIM == 3) ? min(TP, Np - p0) : 1;
        const int rq = min(TQ, Nq - q0);
        for (int f = tid; f < TP * TQ * SCR; f += NT) {
          const int own = f / SCR, i = f - own * SCR;
          const int r = (NDIM == 3) ? own / TQ : 0, cq = own - r * TQ;
          if (i < kk && r < rp && cq < rq) {
            const int t = t0 + i;
            const int k = g.sign > 0 ? t : Na - 1 - t;
            gD[k * g.sa + (p0 + r) * g.sp + (q0 + cq) * g.sq] = Res[f];
          }
        }
        // Res is rewritten only after the next chunk's first barrier.
      }
    }
  }
  if (g.converge && __syncthreads_or(chg) && threadIdx.x == 0)
    __hip_atomic_store(words + kWordChanged, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Requested mode RMODE falls back to the general formula when the image
// classification word rules the fast edge cost out.
template <int NDIM, int TP, int TQ, int K, bool SCANC, int RMODE, bool REC, int NT = kThreads>
__device__ __forceinline__ bool run_pass_mode(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                              const unsigned* cls_word, unsigned long long limit, float* lds, int wg,
                                              int G) {
  if (RMODE == kModeGeneral) {
    if (general_n_ok(gp->sqrt_normal, cls_word))
      return run_pass<NDIM, TP, TQ, K, SCANC, kModeGeneralN, REC, NT>(gp, xbuf, words, limit, lds, wg, G);
    return run_pass<NDIM, TP, TQ, K, SCANC, kModeGeneral, REC, NT>(gp, xbuf, words, limit, lds, wg, G);
  }
  const bool fast = fast_mode_ok(RMODE, ld_relaxed(cls_word));
  if (fast) return run_pass<NDIM, TP, TQ, K, SCANC, RMODE, REC, NT>(gp, xbuf, words, limit, lds, wg, G);
  return run_pass<NDIM, TP, TQ, K, SCANC, kModeGeneral, REC, NT>(gp, xbuf, words, limit, lds, wg, G);
}

}  // namespace dev
}  // namespace ggdt
