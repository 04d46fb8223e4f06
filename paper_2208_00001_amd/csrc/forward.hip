// Forward directional-pass kernels for gfx950.
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
#include "ggdt_internal.h"

namespace ggdt {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Give every
// XCD a contiguous range of logical ids so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, r = b >> 3;
  const int base = G >> 3, extra = G & 7;
  return x * base + min(x, extra) + r;
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
    return sqrtf(fmaf(g.lam, s, g.A[j]));
  }
}

template <int NDIM, int TP, int TQ, int K, bool SCANC, int MODE, bool REC>
__device__ bool run_pass(const PassDesc& g, unsigned* words, unsigned long long limit, float* lds) {
  using L = Layout<NDIM, TP, TQ, K, SCANC>;
  constexpr int BQ = L::BQ, NB = L::NB, SC = L::SC, SCR = L::SCR, STAGE = L::STAGE;
  const int tid = threadIdx.x;
  const int wave0 = tid & ~63;
  float* const Dbuf0 = lds;
  float* const Dbuf1 = lds + NB;
  float* const StD = lds + 2 * NB;
  float* const StI = StD + STAGE;  // C arrays of STAGE floats
  float* const Res = StI + STAGE * g.C;
  const int ntiles = g.ntp * g.ntq;
  const int G = gridDim.x;
  const int wg = xcd_remap(blockIdx.x, G);
  const int Np = g.Np, Nq = g.Nq, Na = g.Na;
  const bool use_img = MODE != kModeLam0;
  const int nch = MODE == kModeGeneral ? g.C : (use_img ? 1 : 0);
  // 16-byte global->LDS copies need q contiguous and every row start 16-byte aligned.
  const bool vec4 = g.sq == 1 && (g.Nq & 3) == 0 && (g.sp & 3) == 0 && (g.sa & 3) == 0;

  // Staged address of plane j, box cell lx.
  auto sidx = [](int j, int lx) { return SCANC ? lx * SC + j : j * NB + lx; };

  // First plane in scan order: never changed by the pass.  Written once when the
  // pass also initialises D, recorded as "keep" when records are asked for.
  if (g.init || REC) {
    const int kf = g.sign > 0 ? 0 : Na - 1;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int rp = min(TP, Np - p0), rq = min(TQ, Nq - q0);
      for (int f = tid; f < rp * rq; f += kThreads) {
        const int r = f / rq, cq = f - r * rq;
        const int x = kf * g.sa + (p0 + r) * g.sp + (q0 + cq) * g.sq;
        if (g.init) g.D[x] = g.v * g.mask[x];
        if (REC) g.rec[x] = 0;
      }
    }
  }

  for (int c = 0; c < g.nchunk; ++c) {
    const int t0 = 1 + c * K;
    const int kk = min(K, Na - t0);
    const unsigned epoch_in = g.epoch_base + (unsigned)c;  // published by chunk c - 1
    const unsigned epoch_out = epoch_in + 1u;
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      const int bp0 = (NDIM == 3) ? p0 - K : 0;
      const int bq0 = q0 - K;

      // 1. Global -> LDS copies of the chunk's planes.  Plane j is scan position
      // t0 - 1 + j.  Cell needed iff its distance outside the tile is <= kk - j.
      // D_old (or the mask, for the initialising pass) for planes j >= 1, and
      // plane 0 too in chunk 0 (the pass's unchanged first plane); the image for
      // all planes.
      {
        const float* dsrc = g.init ? g.mask : g.D;
        if (!SCANC && vec4) {
          // 16-byte groups of 4 cells along q (the contiguous axis): groups never
          // straddle the plane edge because q0 - K and Nq are multiples of 4.
          constexpr int NG = STAGE / 4;
          for (int g0 = 0; g0 < NG; g0 += kThreads) {
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
                __builtin_amdgcn_global_load_lds(g.image + (long long)ch * g.N + x, StI + ch * STAGE + 4 * (g0 + wave0),
                                                 16, 0, 0);
            }
          }
        } else {
          for (int f0 = 0; f0 < STAGE; f0 += kThreads) {
            const int f = f0 + tid;
            int j, lx;
            if (SCANC) {
              lx = f / SC;
              j = f - lx * SC;
            } else {
              j = f / NB;
              lx = f - j * NB;
            }
            const int br = lx / BQ, bc = lx - br * BQ;
            const int pp = bp0 + br, qq = bq0 + bc;
            bool ok = f < STAGE && j <= kk && qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
            ok = ok && outside<NDIM, TP, TQ>(pp, qq, p0, q0) <= kk - j;
            if (ok) {
              const int t = t0 - 1 + j;
              const int k = g.sign > 0 ? t : Na - 1 - t;
              const int x = k * g.sa + pp * g.sp + qq * g.sq;
              if (j >= 1 || c == 0) __builtin_amdgcn_global_load_lds(dsrc + x, StD + f0 + wave0, 4, 0, 0);
              for (int ch = 0; ch < nch; ++ch)
                __builtin_amdgcn_global_load_lds(g.image + (long long)ch * g.N + x, StI + ch * STAGE + f0 + wave0, 4,
                                                 0, 0);
            }
          }
        }
      }

      // Cells of the box outside the plane hold +inf in both D buffers, so that a
      // candidate through them can never win and the candidate loop needs no
      // bounds checks.
      for (int lx = tid; lx < NB; lx += kThreads) {
        const int br = lx / BQ, bc = lx - br * BQ;
        const int pp = bp0 + br, qq = bq0 + bc;
        const bool in = qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
        if (!in) {
          Dbuf0[lx] = __builtin_inff();
          Dbuf1[lx] = __builtin_inff();
        }
      }

      // 2. The plane before the chunk on the tile grown by kk.
      if (c > 0) {
        constexpr int MAXB = (NB + kThreads - 1) / kThreads;
        unsigned long long wv[MAXB];
        int lxs[MAXB];
        const unsigned long long* xin = g.xbuf + (size_t)((c - 1) & 1) * ntiles * (TP * TQ);
#pragma unroll
        for (int n = 0; n < MAXB; ++n) {
          const int lx = tid + n * kThreads;
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
          Dbuf0[lx] = __uint_as_float((unsigned)wv[n]);
        }
        if (__syncthreads_or(fail)) return false;
      }
      __builtin_amdgcn_s_waitcnt(0);  // the global->LDS copies have landed
      __syncthreads();
      if (c == 0) {
        // chunk 0: the boundary is the staged plane 0 of D_old
        for (int lx = tid; lx < NB; lx += kThreads) {
          const int br = lx / BQ, bc = lx - br * BQ;
          const int pp = bp0 + br, qq = bq0 + bc;
          const bool in = qq >= 0 && qq < Nq && (NDIM == 2 || (pp >= 0 && pp < Np));
          if (in) {
            const float d = StD[sidx(0, lx)];
            Dbuf0[lx] = g.init ? g.v * d : d;
          }
        }
        lds_barrier();
      }

      // 3. Advance the chunk's planes.
      float* Dp = Dbuf0;
      float* Dc = Dbuf1;
      unsigned long long* xout = g.xbuf + (size_t)(c & 1) * ntiles * (TP * TQ) + (size_t)tile * (TP * TQ);
      for (int i = 0; i < kk; ++i) {
        const int t = t0 + i;
        const int k = g.sign > 0 ? t : Na - 1 - t;
        const int h = kk - 1 - i;
        const int lp = (NDIM == 3) ? max(0, p0 - h) : 0;
        const int hp = (NDIM == 3) ? min(Np, p0 + TP + h) : 1;
        const int lq = max(0, q0 - h), hq = min(Nq, q0 + TQ + h);
        const int rq = hq - lq, cnt = (hp - lp) * rq;
        const float inv_rq = 1.0f / (float)rq;
        for (int f = tid; f < cnt; f += kThreads) {
          int r, cq;
          if (NDIM == 3) {
            r = (int)(((float)f + 0.5f) * inv_rq);
            cq = f - r * rq;
          } else {
            r = 0;
            cq = f;
          }
          const int pp = lp + r, qq = lq + cq;
          const int lx = (pp - bp0) * BQ + (qq - bq0);
          const float dold = StD[sidx(i + 1, lx)];
          float best = g.init ? g.v * dold : dold;
          int choice = 0;
          const float* sx = StI + sidx(i + 1, lx);
          const float* sy = StI + sidx(i, lx);
          const float* dy = Dp + lx;
          const float ix0 = use_img ? sx[0] : 0.0f;
          // Every neighbour lies inside the box; those outside the plane read +inf.
#pragma unroll
          for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp) {
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) {
              const int j = (NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1;
              const int off = dp * BQ + dq;
              const int soff = SCANC ? off * SC : off;
              const float iy0 = use_img ? sy[soff] : 0.0f;
              const float w = edge_cost<MODE>(g, j, ix0, iy0, sx, sy + soff, STAGE);
              const float cand = dy[off] + w;
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
          Dc[lx] = best;
          if (pp >= p0 && pp < p0 + TP && qq >= q0 && qq < q0 + TQ) {
            const int own = (NDIM == 3 ? (pp - p0) * TQ : 0) + (qq - q0);
            const int x = k * g.sa + pp * g.sp + qq * g.sq;
            if (SCANC)
              Res[own * SCR + i] = best;
            else
              g.D[x] = best;
            if (REC) g.rec[x] = (uint8_t)choice;
            if (i == kk - 1)
              st64_relaxed(xout + own, ((unsigned long long)epoch_out << 32) | __float_as_uint(best));
          }
        }
        lds_barrier();
        float* tD = Dp;
        Dp = Dc;
        Dc = tD;
      }

      // 4. Cell-major results: write each cell's run of scan positions.
      if (SCANC) {
        const int rp = (NDIM == 3) ? min(TP, Np - p0) : 1;
        const int rq = min(TQ, Nq - q0);
        for (int f = tid; f < TP * TQ * SCR; f += kThreads) {
          const int own = f / SCR, i = f - own * SCR;
          const int r = (NDIM == 3) ? own / TQ : 0, cq = own - r * TQ;
          if (i < kk && r < rp && cq < rq) {
            const int t = t0 + i;
            const int k = g.sign > 0 ? t : Na - 1 - t;
            g.D[k * g.sa + (p0 + r) * g.sp + (q0 + cq) * g.sq] = Res[f];
          }
        }
        // Res is rewritten only after the next chunk's first barrier.
      }
    }
  }
  return true;
}

template <int NDIM, int TP, int TQ, int K, bool SCANC, int RMODE, bool REC>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassDesc g, unsigned* words, unsigned long long limit) {
  extern __shared__ float lds[];
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  if (RMODE == kModeGeneral) {
    run_pass<NDIM, TP, TQ, K, SCANC, kModeGeneral, REC>(g, words, limit, lds);
    return;
  }
  const unsigned cls = ld_relaxed(words + kWordClass);
  const bool fast = (RMODE == kModeLam0) ? (cls & kClassHuge) == 0u : cls == 0u;
  if (fast)
    run_pass<NDIM, TP, TQ, K, SCANC, RMODE, REC>(g, words, limit, lds);
  else
    run_pass<NDIM, TP, TQ, K, SCANC, kModeGeneral, REC>(g, words, limit, lds);
}

using PassKernel = void (*)(PassDesc, unsigned*, unsigned long long);

template <int NDIM, int TP, int TQ, int K, bool SCANC>
PassKernel pick_mode(int mode, bool rec) {
  if (rec) {
    if (mode == kModeLam0) return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeLam0, true>;
    if (mode == kModeLam1C1) return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeLam1C1, true>;
    return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeGeneral, true>;
  }
  if (mode == kModeLam0) return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeLam0, false>;
  if (mode == kModeLam1C1) return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeLam1C1, false>;
  return pass_kernel<NDIM, TP, TQ, K, SCANC, kModeGeneral, false>;
}

template <int NDIM, int TP, int TQ, int K>
PassKernel pick_layout(const PassDesc& d) {
  const bool scanc = d.sa == 1;
  return scanc ? pick_mode<NDIM, TP, TQ, K, true>(d.mode, d.rec != nullptr)
               : pick_mode<NDIM, TP, TQ, K, false>(d.mode, d.rec != nullptr);
}

// Tile geometries: 3D planes use 16 x 16 tiles, 2D rows 256-wide tiles; the
// chunk length shrinks when many channels would overflow LDS.
constexpr int kTP3 = 16, kTQ3 = 16, kTQ2 = 256;

size_t lds_bytes_for(int ndim, int K, int C, bool scanc) {
  if (ndim == 3) {
    if (K == 8) return scanc ? Layout<3, kTP3, kTQ3, 8, true>::bytes(C) : Layout<3, kTP3, kTQ3, 8, false>::bytes(C);
    if (K == 4) return scanc ? Layout<3, kTP3, kTQ3, 4, true>::bytes(C) : Layout<3, kTP3, kTQ3, 4, false>::bytes(C);
    if (K == 2) return scanc ? Layout<3, kTP3, kTQ3, 2, true>::bytes(C) : Layout<3, kTP3, kTQ3, 2, false>::bytes(C);
  } else {
    if (K == 32) return scanc ? Layout<2, 1, kTQ2, 32, true>::bytes(C) : Layout<2, 1, kTQ2, 32, false>::bytes(C);
    if (K == 16) return scanc ? Layout<2, 1, kTQ2, 16, true>::bytes(C) : Layout<2, 1, kTQ2, 16, false>::bytes(C);
    if (K == 8) return scanc ? Layout<2, 1, kTQ2, 8, true>::bytes(C) : Layout<2, 1, kTQ2, 8, false>::bytes(C);
  }
  return 0;
}

PassKernel select_kernel(const PassDesc& d, int ndim) {
  if (ndim == 3 && d.TP == kTP3 && d.TQ == kTQ3) {
    if (d.K == 8) return pick_layout<3, kTP3, kTQ3, 8>(d);
    if (d.K == 4) return pick_layout<3, kTP3, kTQ3, 4>(d);
    if (d.K == 2) return pick_layout<3, kTP3, kTQ3, 2>(d);
  } else if (ndim == 2 && d.TP == 1 && d.TQ == kTQ2) {
    if (d.K == 32) return pick_layout<2, 1, kTQ2, 32>(d);
    if (d.K == 16) return pick_layout<2, 1, kTQ2, 16>(d);
    if (d.K == 8) return pick_layout<2, 1, kTQ2, 8>(d);
  }
  return nullptr;
}

__global__ void reset_kernel(unsigned* ws, long long nwords) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) ws[i] = 0u;
}

__global__ __launch_bounds__(256) void classify_kernel(const float* img, long long n, unsigned* words) {
  unsigned bits = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float a = fabsf(img[i]);
    if (!(a <= 0x1p60f)) bits |= kClassHuge;
    else if (a != 0.0f && a < 0x1p-40f) bits |= kClassTiny;
  }
  const int tiny = __syncthreads_or((bits & kClassTiny) ? 1 : 0);
  const int huge = __syncthreads_or((bits & kClassHuge) ? 1 : 0);
  if (threadIdx.x == 0 && (tiny || huge))
    __hip_atomic_fetch_or(words + kWordClass, (tiny ? kClassTiny : 0u) | (huge ? kClassHuge : 0u),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void scale_kernel(const float* mask, float v, float* out, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = v * mask[i];
}

struct CapEntry {
  const void* fn;
  size_t lds;
  int cap;
};
CapEntry g_cap_cache[256];
int g_cap_n = 0;

// Co-resident workgroups of `fn` with `lds` dynamic LDS bytes (also raises the
// kernel's dynamic-LDS limit once).  0 on failure.
int capacity_for(PassKernel fn, size_t lds) {
  for (int i = 0; i < g_cap_n; ++i)
    if (g_cap_cache[i].fn == (const void*)fn && g_cap_cache[i].lds == lds) return g_cap_cache[i].cap;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kThreads, lds) != hipSuccess) return 0;
  const int cap = per_cu * cus;
  if (g_cap_n < 256) g_cap_cache[g_cap_n++] = CapEntry{(const void*)fn, lds, cap};
  return cap;
}

}  // namespace

int pass_chunk_for(int ndim, int C, bool scan_contiguous) {
  const int ks3[3] = {8, 4, 2}, ks2[3] = {32, 16, 8};
  for (int i = 0; i < 3; ++i) {
    const int K = ndim == 3 ? ks3[i] : ks2[i];
    if (lds_bytes_for(ndim, K, C, scan_contiguous) <= kMaxLdsBytes) return K;
  }
  return 0;
}

hipError_t launch_pass(const PassDesc& d, int ndim, unsigned* words, unsigned long long spin_limit,
                       hipStream_t stream) {
  PassKernel fn = select_kernel(d, ndim);
  if (!fn) return hipErrorInvalidConfiguration;
  const size_t lds = lds_bytes_for(ndim, d.K, d.C, d.sa == 1);
  if (lds == 0 || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
  const int cap = capacity_for(fn, lds);
  if (cap <= 0) return hipErrorInvalidConfiguration;
  const int ntiles = d.ntp * d.ntq;
  const int grid = ntiles < cap ? ntiles : cap;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), lds, stream, d, words, spin_limit);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned* ws, long long nwords, hipStream_t stream) {
  long long blocks = (nwords + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ws, nwords);
  return hipGetLastError();
}

hipError_t launch_classify(const float* image, long long n, unsigned* words, hipStream_t stream) {
  long long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(classify_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, image, n, words);
  return hipGetLastError();
}

hipError_t launch_scale(const float* mask, float v, float* out, long long n, hipStream_t stream) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, mask, v, out, n);
  return hipGetLastError();
}

}  // namespace ggdt
