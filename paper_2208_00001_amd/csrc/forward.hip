// Forward directional-pass kernels for gfx950.
//
// One launch runs one directional pass (FastGeodis paper, section
// "Implementation": a row (2D) or plane (3D) is updated in parallel from the
// previous one, so values propagate along the pass direction).  The launch is
// persistent along the scan axis: the plane is cut into TP x TQ tiles, each tile
// owned by one workgroup, and the scan axis into chunks of K steps.  For a chunk
// a workgroup loads the last finished plane on its tile grown by K voxels on every
// side (overlapped tiling) and then advances K planes with LDS exchange and one
// workgroup barrier per plane, recomputing a shrinking halo so that no other
// workgroup is consulted inside the chunk.  Between chunks a workgroup waits only
// for its (up to 8) neighbouring tiles' progress words.
//
// Halo voxels read D from memory that the owning neighbour may be overwriting in
// the same chunk.  Either value gives the same result: the neighbour writes
// min(D_old, candidates) and this workgroup takes min(read value, the same
// candidates), so the halo value it recomputes is identical bit for bit.
#include "ggdt_internal.h"

namespace ggdt {
namespace {

constexpr int kThreads = 256;

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

// Wait until every neighbouring tile (p +- 1, q +- 1) has published `target`.
// Lanes of wave 0 poll one neighbour each.  Returns false when the wait was
// abandoned because a poll budget ran out here or anywhere else in the launch.
template <int NDIM>
__device__ bool wait_neighbours(const unsigned* flags, unsigned* words, int tp, int tq, int ntp, int ntq,
                                unsigned target, unsigned long long limit, int* s_ok) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    bool ok = true;
    const int dp = (NDIM == 3) ? lane / 3 - 1 : 0;
    const int dq = (NDIM == 3) ? lane % 3 - 1 : lane - 1;
    const int np = tp + dp, nq = tq + dq;
    const bool poll = lane < (NDIM == 3 ? 9 : 3) && !(dp == 0 && dq == 0) && np >= 0 && np < ntp && nq >= 0 &&
                      nq < ntq;
    if (poll) {
      const unsigned* f = flags + np * ntq + nq;
      unsigned long long n = 0;
      while (ld_relaxed(f) < target) {
        if (ld_relaxed(words + kWordAbort) != 0u) {
          ok = false;
          break;
        }
        if (++n > limit) {
          __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const int all_ok = __all(ok ? 1 : 0);
    if (lane == 0) *s_ok = all_ok;
  }
  __syncthreads();
  const bool ok = *s_ok != 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

// Edge cost between x and its candidate parent y through offset j.
template <int MODE>
__device__ __forceinline__ float edge_cost(const PassDesc& g, int j, float ix0, float iy0, const float* Ic,
                                           const float* Ip, int lx, int ly, int NB) {
  if (MODE == kModeLam0) {
    return g.W0[j];
  } else if (MODE == kModeLam1C1) {
    return fabsf(ix0 - iy0);
  } else {
    const float d0 = ix0 - iy0;
    float s = d0 * d0;
    for (int c = 1; c < g.C; ++c) {
      const float dc = Ic[c * NB + lx] - Ip[c * NB + ly];
      s = fmaf(dc, dc, s);
    }
    return sqrtf(fmaf(g.lam, s, g.A[j]));
  }
}

template <int NDIM, int TP, int TQ, int MODE, bool REC>
__device__ bool run_pass(const PassDesc& g, unsigned* words, unsigned* flags, unsigned long long limit,
                         float* lds, int* s_ok) {
  const int tid = threadIdx.x;
  const int K = g.K;
  const int BQ = TQ + 2 * K;
  const int BP = (NDIM == 3) ? TP + 2 * K : 1;
  const int NB = BP * BQ;
  float* Dbuf0 = lds;
  float* Dbuf1 = lds + NB;
  float* Ibuf0 = lds + 2 * NB;
  float* Ibuf1 = Ibuf0 + g.C * NB;
  const int ntiles = g.ntp * g.ntq;
  const int G = gridDim.x;
  const int wg = xcd_remap(blockIdx.x, G);
  const int Np = g.Np, Nq = g.Nq, Na = g.Na;

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
    for (int tile = wg; tile < ntiles; tile += G) {
      const int tp = tile / g.ntq, tq = tile - tp * g.ntq;
      const int p0 = tp * TP, q0 = tq * TQ;
      if (c > 0) {
        if (!wait_neighbours<NDIM>(flags, words, tp, tq, g.ntp, g.ntq, g.flag_base + c, limit, s_ok))
          return false;
      }
      // Box origin of the tile's LDS planes.
      const int bp0 = (NDIM == 3) ? p0 - K : 0;
      const int bq0 = q0 - K;

      // The finished plane before this chunk, on the tile grown by kk.
      {
        const int kb = g.sign > 0 ? t0 - 1 : Na - t0;
        const int lp = (NDIM == 3) ? max(0, p0 - kk) : 0;
        const int hp = (NDIM == 3) ? min(Np, p0 + TP + kk) : 1;
        const int lq = max(0, q0 - kk), hq = min(Nq, q0 + TQ + kk);
        const int rq = hq - lq, cnt = (hp - lp) * rq;
        const bool from_mask = (c == 0) && g.init;
        for (int f = tid; f < cnt; f += kThreads) {
          const int r = f / rq, cq = f - r * rq;
          const int pp = lp + r, qq = lq + cq;
          const int x = kb * g.sa + pp * g.sp + qq * g.sq;
          const int l = (pp - bp0) * BQ + (qq - bq0);
          Dbuf0[l] = from_mask ? g.v * g.mask[x] : g.D[x];
          if (MODE != kModeLam0) {
            for (int ch = 0; ch < (MODE == kModeLam1C1 ? 1 : g.C); ++ch)
              Ibuf0[ch * NB + l] = g.image[(long long)ch * g.N + x];
          }
        }
      }
      __syncthreads();

      float* Dp = Dbuf0;
      float* Dc = Dbuf1;
      float* Ip = Ibuf0;
      float* Ic = Ibuf1;
      for (int i = 0; i < kk; ++i) {
        const int t = t0 + i;
        const int k = g.sign > 0 ? t : Na - 1 - t;
        const int h = kk - 1 - i;
        const int lp = (NDIM == 3) ? max(0, p0 - h) : 0;
        const int hp = (NDIM == 3) ? min(Np, p0 + TP + h) : 1;
        const int lq = max(0, q0 - h), hq = min(Nq, q0 + TQ + h);
        const int rq = hq - lq, cnt = (hp - lp) * rq;
        for (int f = tid; f < cnt; f += kThreads) {
          const int r = f / rq, cq = f - r * rq;
          const int pp = lp + r, qq = lq + cq;
          const int x = k * g.sa + pp * g.sp + qq * g.sq;
          const int lx = (pp - bp0) * BQ + (qq - bq0);
          float best = g.init ? g.v * g.mask[x] : g.D[x];
          int choice = 0;
          float ix0 = 0.0f;
          if (MODE != kModeLam0) {
            ix0 = g.image[x];
            Ic[lx] = ix0;
            if (MODE == kModeGeneral)
              for (int ch = 1; ch < g.C; ++ch) Ic[ch * NB + lx] = g.image[(long long)ch * g.N + x];
          }
#pragma unroll
          for (int dp = (NDIM == 3 ? -1 : 0); dp <= (NDIM == 3 ? 1 : 0); ++dp) {
            const int yp = pp + dp;
            const bool okp = (NDIM == 2) || (yp >= 0 && yp < Np);
#pragma unroll
            for (int dq = -1; dq <= 1; ++dq) {
              const int j = (NDIM == 3 ? (dp + 1) * 3 : 0) + dq + 1;
              const int yq = qq + dq;
              if (!okp || yq < 0 || yq >= Nq) continue;
              const int ly = lx + dp * BQ + dq;
              const float iy0 = (MODE != kModeLam0) ? Ip[ly] : 0.0f;
              const float w = edge_cost<MODE>(g, j, ix0, iy0, Ic, Ip, lx, ly, NB);
              const float cand = Dp[ly] + w;
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
            g.D[x] = best;
            if (REC) g.rec[x] = (uint8_t)choice;
          }
        }
        __syncthreads();
        float* tD = Dp;
        Dp = Dc;
        Dc = tD;
        float* tI = Ip;
        Ip = Ic;
        Ic = tI;
      }
      // Publish: every thread's stores are made visible device-wide, then one
      // release store of the tile's progress word.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(flags + tile, g.flag_base + c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return true;
}

template <int NDIM, int TP, int TQ, int RMODE, bool REC>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassDesc g, unsigned* words, unsigned* flags,
                                                        unsigned long long limit) {
  extern __shared__ float lds[];
  __shared__ int s_ok;
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  if (RMODE == kModeGeneral) {
    run_pass<NDIM, TP, TQ, kModeGeneral, REC>(g, words, flags, limit, lds, &s_ok);
    return;
  }
  const unsigned cls = ld_relaxed(words + kWordClass);
  const bool fast = (RMODE == kModeLam0) ? (cls & kClassHuge) == 0u : cls == 0u;
  if (fast)
    run_pass<NDIM, TP, TQ, RMODE, REC>(g, words, flags, limit, lds, &s_ok);
  else
    run_pass<NDIM, TP, TQ, kModeGeneral, REC>(g, words, flags, limit, lds, &s_ok);
}

using PassKernel = void (*)(PassDesc, unsigned*, unsigned*, unsigned long long);

template <int NDIM, int TP, int TQ>
PassKernel pick(int mode, bool rec) {
  if (rec) {
    if (mode == kModeLam0) return pass_kernel<NDIM, TP, TQ, kModeLam0, true>;
    if (mode == kModeLam1C1) return pass_kernel<NDIM, TP, TQ, kModeLam1C1, true>;
    return pass_kernel<NDIM, TP, TQ, kModeGeneral, true>;
  }
  if (mode == kModeLam0) return pass_kernel<NDIM, TP, TQ, kModeLam0, false>;
  if (mode == kModeLam1C1) return pass_kernel<NDIM, TP, TQ, kModeLam1C1, false>;
  return pass_kernel<NDIM, TP, TQ, kModeGeneral, false>;
}

PassKernel select_kernel(const PassDesc& d, int ndim) {
  const bool rec = d.rec != nullptr;
  if (ndim == 3) return pick<3, 16, 16>(d.mode, rec);
  return pick<2, 1, 256>(d.mode, rec);
}

__global__ void reset_kernel(unsigned* ws, int nwords) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) ws[i] = 0u;
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
CapEntry g_cap_cache[64];
int g_cap_n = 0;

int capacity_for(PassKernel fn, size_t lds) {
  for (int i = 0; i < g_cap_n; ++i)
    if (g_cap_cache[i].fn == (const void*)fn && g_cap_cache[i].lds == lds) return g_cap_cache[i].cap;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kThreads, lds) != hipSuccess) return 0;
  const int cap = per_cu * cus;
  if (g_cap_n < 64) g_cap_cache[g_cap_n++] = CapEntry{(const void*)fn, lds, cap};
  return cap;
}

}  // namespace

size_t pass_lds_bytes(const PassDesc& d, int ndim) {
  const int BQ = d.TQ + 2 * d.K;
  const int BP = ndim == 3 ? d.TP + 2 * d.K : 1;
  return (size_t)(2 + 2 * d.C) * (size_t)(BP * BQ) * sizeof(float);
}

int pass_grid_capacity(const PassDesc& d, int ndim) { return capacity_for(select_kernel(d, ndim), pass_lds_bytes(d, ndim)); }

hipError_t launch_pass(const PassDesc& d, int ndim, unsigned* words, unsigned* flags, unsigned long long spin_limit,
                       int grid_cap, hipStream_t stream) {
  PassKernel fn = select_kernel(d, ndim);
  const size_t lds = pass_lds_bytes(d, ndim);
  const int ntiles = d.ntp * d.ntq;
  int cap = grid_cap > 0 ? grid_cap : capacity_for(fn, lds);
  if (cap <= 0) return hipErrorInvalidConfiguration;
  const int grid = ntiles < cap ? ntiles : cap;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), lds, stream, d, words, flags, spin_limit);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned* ws, int nwords, hipStream_t stream) {
  const int grid = (nwords + 255) / 256 < 64 ? (nwords + 255) / 256 : 64;
  hipLaunchKernelGGL(reset_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, stream, ws, nwords);
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
