// Batched ragged GGDT: every pass of every instance in one persistent launch.
//
// Each instance owns a contiguous range of logical workgroups (split at plan
// time in proportion to its work).  Its workgroups run its passes in schedule
// order with the single-instance pass code (pass_device.h); between passes they
// meet at an instance-local barrier (release fence, counter, bounded wait,
// acquire fence), so instances never wait for each other.  The launch is sized to
// the co-resident capacity, which the bounded waits require.
#include "pass_cell.h"
#include "pass_device.h"
#include "grid_sync.h"
#include "layout.h"

namespace ggdt {
namespace {

using namespace dev;

// All workgroups of an instance have finished the pass: arrive on the counter
// and wait until `target` arrivals are seen.  False if the wait was abandoned.
__device__ __forceinline__ bool instance_barrier(unsigned* counter, unsigned target, unsigned* words,
                                                 unsigned long long limit) {
  return counter_barrier<unsigned>(counter, target, words, limit);
}

// Batched workgroups have kBatchThreads threads: single-channel 3D instances
// (class 0, K = 8) run the thread-per-cell pass, the others the tile pass with
// that many threads.
constexpr int kBatchThreads = kCellThreads;

template <int NDIM, int TP, int TQ, int K, bool REC>
__device__ __forceinline__ bool run_pass_rt(const PassDesc* gp, unsigned long long* xbuf, unsigned* words,
                                            const unsigned* cls, int mode, unsigned long long limit, float* lds,
                                            int wg, int G) {
  constexpr int NT = kBatchThreads;
  const bool scanc = gp->sa == 1;
  if (scanc) {
    if (mode == kModeLam0) return run_pass_mode<NDIM, TP, TQ, K, true, kModeLam0, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
    if (mode == kModeLam1C1) return run_pass_mode<NDIM, TP, TQ, K, true, kModeLam1C1, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
    return run_pass_mode<NDIM, TP, TQ, K, true, kModeGeneral, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
  }
  if (mode == kModeLam0) return run_pass_mode<NDIM, TP, TQ, K, false, kModeLam0, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
  if (mode == kModeLam1C1) return run_pass_mode<NDIM, TP, TQ, K, false, kModeLam1C1, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
  return run_pass_mode<NDIM, TP, TQ, K, false, kModeGeneral, REC, NT>(gp, xbuf, words, cls, limit, lds, wg, G);
}

// A layout change of one instance (PassDesc::op) by its G workgroups;
// PassDesc::K: tiles per round the launch's LDS holds (4, else 1).
__device__ __forceinline__ bool run_layout_op(const PassDesc* gp, unsigned* words, float* lds, int wg, int G) {
  const PassDesc g = resolve_offsets(*gp, words);
  const TransposeShape sh = transpose_shape(g.op == kOpToScanMajor, g.Np, g.Nq, g.Na);
  if (g.esz == 1) {  // records (byte volumes)
    const uint8_t* src = reinterpret_cast<const uint8_t*>(g.image);
    uint8_t* dst = reinterpret_cast<uint8_t*>(g.D);
    uint8_t* tiles = reinterpret_cast<uint8_t*>(lds);
    if (g.K >= 4) layout_rounds<uint8_t, kBatchThreads, 4>(src, dst, sh, tiles, wg, G);
    else layout_rounds<uint8_t, kBatchThreads, 1>(src, dst, sh, tiles, wg, G);
  } else if (g.K >= 4) {
    layout_rounds<float, kBatchThreads, 4>(g.image, g.D, sh, lds, wg, G);
  } else {
    layout_rounds<float, kBatchThreads, 1>(g.image, g.D, sh, lds, wg, G);
  }
  return true;
}

// CT: tile side of the thread-per-cell pass for 3D instances (0: the tile pass).
template <int K3, int K2, bool REC, int CT>
__global__ __launch_bounds__(kBatchThreads) void batched_kernel(const BatchInst* __restrict__ insts, int ninst,
                                                           const PassDesc* __restrict__ passes, unsigned char* ws,
                                                           unsigned long long limit) {
  extern __shared__ __align__(16) float lds[];
  unsigned* words = reinterpret_cast<unsigned*>(ws);
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (insts[mid].wg0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchInst in = insts[lo];
  const int wg = b - in.wg0;
  if (wg < 0 || wg >= in.nwg) return;
  unsigned long long* xbuf = reinterpret_cast<unsigned long long*>(ws + in.xbuf_off);
  unsigned* ctr = reinterpret_cast<unsigned*>(ws + in.ctr_off);
  const unsigned* cls = reinterpret_cast<const unsigned*>(ws + in.cls_off);
  for (int p = 0; p < in.npass; ++p) {
    const PassDesc* gp = passes + in.pass0 + p;
    bool ok;
    if (gp->op != kOpPass) {
      ok = run_layout_op(gp, words, lds, wg, in.nwg);
    } else if (in.ndim == 3) {
      if constexpr (CT != 0)
        ok = run_pass_cell_rt<REC, CT, K3>(gp, xbuf, words, cls, in.mode, limit, carve_cell_lds(lds), wg, in.nwg);
      else
        ok = run_pass_rt<3, kTP3, kTQ3, K3, REC>(gp, xbuf, words, cls, in.mode, limit, lds, wg, in.nwg);
    } else {
      ok = run_pass_rt<2, 1, kTQ2, K2, REC>(gp, xbuf, words, cls, in.mode, limit, lds, wg, in.nwg);
    }
    if (!ok) return;
    if (p + 1 < in.npass && !instance_barrier(ctr, (unsigned)(p + 1) * (unsigned)in.nwg, words, limit)) return;
  }
}

// Classification of every instance's image into its class word (grid-stride
// over the instances' values; one workgroup-level OR per instance per block).
__global__ __launch_bounds__(256) void batched_classify_kernel(const BatchInst* __restrict__ insts, int ninst,
                                                               unsigned char* ws) {
  for (int i = 0; i < ninst; ++i) {
    const BatchInst in = insts[i];
    unsigned bits = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < in.nimg; t += stride) {
      const float a = fabsf(to_gmem(in.image)[t]);
      if (!(a <= 0x1p60f)) bits |= kClassHuge;
      else if (a != 0.0f && a < 0x1p-24f) bits |= a < 0x1p-40f ? (kClassSmall | kClassTiny) : kClassSmall;
    }
    const int tiny = __syncthreads_or((bits & kClassTiny) ? 1 : 0);
    const int huge = __syncthreads_or((bits & kClassHuge) ? 1 : 0);
    const int small = __syncthreads_or((bits & kClassSmall) ? 1 : 0);
    if (threadIdx.x == 0 && (tiny || huge || small))
      __hip_atomic_fetch_or(reinterpret_cast<unsigned*>(ws + in.cls_off),
                            (tiny ? kClassTiny : 0u) | (huge ? kClassHuge : 0u) | (small ? kClassSmall : 0u),
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

using BatchedKernel = void (*)(const BatchInst*, int, const PassDesc*, unsigned char*, unsigned long long);

static_assert(kBatchTile3[0] == kCellTP && kBatchK3[0] == kCellK && kBatchTile3[2] == kCellWideTP &&
                  kBatchK3[2] == kCellWideK,
              "batched classes 0 and 2 run the thread-per-cell pass geometries");

template <int C>
BatchedKernel pick_class(bool rec) {
  constexpr int CT = C == 1 ? 0 : kBatchTile3[C];
  return rec ? batched_kernel<kBatchK3[C], kBatchK2[C], true, CT> : batched_kernel<kBatchK3[C], kBatchK2[C], false, CT>;
}

BatchedKernel pick(int kclass, bool rec) {
  if (kclass == 0) return pick_class<0>(rec);
  if (kclass == 2) return pick_class<2>(rec);
  return pick_class<1>(rec);
}

template <int K3, int K2, bool CELL>
size_t lds_for(int C, bool has2d, bool has3d) {
  size_t b = 0;
  if (has3d) {
    if (CELL) {
      b = max(b, kCellLdsBytes);
    } else {
      b = max(b, Layout<3, kTP3, kTQ3, K3, true>::bytes(C));
      b = max(b, Layout<3, kTP3, kTQ3, K3, false>::bytes(C));
    }
  }
  if (has2d) {
    b = max(b, Layout<2, 1, kTQ2, K2, true>::bytes(C));
    b = max(b, Layout<2, 1, kTQ2, K2, false>::bytes(C));
  }
  return b;
}

}  // namespace

size_t batched_lds_bytes(int kclass, int C, bool has2d, bool has3d) {
  if (kclass == 0) return lds_for<kBatchK3[0], kBatchK2[0], true>(C, has2d, has3d);
  if (kclass == 2) return lds_for<kBatchK3[2], kBatchK2[2], true>(C, has2d, has3d);
  return lds_for<kBatchK3[1], kBatchK2[1], false>(C, has2d, has3d);
}

int batched_capacity(int kclass, bool rec, size_t lds) {
  BatchedKernel fn = pick(kclass, rec);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBatchThreads, lds) != hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t launch_batched(int kclass, bool rec, const BatchInst* insts, int ninst, const PassDesc* passes,
                          unsigned char* ws, int grid, size_t lds, unsigned long long spin_limit, hipStream_t stream) {
  BatchedKernel fn = pick(kclass, rec);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBatchThreads), lds, stream, insts, ninst, passes, ws, spin_limit);
  return hipGetLastError();
}

hipError_t launch_batched_classify(const BatchInst* insts, int ninst, unsigned char* ws, hipStream_t stream) {
  hipLaunchKernelGGL(batched_classify_kernel, dim3(1024), dim3(256), 0, stream, insts, ninst, ws);
  return hipGetLastError();
}

}  // namespace ggdt
