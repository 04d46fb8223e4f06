// Backward (reverse-mode) kernels: one launch per reversed pass of one instance,
// and the batched persistent launch over many instances (see backward_device.h).
#include "backward_cell.h"
#include "backward_device.h"
#include "grid_sync.h"
#include "layout.h"

namespace ggdt {
namespace {

using namespace dev;

template <int NDIM, int TP, int TQ, int K, bool SCANC>
__global__ __launch_bounds__(kThreads) void bwd_pass_kernel(BwdDesc g, unsigned* words, unsigned long long limit) {
  extern __shared__ __align__(16) float lds[];
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  run_bwd_pass_mode<NDIM, TP, TQ, K, SCANC>(&g, g.xbuf, words, words + kWordClass, limit, lds,
                                            xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Single-channel 3D reversed passes on 16 x 16 tiles with K = 8: one thread per box cell.
__global__ __launch_bounds__(kCellThreads) void bwd_pass_cell_kernel(BwdDesc g, unsigned* words,
                                                                     unsigned long long limit) {
  __shared__ float lds[(kBwdCellLdsBytes + 3) / 4];
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  run_bwd_pass_cell_mode(&g, g.xbuf, words, words + kWordClass, limit, lds, xcd_remap(blockIdx.x, gridDim.x),
                         gridDim.x);
}

bool use_bwd_cell(const BwdDesc& d, int ndim) {
  return ndim == 3 && d.C == 1 && d.K == kCellK && d.TP == kCellTP && d.TQ == kCellTQ;
}

using BwdKernel = void (*)(BwdDesc, unsigned*, unsigned long long);

template <int NDIM, int TP, int TQ, int K>
BwdKernel pick_bwd(bool scanc) {
  return scanc ? bwd_pass_kernel<NDIM, TP, TQ, K, true> : bwd_pass_kernel<NDIM, TP, TQ, K, false>;
}

BwdKernel select_bwd(const BwdDesc& d, int ndim) {
  const bool scanc = d.sa == 1;
  if (ndim == 3) {
    if (d.K == 4) return pick_bwd<3, kTP3, kTQ3, 4>(scanc);
    if (d.K == 2) return pick_bwd<3, kTP3, kTQ3, 2>(scanc);
  } else {
    if (d.K == 16) return pick_bwd<2, 1, kTQ2, 16>(scanc);
    if (d.K == 8) return pick_bwd<2, 1, kTQ2, 8>(scanc);
  }
  return nullptr;
}

size_t bwd_lds(int ndim, int K, int C, bool scanc) {
  if (ndim == 3) {
    if (K == 4) return scanc ? BLayout<3, kTP3, kTQ3, 4, true>::bytes(C) : BLayout<3, kTP3, kTQ3, 4, false>::bytes(C);
    if (K == 2) return scanc ? BLayout<3, kTP3, kTQ3, 2, true>::bytes(C) : BLayout<3, kTP3, kTQ3, 2, false>::bytes(C);
  } else {
    if (K == 16) return scanc ? BLayout<2, 1, kTQ2, 16, true>::bytes(C) : BLayout<2, 1, kTQ2, 16, false>::bytes(C);
    if (K == 8) return scanc ? BLayout<2, 1, kTQ2, 8, true>::bytes(C) : BLayout<2, 1, kTQ2, 8, false>::bytes(C);
  }
  return 0;
}

int capacity_of(const void* fn, size_t lds, int threads = kThreads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (lds > 0 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

// Batched: every reversed pass of every instance, instance-local barriers in
// between (same structure as the batched forward kernel).
__device__ __forceinline__ bool bwd_instance_barrier(unsigned* counter, unsigned target, unsigned* words,
                                                     unsigned long long limit) {
  return counter_barrier<unsigned>(counter, target, words, limit);
}

// Batched reverse workgroups have 1024 threads.  Class 0 (every instance a
// single-channel volume): the thread-per-cell reverse pass only; class 1: the
// tile reverse passes (2D and 3D) with 1024 threads.
static_assert(kBwdBatchKCell == kCellK, "batched single-channel 3D reverse passes use the cell chunk length");

// A layout change of one of an instance's volumes (BwdDesc::op, K tiles per
// round) by its G workgroups.
__device__ __forceinline__ void run_bwd_layout_op(const BwdDesc* gp, unsigned char* ws, float* lds, int wg, int G) {
  const TransposeShape sh = transpose_shape(gp->op == kOpToScanMajor, gp->Np, gp->Nq, gp->Na);
  const void* src = gp->lsrc_off >= 0 ? (const void*)(ws + gp->lsrc_off) : gp->lsrc;
  void* dst = gp->ldst_off >= 0 ? (void*)(ws + gp->ldst_off) : gp->ldst;
  if (gp->esz == 4) {
    if (gp->K >= 4)
      layout_rounds<float, kCellThreads, 4>((const float*)src, (float*)dst, sh, lds, wg, G);
    else
      layout_rounds<float, kCellThreads, 1>((const float*)src, (float*)dst, sh, lds, wg, G);
  } else {
    uint8_t* bl = reinterpret_cast<uint8_t*>(lds);
    if (gp->K >= 4)
      layout_rounds<uint8_t, kCellThreads, 4>((const uint8_t*)src, (uint8_t*)dst, sh, bl, wg, G);
    else
      layout_rounds<uint8_t, kCellThreads, 1>((const uint8_t*)src, (uint8_t*)dst, sh, bl, wg, G);
  }
}

// The same, out of line: the thread-per-cell reverse pass already needs the
// registers a 1024-thread workgroup has, and an inlined layout change would
// make it spill.
__device__ __attribute__((noinline)) void run_bwd_layout_op_call(const BwdDesc* gp, unsigned char* ws, float* lds,
                                                                 int wg, int G) {
  run_bwd_layout_op(gp, ws, lds, wg, G);
}

template <bool CELL3D>
__global__ __launch_bounds__(kCellThreads) void batched_bwd_kernel(const BatchInst* __restrict__ insts, int ninst,
                                                               const BwdDesc* __restrict__ passes, unsigned char* ws,
                                                               unsigned long long limit) {
  // The dynamic area is placed after the static LDS variables (the pass
  // barrier's flag): without the alignment it would start 4 bytes in, and every
  // 8- or 16-byte LDS access of the pass would be misaligned.
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
    const BwdDesc* gp = passes + in.pass0 + p;
    if (gp->op != kOpPass) {
      if constexpr (CELL3D)
        run_bwd_layout_op_call(gp, ws, lds, wg, in.nwg);
      else
        run_bwd_layout_op(gp, ws, lds, wg, in.nwg);
      if (p + 1 < in.npass && !bwd_instance_barrier(ctr, (unsigned)(p + 1) * (unsigned)in.nwg, words, limit)) return;
      continue;
    }
    const bool scanc = gp->sa == 1;
    constexpr int NT = kCellThreads;
    bool ok;
    if constexpr (CELL3D) {
      ok = run_bwd_pass_cell_mode(gp, xbuf, words, cls, limit, lds, wg, in.nwg);
    } else if (in.ndim == 3) {
      ok = scanc ? run_bwd_pass_mode<3, kTP3, kTQ3, kBwdBatchK3, true, NT>(gp, xbuf, words, cls, limit, lds, wg, in.nwg)
                 : run_bwd_pass_mode<3, kTP3, kTQ3, kBwdBatchK3, false, NT>(gp, xbuf, words, cls, limit, lds, wg, in.nwg);
    } else {
      ok = scanc ? run_bwd_pass_mode<2, 1, kTQ2, kBwdBatchK2, true, NT>(gp, xbuf, words, cls, limit, lds, wg, in.nwg)
                 : run_bwd_pass_mode<2, 1, kTQ2, kBwdBatchK2, false, NT>(gp, xbuf, words, cls, limit, lds, wg, in.nwg);
    }
    if (!ok) return;
    if (p + 1 < in.npass && !bwd_instance_barrier(ctr, (unsigned)(p + 1) * (unsigned)in.nwg, words, limit)) return;
  }
}

}  // namespace

int bwd_chunk_for(int ndim, int C, bool scan_contiguous) {
  if (ndim == 3 && C == 1) return kCellK;  // thread-per-cell reverse pass
  const int ks3[2] = {4, 2}, ks2[2] = {16, 8};
  for (int i = 0; i < 2; ++i) {
    const int K = ndim == 3 ? ks3[i] : ks2[i];
    if (bwd_lds(ndim, K, C, scan_contiguous) <= kMaxLdsBytes) return K;
  }
  return 0;
}

hipError_t launch_bwd_pass(const BwdDesc& d, int ndim, unsigned* words, unsigned long long spin_limit,
                           hipStream_t stream) {
  if (use_bwd_cell(d, ndim)) {
    static int cap_cell = 0;
    if (cap_cell <= 0) cap_cell = capacity_of((const void*)bwd_pass_cell_kernel, 0, kCellThreads);
    if (cap_cell <= 0) return hipErrorInvalidConfiguration;
    const int ntiles = d.ntp * d.ntq;
    const int grid = ntiles < cap_cell ? ntiles : cap_cell;
    hipLaunchKernelGGL(bwd_pass_cell_kernel, dim3(grid), dim3(kCellThreads), 0, stream, d, words, spin_limit);
    return hipGetLastError();
  }
  BwdKernel fn = select_bwd(d, ndim);
  if (!fn) return hipErrorInvalidConfiguration;
  const size_t lds = bwd_lds(ndim, d.K, d.C, d.sa == 1);
  if (lds == 0 || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
  const int cap = capacity_of((const void*)fn, lds);
  if (cap <= 0) return hipErrorInvalidConfiguration;
  const int ntiles = d.ntp * d.ntq;
  const int grid = ntiles < cap ? ntiles : cap;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), lds, stream, d, words, spin_limit);
  return hipGetLastError();
}

// c2 / c3: the largest channel count of the batch's 2D / 3D instances (0: none).
size_t batched_bwd_lds_bytes(int c2, int c3) {
  size_t b = 0;
  if (c3 > 0) {
    if (c3 == 1 && c2 == 0) {
      b = max(b, kBwdCellLdsBytes);  // class 0: thread-per-cell reverse pass
    } else {
      b = max(b, BLayout<3, kTP3, kTQ3, kBwdBatchK3, true>::bytes(c3));
      b = max(b, BLayout<3, kTP3, kTQ3, kBwdBatchK3, false>::bytes(c3));
    }
  }
  if (c2 > 0) {
    b = max(b, BLayout<2, 1, kTQ2, kBwdBatchK2, true>::bytes(c2));
    b = max(b, BLayout<2, 1, kTQ2, kBwdBatchK2, false>::bytes(c2));
  }
  return b;
}

int batched_bwd_capacity(int bclass, size_t lds) {
  return capacity_of(bclass == 0 ? (const void*)batched_bwd_kernel<true> : (const void*)batched_bwd_kernel<false>,
                     lds, kCellThreads);
}

hipError_t launch_batched_bwd(int bclass, const BatchInst* insts, int ninst, const BwdDesc* passes, unsigned char* ws,
                              int grid, size_t lds, unsigned long long spin_limit, hipStream_t stream) {
  if (bclass == 0)
    hipLaunchKernelGGL(batched_bwd_kernel<true>, dim3(grid), dim3(kCellThreads), lds, stream, insts, ninst, passes,
                       ws, spin_limit);
  else
    hipLaunchKernelGGL(batched_bwd_kernel<false>, dim3(grid), dim3(kCellThreads), lds, stream, insts, ninst, passes,
                       ws, spin_limit);
  return hipGetLastError();
}

}  // namespace ggdt
