// Forward directional-pass kernels for gfx950: one launch per pass of one
// instance (see pass_device.h for the pass itself), plus the small helper
// kernels (workspace reset, image classification, v * M).
#include "pass_cell.h"
#include "pass_device.h"
#include "pass_row.h"

namespace ggdt {
namespace {

using namespace dev;

template <int NDIM, int TP, int TQ, int K, bool SCANC, int RMODE, bool REC>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassDesc g, unsigned* words, unsigned long long limit) {
  extern __shared__ __align__(16) float lds[];
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  if (g.converge && ld_relaxed(words + kWordDone) != 0u) return;  // an earlier iteration changed nothing
  run_pass_mode<NDIM, TP, TQ, K, SCANC, RMODE, REC>(&g, g.xbuf, words, words + kWordClass, limit, lds,
                                                    xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Single-channel 3D passes on 16 x 16 tiles with K = 8: one thread per box cell.
template <bool SCANC, int RMODE, bool REC, int FMT = kImgF32>
__global__ __launch_bounds__(kCellThreads) void pass_cell_kernel(PassDesc g, unsigned* words,
                                                                 unsigned long long limit) {
  __shared__ float2 pair[2 * kCellThreads];
  __shared__ int fail;
  CellLds lds{pair, nullptr, nullptr, nullptr, &fail};
  if constexpr (SCANC) {
    __shared__ float stD[kCellStage];
    __shared__ float stI[kCellStage];
    __shared__ float res[kCellTP * kCellTQ * kCellSCR];
    lds.stD = stD;
    lds.stI = stI;
    lds.res = res;
  }
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  if (g.converge && ld_relaxed(words + kWordDone) != 0u) return;  // an earlier iteration changed nothing
  run_pass_cell_mode<SCANC, RMODE, REC, kCellTP, kCellK, FMT>(&g, g.xbuf, words, words + kWordClass, limit, lds,
                                                             xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// 2D passes of images with up to kRowMaxC channels: one wave per 32-cell tile.
template <int RMODE, int NCH, bool REC, int FMT = kImgF32>
__global__ __launch_bounds__(kRowLanes) void pass_row_kernel(PassDesc g, unsigned* words, unsigned long long limit) {
  if (ld_relaxed(words + kWordAbort) != 0u) return;
  if (g.converge && ld_relaxed(words + kWordDone) != 0u) return;  // an earlier iteration changed nothing
  run_pass_row_mode<RMODE, NCH, REC, FMT>(&g, g.xbuf, words, words + kWordClass, limit,
                                          xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

using PassKernel = void (*)(PassDesc, unsigned*, unsigned long long);

bool use_row_path(const PassDesc& d, int ndim) {
  return ndim == 2 && d.TP == 1 && d.TQ == kRowTQ && d.K == kRowK && d.C >= 1 && d.C <= kRowMaxC && d.ntp == 1;
}

template <int NCH, bool REC, int FMT = kImgF32>
PassKernel select_row_mode(int mode) {
  if (mode == kModeLam0) return pass_row_kernel<kModeLam0, NCH, REC, FMT>;
  if (NCH == 1 && mode == kModeLam1C1) return pass_row_kernel<kModeLam1C1, 1, REC, FMT>;
  return pass_row_kernel<kModeGeneral, NCH, REC, FMT>;
}

template <bool REC, int FMT = kImgF32>
PassKernel select_row_channels(const PassDesc& d) {
  if (d.C == 1) return select_row_mode<1, REC, FMT>(d.mode);
  if (d.C == 2) return select_row_mode<2, REC, FMT>(d.mode);
  return select_row_mode<3, REC, FMT>(d.mode);
}

// 16-bit images: plain forward passes only (no records).
PassKernel select_row_kernel(const PassDesc& d) {
  if (d.img_fmt == kImgBF16) return d.rec ? nullptr : select_row_channels<false, kImgBF16>(d);
  if (d.img_fmt == kImgF16) return d.rec ? nullptr : select_row_channels<false, kImgF16>(d);
  return d.rec ? select_row_channels<true>(d) : select_row_channels<false>(d);
}

bool use_cell_path(const PassDesc& d, int ndim) {
  return ndim == 3 && d.C == 1 && d.TP == kCellTP && d.TQ == kCellTQ && d.K == kCellK;
}

template <bool SCANC, int FMT>
PassKernel select_cell_fmt(const PassDesc& d) {
  if (d.rec) return nullptr;
  if (d.mode == kModeLam0) return pass_cell_kernel<SCANC, kModeLam0, false, FMT>;
  if (d.mode == kModeLam1C1) return pass_cell_kernel<SCANC, kModeLam1C1, false, FMT>;
  return pass_cell_kernel<SCANC, kModeGeneral, false, FMT>;
}

template <bool SCANC>
PassKernel select_cell_mode(const PassDesc& d) {
  // 16-bit images: plain forward passes only (no records)
  if (d.img_fmt == kImgBF16) return select_cell_fmt<SCANC, kImgBF16>(d);
  if (d.img_fmt == kImgF16) return select_cell_fmt<SCANC, kImgF16>(d);
  if (d.rec) {
    if (d.mode == kModeLam0) return pass_cell_kernel<SCANC, kModeLam0, true>;
    if (d.mode == kModeLam1C1) return pass_cell_kernel<SCANC, kModeLam1C1, true>;
    return pass_cell_kernel<SCANC, kModeGeneral, true>;
  }
  if (d.mode == kModeLam0) return pass_cell_kernel<SCANC, kModeLam0, false>;
  if (d.mode == kModeLam1C1) return pass_cell_kernel<SCANC, kModeLam1C1, false>;
  return pass_cell_kernel<SCANC, kModeGeneral, false>;
}

PassKernel select_cell_kernel(const PassDesc& d) {
  return d.sa == 1 ? select_cell_mode<true>(d) : select_cell_mode<false>(d);
}

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

// Tile geometries (kTP3, kTQ3, kTQ2 in ggdt_internal.h): 3D planes use 16 x 16
// tiles, 2D rows 256-wide tiles; the chunk length shrinks when many channels
// would overflow LDS.

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

template <int FMT>
__global__ __launch_bounds__(256) void classify_kernel(const float* image, long long n, unsigned* words) {
  const auto img = image_of<FMT>(image);
  unsigned bits = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float a = fabsf(widen<FMT>(img[i]));
    if (!(a <= 0x1p60f)) bits |= kClassHuge;
    else if (a != 0.0f && a < 0x1p-24f) bits |= a < 0x1p-40f ? (kClassSmall | kClassTiny) : kClassSmall;
  }
  const int tiny = __syncthreads_or((bits & kClassTiny) ? 1 : 0);
  const int huge = __syncthreads_or((bits & kClassHuge) ? 1 : 0);
  const int small = __syncthreads_or((bits & kClassSmall) ? 1 : 0);
  if (threadIdx.x == 0 && (tiny || huge || small))
    __hip_atomic_fetch_or(words + kWordClass,
                          (tiny ? kClassTiny : 0u) | (huge ? kClassHuge : 0u) | (small ? kClassSmall : 0u),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// End of iteration `it` in convergence mode (one thread): if no pass lowered a
// value the transform is at its fixed point (later passes return at once);
// otherwise the iteration is counted and the change word cleared.
__global__ void iteration_end_kernel(unsigned* words, int it) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (ld_relaxed(words + kWordDone) != 0u || ld_relaxed(words + kWordAbort) != 0u) return;
  if (ld_relaxed(words + kWordChanged) == 0u) {
    __hip_atomic_store(words + kWordDone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  __hip_atomic_store(words + kWordIters, (unsigned)it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(words + kWordChanged, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// out = v * mask, 16 bytes per thread and iteration when both arrays are
// 16-byte aligned (a plain streaming kernel; also the reference for the
// achievable HBM rate).
__global__ __launch_bounds__(256) void scale_kernel(const float* mask, float v, float* out, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool vec = ((reinterpret_cast<uintptr_t>(mask) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
  const long long n4 = vec ? n / 4 : 0;
  const float4* m4 = reinterpret_cast<const float4*>(mask);
  float4* o4 = reinterpret_cast<float4*>(out);
  for (long long i = t; i < n4; i += stride) {
    const float4 m = m4[i];
    o4[i] = make_float4(v * m.x, v * m.y, v * m.z, v * m.w);
  }
  for (long long i = 4 * n4 + t; i < n; i += stride) out[i] = v * mask[i];
}

struct CapEntry {
  const void* fn;
  size_t lds;
  int threads;
  int cap;
};
CapEntry g_cap_cache[256];
int g_cap_n = 0;

// Co-resident workgroups of `fn` with `lds` dynamic LDS bytes (also raises the
// kernel's dynamic-LDS limit once).  0 on failure.
int capacity_for(PassKernel fn, size_t lds, int threads = kThreads) {
  for (int i = 0; i < g_cap_n; ++i)
    if (g_cap_cache[i].fn == (const void*)fn && g_cap_cache[i].lds == lds && g_cap_cache[i].threads == threads)
      return g_cap_cache[i].cap;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, threads, lds) != hipSuccess) return 0;
  const int cap = per_cu * cus;
  if (g_cap_n < 256) g_cap_cache[g_cap_n++] = CapEntry{(const void*)fn, lds, threads, cap};
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
  if (use_row_path(d, ndim)) {
    PassKernel fn = select_row_kernel(d);
    if (!fn) return hipErrorInvalidConfiguration;
    const int cap = capacity_for(fn, 0, kRowLanes);
    if (cap <= 0) return hipErrorInvalidConfiguration;
    const int grid = d.ntq < cap ? d.ntq : cap;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kRowLanes), 0, stream, d, words, spin_limit);
    return hipGetLastError();
  }
  if (use_cell_path(d, ndim)) {
    PassKernel fn = select_cell_kernel(d);
    if (!fn) return hipErrorInvalidConfiguration;
    const int cap = capacity_for(fn, 0, kCellThreads);
    if (cap <= 0) return hipErrorInvalidConfiguration;
    const int ntiles = d.ntp * d.ntq;
    const int grid = ntiles < cap ? ntiles : cap;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kCellThreads), 0, stream, d, words, spin_limit);
    return hipGetLastError();
  }
  if (d.img_fmt != kImgF32) return hipErrorInvalidConfiguration;  // 16-bit images: cell and row kernels only
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

hipError_t launch_classify(const float* image, long long n, unsigned* words, hipStream_t stream, int img_fmt) {
  long long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  auto fn = img_fmt == kImgBF16 ? classify_kernel<kImgBF16>
                                : (img_fmt == kImgF16 ? classify_kernel<kImgF16> : classify_kernel<kImgF32>);
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, stream, image, n, words);
  return hipGetLastError();
}

hipError_t launch_iteration_end(unsigned* words, int it, hipStream_t stream) {
  hipLaunchKernelGGL(iteration_end_kernel, dim3(1), dim3(64), 0, stream, words, it);
  return hipGetLastError();
}

hipError_t launch_scale(const float* mask, float v, float* out, long long n, hipStream_t stream) {
  long long blocks = (n / 4 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, mask, v, out, n);
  return hipGetLastError();
}

}  // namespace ggdt
