// Pointwise kernels of the signed distance and the geodesic symmetric filter:
// streaming FP32 maps over whole volumes, 16 bytes per lane and iteration when
// every operand is 16-byte aligned.  out may be a (in place).
#include "ggdt_internal.h"

namespace ggdt {
namespace {

template <int OP>
__device__ __forceinline__ float apply(float a, float b, float s) {
  if (OP == kOpComplement) return 1.0f - a;
  if (OP == kOpObjectMask) return a < s ? 0.0f : 1.0f;
  if (OP == kOpSub) return a - b;
  return (a + b) + s;
}

template <int OP>
__global__ __launch_bounds__(256) void compose_kernel(const float* a, const float* b,
                                                      float s, float* out, long long n) {
  constexpr bool USE_B = OP == kOpSub || OP == kOpSumShift;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const uintptr_t bits = reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(out) |
                         (USE_B ? reinterpret_cast<uintptr_t>(b) : 0u);
  const long long n4 = (bits & 15u) == 0 ? n / 4 : 0;
  for (long long i = t; i < n4; i += stride) {
    const float4 x = reinterpret_cast<const float4*>(a)[i];
    const float4 y = USE_B ? reinterpret_cast<const float4*>(b)[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    reinterpret_cast<float4*>(out)[i] =
        make_float4(apply<OP>(x.x, y.x, s), apply<OP>(x.y, y.y, s), apply<OP>(x.z, y.z, s), apply<OP>(x.w, y.w, s));
  }
  for (long long i = 4 * n4 + t; i < n; i += stride) out[i] = apply<OP>(a[i], USE_B ? b[i] : 0.0f, s);
}

}  // namespace

hipError_t launch_compose(int op, const float* a, const float* b, float s, float* out, long long n,
                          hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n / 4 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(256);
  switch (op) {
    case kOpComplement: hipLaunchKernelGGL(compose_kernel<kOpComplement>, grid, block, 0, stream, a, b, s, out, n); break;
    case kOpObjectMask: hipLaunchKernelGGL(compose_kernel<kOpObjectMask>, grid, block, 0, stream, a, b, s, out, n); break;
    case kOpSub: hipLaunchKernelGGL(compose_kernel<kOpSub>, grid, block, 0, stream, a, b, s, out, n); break;
    case kOpSumShift: hipLaunchKernelGGL(compose_kernel<kOpSumShift>, grid, block, 0, stream, a, b, s, out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ggdt
