// Internal declarations shared by the GGDT HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ggdt {

// Workspace layout: a 256-byte header of 32-bit words, then one progress word per
// tile (rounded up to 256 bytes).
constexpr int kHeaderWords = 64;
constexpr int kWordAbort = 0;   // non-zero once a bounded wait expired (watchdog)
constexpr int kWordClass = 1;   // image classification bits, see below
constexpr unsigned kClassTiny = 1u;  // some image value with 0 < |I| < 2^-40
constexpr unsigned kClassHuge = 2u;  // some image value with |I| > 2^60 or not finite

// Edge-cost evaluation modes.  The fast modes give the same bits as the general
// formula whenever the classification word allows them (checked on the device).
enum Mode : int {
  kModeLam0 = 0,     // lambda == 0: w = sqrtf(A_j), a per-offset constant
  kModeLam1C1 = 1,   // lambda == 1 and C == 1: w = |I(x) - I(y)|
  kModeGeneral = 2,  // w = sqrtf(fmaf(lambda, g, A_j))
};

// Geometry and parameters of one directional pass over one instance.  The pass
// runs along the scan axis (length Na, element stride sa); rows/planes are
// indexed by (p, q), p the slower and q the faster of the non-scan axes (in 2D,
// Np = 1).  Plane k of the pass is the k-th position along the scan axis in
// array order; sign = +1 scans k = 1 .. Na-1, sign = -1 scans k = Na-2 .. 0.
struct PassDesc {
  const float* image;  // (C, N)
  const float* mask;   // (N), read when init != 0
  float* D;            // (N), in/out
  uint8_t* rec;        // (N) records of this pass, or nullptr
  int N;               // voxels per channel
  int sa, sp, sq;      // element strides of the scan axis and of p, q
  int Na, Np, Nq;
  int sign;
  int C;
  int TP, TQ;          // plane tile (must match the kernel instantiation)
  int K;               // scan steps per chunk (1 <= K <= min(TP (3D), TQ))
  int ntp, ntq;        // tiles along p and q
  int nchunk;          // ceil((Na - 1) / K)
  int init;            // D_old := v * M (first pass of a schedule)
  int mode;            // requested Mode
  float v, lam;
  float A[9];          // (float)((1 - lambda) * |dx|_s^2) per offset j
  float W0[9];         // sqrtf(A[j]), used when lambda == 0
  unsigned flag_base;  // progress words of this pass count up from flag_base
};

// Launch one directional pass.  `words` is the workspace header, `flags` the
// per-tile progress words (at least ntp * ntq).  Returns a hipError_t.
hipError_t launch_pass(const PassDesc& d, int ndim, unsigned* words, unsigned* flags,
                       unsigned long long spin_limit, int grid_cap, hipStream_t stream);

// Largest grid of co-resident workgroups for the pass kernel that `d` selects.
int pass_grid_capacity(const PassDesc& d, int ndim);

// LDS bytes the pass kernel needs for this geometry.
size_t pass_lds_bytes(const PassDesc& d, int ndim);

hipError_t launch_reset(unsigned* ws, int nwords, hipStream_t stream);
hipError_t launch_classify(const float* image, long long n, unsigned* words, hipStream_t stream);
hipError_t launch_scale(const float* mask, float v, float* out, long long n, hipStream_t stream);

}  // namespace ggdt
