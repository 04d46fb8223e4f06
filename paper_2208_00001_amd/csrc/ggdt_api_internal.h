// Host-side helpers shared by the C-ABI sources (not part of the C ABI).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "ggdt_internal.h"

namespace ggdt {

constexpr int kMaxChannels = 16;
constexpr unsigned long long kDefaultSpinLimit = 1ull << 21;
constexpr int kTileP3 = 16, kTileQ3 = 16;  // 3D plane tile
constexpr int kTileQ2 = 256;              // 2D row tile

extern unsigned long long g_spin_limit;

struct Problem {
  int ndim;
  int dims[3];
  int C;
  long long N;
};

struct Tuning {
  int tile_p = 0;
  int tile_q = 0;
  int chunk = 0;
  int wg_per_cu = 0;
};

const char* status_text(int status);
// Record the profiling event before / after a profiled kernel launch (no-ops
// when profiling is off or its capacity is used up).
void prof_before(hipStream_t stream);
void prof_after(hipStream_t stream);
// Build the pass descriptor of pass number p (0-based, schedule order) of an
// instance; xbuf is left null.
int build_pass(const Problem& pr, const float* image, const float* mask, const float* spacing, float v, float lam,
               float* out, uint8_t* records, int p, unsigned epoch_base, PassDesc* d);
// Launch a pass kernel, recording profiling events around it when profiling is on.
hipError_t launch_pass_profiled(const PassDesc& d, int ndim, unsigned* words, hipStream_t stream);
int check_device();
int make_problem(int ndim, const int* dims, int C, Problem* pr);
int check_params(int ndim, const float* spacing, float v, float lam, int iterations);
int check_alias(const void* out, size_t nout, const void* const* ins, const size_t* nins, int nin);
void tile_shape(const Problem& pr, const Tuning& tu, int* TP, int* TQ);
void pass_geometry(const Problem& pr, int axis, PassDesc* d);
void edge_constants(const Problem& pr, int axis, const float* spacing, float lam, float* A, float* W0);
int sqrt_normal_for(const float* A, int n);  // kSqrtNormal* for the constants A_0..A_{n-1}
int requested_mode(float lam, int C);
int max_tiles(const Problem& pr, const Tuning& tu);
int build_bwd_pass(const Problem& pr, const float* image, const uint8_t* records, const float* spacing, float lam,
                   float* gI, int p, int K, unsigned epoch_base, BwdDesc* d);
size_t workspace_for(const Problem& pr, const Tuning& tu);
// Scan-major copies of D and of the image for the passes along the last axis
// of a single-channel volume (see layout.hip).
size_t scan_major_bytes(const Problem& pr);
size_t scan_major_vol_bytes(const Problem& pr);  // one fp32 volume, 256-byte aligned
struct ScanMajor {
  bool on;
  float* D;      // D laid out [W][D][H]
  void* image;   // the image in its storage format, laid out [W][D][H]
  uint8_t* rec;  // one pass's records laid out [W][D][H] (forward with records)
};
// The copies in `buf` (scan_major_bytes(pr) bytes), if the schedule uses them.
ScanMajor scan_major_for(const Problem& pr, const uint8_t* records, void* buf);
// The scan-major area of a forward workspace of wsb bytes (after the first
// workspace_for(pr, tu) bytes), or null if the workspace has no room for it.
void* scan_major_in(const Problem& pr, const Tuning& tu, void* ws, size_t wsb);
// Enqueue the whole forward schedule of one instance on `stream` (arguments
// already validated; ws holds at least workspace_for(pr, tu) bytes).  With
// `scan_major` (scan_major_bytes(pr) bytes, or null) the passes along the last
// axis of a single-channel volume without records run on scan-major copies.
int enqueue_forward(const Problem& pr, const float* image, const float* mask, const float* spacing, float v,
                    float lam, int iterations, float* out, uint8_t* records, void* ws, const Tuning& tu,
                    hipStream_t stream, int img_fmt = kImgF32, void* scan_major = nullptr);

}  // namespace ggdt
