// Internal declarations shared by the GGDT HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ggdt {

// Workspace layout: a 256-byte header of 32-bit words, then the tile exchange
// area (see PassDesc::xbuf), 256-byte aligned.
constexpr int kHeaderWords = 64;
constexpr int kWordAbort = 0;   // non-zero once a bounded wait expired (watchdog)
constexpr int kWordClass = 1;   // image classification bits, see below
// Convergence mode: set by a pass that lowered some value, cleared per iteration;
// set once an iteration changed nothing; the number of iterations that did.
constexpr int kWordChanged = 2;
constexpr int kWordDone = 3;
constexpr int kWordIters = 4;
constexpr int kWordSink = 5;    // written by idle lanes to keep a kernel's stores unconditional; never read
constexpr unsigned kClassTiny = 1u;   // some image value with 0 < |I| < 2^-40
constexpr unsigned kClassHuge = 2u;   // some image value with |I| > 2^60 or not finite
constexpr unsigned kClassSmall = 4u;  // some image value with 0 < |I| < 2^-24 (implied by kClassTiny)
// Values of PassDesc::sqrt_normal: when the general root's argument lies in
// the normal range where kModeGeneralN's root gives sqrtf's bits.
constexpr int kSqrtNormalNever = 0;
constexpr int kSqrtNormalUnlessHuge = 1;  // min_j A_j >= 2^-96: fmaf(lambda, g, A_j) >= A_j
constexpr int kSqrtNormalLam1 = 2;        // every A_j = 0 (lambda 1): the argument is g, which is 0 or in
                                          // [2^-94, 2^126] when no image value is small or huge

constexpr int kThreads = 256;         // threads per pass workgroup
constexpr size_t kMaxLdsBytes = 159 * 1024;  // 160 KiB per CU, less room for static LDS

// Edge-cost evaluation modes.  The fast modes give the same bits as the general
// formula whenever the classification word allows them (checked on the device).
enum Mode : int {
  kModeLam0 = 0,     // lambda == 0: w = sqrtf(A_j), a per-offset constant
  kModeLam1C1 = 1,   // lambda == 1 and C == 1: w = |I(x) - I(y)|
  kModeGeneral = 2,  // w = sqrtf(fmaf(lambda, g, A_j))
  kModeGeneralN = 3, // the same, with the root's argument known to lie in [2^-96, FLT_MAX]
};

// Storage formats of the image.  A 16-bit format is widened to fp32 on load
// (exactly: both are subsets of fp32) and every later step is the same FP32
// arithmetic as for an fp32 image.
enum ImgFmt : int {
  kImgF32 = 0,
  kImgBF16 = 1,  // bfloat16: the high 16 bits of an fp32
  kImgF16 = 2,   // IEEE binary16
};

// LDS layout of the pass kernel for one tile geometry.  A chunk stages K + 1
// planes (scan positions t0-1 .. t0+K-1) of the image and of D_old on the tile's
// box (tile grown by K on each plane axis).  When the scan axis is the
// contiguous memory axis, staged planes are stored cell-major: each cell holds a
// run of SC consecutive memory positions along the scan axis, starting at a
// multiple of 4, so that 16-byte global->LDS copies read aligned groups.
template <int NDIM, int TP, int TQ, int K, bool SCANC>
struct Layout {
  static constexpr int BQ = TQ + 2 * K;
  static constexpr int BP = NDIM == 3 ? TP + 2 * K : 1;
  static constexpr int NB = BP * BQ;               // cells of a box plane
  static constexpr int P = K + 1;                   // staged planes per chunk
  static constexpr int SC = 4 * ((K + 4 + 3) / 4);  // cell-major run: K + 1 planes + up to 3 alignment slots
  static constexpr int SCR = (K % 2 == 0) ? K + 1 : K; // odd per-cell stride of staged results
  static constexpr int STAGE = SCANC ? NB * SC : NB * P;  // floats of one staged array
  static constexpr int RES = SCANC ? TP * TQ * SCR : 0;   // floats of the staged results
  // two (D, I) pair planes, the staged D_old and image arrays, the staged results
  static constexpr size_t bytes(int C) { return sizeof(float) * (size_t)(4 * NB + STAGE * (1 + C) + RES); }
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
  unsigned long long* xbuf;  // exchange words [2][ntp * ntq][TP * TQ]
  int N;               // voxels per channel
  int sa, sp, sq;      // element strides of the scan axis and of p, q
  int Na, Np, Nq;
  int sign;
  int C;
  int TP, TQ, K;       // plane tile and chunk length (select the kernel instantiation)
  int ntp, ntq;        // tiles along p and q
  int nchunk;          // ceil((Na - 1) / K)
  int init;            // D_old := v * M (first pass of a schedule)
  int mode;            // requested Mode
  float v, lam;
  float A[9];          // (float)((1 - lambda) * |dx|_s^2) per offset j
  float W0[9];         // sqrtf(A[j]), used when lambda == 0
  unsigned epoch_base; // exchange words of chunk c carry epoch_base + c + 1
  int sqrt_normal;     // kSqrtNormal*: when the general root may use kModeGeneralN
  int converge;        // convergence mode: skip when done, report changes in kWordChanged
  int img_fmt;         // ImgFmt of `image` (16-bit formats: image points to 2-byte elements)
  // Batched launches only.  op != kOpPass: instead of a pass, the instance's
  // workgroups change the layout of the esz-byte volume [Np][Nq][Na] at
  // `image` into `D` (kOpToScanMajor: to [Na][Np][Nq]; kOpFromScanMajor:
  // back).  image_off / d_off / rec_off >= 0: `image` / `D` / `rec` are at
  // that byte offset of the launch's workspace (the instance's scan-major
  // copies and records staging).
  int op;
  int esz;
  long long image_off;
  long long d_off;
  long long rec_off;
};
enum PassOp : int { kOpPass = 0, kOpToScanMajor = 1, kOpFromScanMajor = 2 };

// Reverse of one forward pass (see backward_device.h).  Geometry fields as in
// PassDesc; abar is read from a_in and written to a_out; gI accumulates dL/dI.
struct BwdDesc {
  const float* image;   // (C, N)
  const uint8_t* rec;   // records of the forward pass (N)
  const float* a_in;    // (N)
  float* a_out;         // (N)
  float* gI;            // (C, N)
  unsigned long long* xbuf;
  int N;
  int sa, sp, sq;
  int Na, Np, Nq;
  int sign;
  int C;
  int TP, TQ, K;
  int ntp, ntq;
  int nchunk;           // ceil((Na - 1) / K)
  int mode;
  float lam;
  float A[9];
  unsigned epoch_base;
  long long a_in_off;   // >= 0: a_in is at this byte offset of the workspace (batched scratch)
  long long a_out_off;  // >= 0: same for a_out
  int sqrt_normal;      // as in PassDesc
  // Batched launches only (as PassDesc::op).  op != kOpPass: a layout change
  // of the instance's esz-byte volume [Np][Nq][Na] at lsrc into ldst (K tiles
  // per round); for passes, image_off / rec_off / gi_off >= 0 place image /
  // rec / gI at that byte offset of the workspace (lsrc_off / ldst_off the
  // same for an op's operands).
  int op;
  int esz;
  const void* lsrc;
  void* ldst;
  long long lsrc_off, ldst_off, image_off, rec_off, gi_off;
};

// One instance of a batched launch (device-resident table).  Its passes are
// entries [pass0, pass0 + npass) of the pass table; it runs on logical
// workgroups [wg0, wg0 + nwg).  Offsets are in bytes from the workspace base.
struct BatchInst {
  int ndim;
  int mode;            // requested Mode
  int npass;
  int pass0;
  int wg0, nwg;
  long long xbuf_off;  // exchange words of this instance
  long long ctr_off;   // pass-barrier counter (one 32-bit word)
  long long cls_off;   // image classification word
  const float* image;  // for the classification
  long long nimg;      // C * N
};

// Tile geometry of the batched kernels (3D plane tile TP3 x TQ3, 2D row tile TQ2).
constexpr int kTP3 = 16, kTQ3 = 16, kTQ2 = 256;
// 2D row kernel (pass_row.h): one 64-lane wave per tile, chunks of kRowK rows,
// kRowTQ = 64 - 2 kRowK owned cells per tile, images of up to kRowMaxC channels.
constexpr int kRowLanes = 64, kRowK = 16, kRowTQ = kRowLanes - 2 * kRowK, kRowMaxC = 3;

// Batched kernel classes: 0 for single-channel batches (3D: thread-per-cell
// pass on 16 x 16 tiles, K = 8); 1 for up to 4 channels (tile passes, K = 4 /
// 16); 2 single-channel, chosen by tuning (3D: thread-per-cell pass on 24 x 24
// tiles, K = 4, less halo arithmetic for twice the exchanges).  Chunk lengths
// (3D / 2D), 3D tile side, channel limit:
constexpr int kBatchK3[3] = {8, 4, 4};
constexpr int kBatchK2[3] = {32, 16, 32};
constexpr int kBatchTile3[3] = {16, 16, 24};
constexpr int kBatchMaxC[3] = {1, 4, 1};

size_t batched_lds_bytes(int kclass, int C, bool has2d, bool has3d);
int batched_capacity(int kclass, bool rec, size_t lds);
hipError_t launch_batched(int kclass, bool rec, const BatchInst* insts, int ninst, const PassDesc* passes,
                          unsigned char* ws, int grid, size_t lds, unsigned long long spin_limit, hipStream_t stream);
hipError_t launch_batched_classify(const BatchInst* insts, int ninst, unsigned char* ws, hipStream_t stream);

// Chunk length of the backward kernels for a geometry (0 if none fits).
int bwd_chunk_for(int ndim, int C, bool scan_contiguous);
hipError_t launch_bwd_pass(const BwdDesc& d, int ndim, unsigned* words, unsigned long long spin_limit,
                           hipStream_t stream);
size_t batched_bwd_lds_bytes(int c2, int c3);
// Batched reverse kernel class: 0 when every instance is a single-channel volume
// (thread-per-cell reverse pass), else 1 (tile reverse passes).
int batched_bwd_capacity(int bclass, size_t lds);
hipError_t launch_batched_bwd(int bclass, const BatchInst* insts, int ninst, const BwdDesc* passes, unsigned char* ws,
                              int grid, size_t lds, unsigned long long spin_limit, hipStream_t stream);
// Chunk lengths of the batched backward kernel.
constexpr int kBwdBatchK3 = 4, kBwdBatchK2 = 16;
// Chunk length of single-channel 3D instances in batched reverse passes (the
// thread-per-cell reverse pass).
constexpr int kBwdBatchKCell = 8;

// Pick the chunk length for a tile geometry so that the kernel's LDS fits.
// Returns 0 if no instantiation fits (too many channels).
int pass_chunk_for(int ndim, int C, bool scan_contiguous);

// Launch one directional pass.  `words` is the workspace header.  Returns a
// hipError_t (hipErrorInvalidConfiguration if no kernel fits).
hipError_t launch_pass(const PassDesc& d, int ndim, unsigned* words, unsigned long long spin_limit,
                       hipStream_t stream);

hipError_t launch_reset(unsigned* ws, long long nwords, hipStream_t stream);
hipError_t launch_classify(const float* image, long long n, unsigned* words, hipStream_t stream,
                           int img_fmt = kImgF32);
hipError_t launch_scale(const float* mask, float v, float* out, long long n, hipStream_t stream);
// Layout changes of a [D0][D1][D2] volume of 4-, 2- or 1-byte elements (layout.hip):
// to [D2][D0][D1] and back.  With `skip` non-null, a launch finding *skip != 0
// does nothing.
hipError_t launch_to_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                const unsigned* skip, hipStream_t stream);
hipError_t launch_from_scan_major(const void* src, void* dst, int elem_bytes, int D0, int D1, int D2,
                                  const unsigned* skip, hipStream_t stream);
hipError_t launch_iteration_end(unsigned* words, int it, hipStream_t stream);

// Pointwise steps of the signed distance and the geodesic symmetric filter
// (compose.hip), FP32, element i of n:
//   kOpComplement  out = 1 - a
//   kOpObjectMask  out = a < s ? 0 : 1
//   kOpSub         out = a - b
//   kOpSumShift    out = (a + b) + s
enum ComposeOp { kOpComplement = 0, kOpObjectMask = 1, kOpSub = 2, kOpSumShift = 3 };
hipError_t launch_compose(int op, const float* a, const float* b, float s, float* out, long long n,
                          hipStream_t stream);

}  // namespace ggdt
