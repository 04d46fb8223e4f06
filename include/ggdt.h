/*
 * ggdt.h — C ABI of the MI355X (gfx950) generalised geodesic distance transform.
 *
 * Method (FastGeodis paper, section "Implementation"; formula of the generalised
 * GDT of Criminisi et al. 2008 that the paper implements, section "Statement of
 * need"):
 *
 *   D0(x)   = v * M(x)                                   M: soft seed mask in [0, 1]
 *   w(x, y) = sqrt((1 - lambda) * |x - y|_s^2 + lambda * sum_c (I_c(x) - I_c(y))^2)
 *   a pass along axis a, direction +1 (ascending) or -1 (descending), visits the
 *   rows (2D) / planes (3D) orthogonal to a in scan order; every voxel x of a
 *   row/plane is updated in parallel from the 3 (2D) / 9 (3D) neighbours y in the
 *   previous row/plane (already updated by this pass):
 *       D(x) <- min(D(x), min_y D(y) + w(x, y))
 *   one iteration = passes (axis 0, +1), (0, -1), (1, +1), (1, -1) [, (2, +1), (2, -1)].
 *
 * FP32 operation sequence (bitwise reproducible against a CPU implementation):
 *   d_c = I_c(x) - I_c(y);  g = d_0 * d_0;  g = fmaf(d_c, d_c, g) (c = 1..C-1)
 *   w = sqrtf(fmaf(lambda, g, A)),  A = (float)((1 - (double)lambda) * S),
 *   S = sum over axes b ascending of (double(s_b) * |x_b - y_b|)^2 in double;
 *   cand = D(y) + w; ties keep the current value, then the earlier offset in
 *   lexicographic order over the non-scan axes (ascending axis, -1, 0, +1).
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers of the current HIP device, fp32,
 *     C-contiguous (row-major): image (C, [D,] H, W), softmask and out ([D,] H, W).
 *     spacing is a HOST pointer to ndim floats in array-axis order ([D,] H, W).
 *   - All buffers are owned by the caller.  The library allocates no device memory
 *     on these paths; per-call scratch lives in the caller's workspace.
 *   - Work is enqueued on `stream` and runs asynchronously; the call returns after
 *     validation and enqueueing.  Device-side faults surface at the next sync.
 *   - Validation happens before anything is enqueued: on an error return nothing
 *     has been written.
 *   - Calls that share one workspace must not overlap in time (same stream, or
 *     synchronised); distinct workspaces may run concurrently.
 *   - No C++ exception crosses this boundary.
 *
 * Domain: v finite and >= 0, lambda in [0, 1], spacing finite and > 0,
 * iterations >= 0, 1 <= C <= 16, every dimension >= 1.  Non-finite image or mask
 * values are not rejected; results for them are unspecified.
 */
#ifndef GGDT_H_
#define GGDT_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  0 = success, negative = error. */
#define GGDT_OK 0
#define GGDT_ERR_NULL_PTR -1            /* a required pointer is NULL */
#define GGDT_ERR_BAD_SHAPE -2           /* ndim, C or a dimension out of range, or size overflow */
#define GGDT_ERR_BAD_PARAM -3           /* v, lambda, spacing or iterations outside the domain */
#define GGDT_ERR_WORKSPACE_TOO_SMALL -4 /* workspace_bytes below the required size */
#define GGDT_ERR_HIP -5                 /* a HIP runtime call or kernel launch failed */
#define GGDT_ERR_WATCHDOG -6            /* a bounded inter-workgroup wait expired (see ggdt_workspace_status) */
#define GGDT_ERR_ALIAS -7               /* an output overlaps an input */
#define GGDT_ERR_UNSUPPORTED -8         /* valid request this build cannot run (e.g. no gfx950 device) */

/* Human-readable text for a status code (static storage, never NULL). */
const char* ggdt_strerror(int status);

/* Bytes of device workspace the forward entry points (plain, records,
 * fixed point, 16-bit image) use for a problem of `ndim` (2 or 3) spatial dims
 * `dims` (array-axis order) and C channels.  Returns 0 for invalid shapes.  The
 * workspace holds inter-workgroup progress flags, the image classification
 * word and the watchdog word; its content need not be initialised by the
 * caller.  For single-channel volumes it also holds copies of D and of the
 * image laid out [W][D][H] (the last axis slowest), on which the passes along
 * the last axis run as strided passes, and room for one such pass's records
 * before they are moved to the array layout (a library addition; the passes
 * compute the same values and records).  ggdt_workspace_min_bytes is the smallest size the
 * forward accepts: with less than ggdt_workspace_bytes it runs those passes in
 * place, more slowly.  The two are equal for images and multi-channel
 * volumes. */
size_t ggdt_workspace_bytes(int ndim, const int* dims, int C);
size_t ggdt_workspace_min_bytes(int ndim, const int* dims, int C);

/* Plain forward, 2D: out = GGDT(image, softmask) after `iterations` iterations of
 * the four passes.  iterations = 0 writes v * softmask.  `out` must not overlap
 * `image` or `softmask`. */
int ggdt2d(const float* image, const float* softmask, const float* spacing, float v, float lambda,
           int iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
           hipStream_t stream);

/* Plain forward, 3D: as ggdt2d with six passes per iteration and spacing[3]. */
int ggdt3d(const float* image, const float* softmask, const float* spacing, float v, float lambda,
           int iterations, float* out, int C, int D, int H, int W, void* workspace,
           size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------- 16-bit image storage
 * The same forward with the image stored in a 16-bit format, which halves the
 * image bytes every pass reads (12 -> 10 bytes per voxel update for one
 * channel).  Every value is widened to fp32 exactly on load and the transform
 * then runs the FP32 operation sequence above unchanged, so the result equals
 * ggdt2d/ggdt3d on the widened image bit for bit; its difference from ggdt2d/
 * ggdt3d on the original fp32 image is the effect of rounding the image to the
 * 16-bit format (bf16 keeps 8 significant bits, binary16 11 and a smaller
 * range).  `image` points to 2-byte elements, layout (C, [D,] H, W) as above;
 * `format` is GGDT_IMAGE_BF16 (bfloat16: the high half of an fp32) or
 * GGDT_IMAGE_F16 (IEEE binary16), else GGDT_ERR_BAD_PARAM.  Supported: 2D with
 * C <= 3 and 3D with C = 1 (GGDT_ERR_UNSUPPORTED otherwise); same workspace as
 * ggdt2d/ggdt3d. */
#define GGDT_IMAGE_BF16 1
#define GGDT_IMAGE_F16 2
int ggdt2d_half(const uint16_t* image, int format, const float* softmask, const float* spacing, float v,
                float lambda, int iterations, float* out, int C, int H, int W, void* workspace,
                size_t workspace_bytes, hipStream_t stream);
int ggdt3d_half(const uint16_t* image, int format, const float* softmask, const float* spacing, float v,
                float lambda, int iterations, float* out, int C, int D, int H, int W, void* workspace,
                size_t workspace_bytes, hipStream_t stream);

/* Bytes of argmin records for the forward-with-records entries (records feed
 * the backward below; they are not part of the paper's transform):
 * iterations * (2 * ndim) * prod(dims).  Layout: one byte per voxel per pass,
 * pass-major (pass p = iteration * 2*ndim + 2*axis + (descending ? 1 : 0)), voxels
 * row-major inside a pass.  Value 0 = the voxel kept its value in that pass;
 * 1 + j = it took D(y) + w through offset j, where j enumerates the offsets over
 * the non-scan axes lexicographically (ascending axis, components -1, 0, +1):
 * j = delta_q + 1 in 2D, j = 3 * (delta_p + 1) + (delta_q + 1) in 3D, with p < q the
 * non-scan axes and y = x - sign * e_axis + delta. */
size_t ggdt_records_bytes(int ndim, const int* dims, int iterations);

/* Forward that also writes the argmin records (device, ggdt_records_bytes bytes).
 * `out` equals the plain forward's bit for bit. */
int ggdt2d_forward_rec(const float* image, const float* softmask, const float* spacing, float v,
                       float lambda, int iterations, float* out, uint8_t* records, int C, int H, int W,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);
int ggdt3d_forward_rec(const float* image, const float* softmask, const float* spacing, float v,
                       float lambda, int iterations, float* out, uint8_t* records, int C, int D, int H,
                       int W, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Forward run to its fixed point.  The paper's transform repeats the directional
 * passes for a given number of iterations (section "Implementation"); each
 * iteration can only lower D, so repeating until an iteration changes nothing
 * gives the converged transform, the exact shortest-path distance on the 8/26-
 * connected grid with the same edge costs.  Runs whole iterations (same
 * schedule and arithmetic as ggdt2d/ggdt3d) until one lowers no value, at most
 * max_iterations (>= 0); arguments otherwise as ggdt2d/ggdt3d, same workspace
 * size.  Iterations are enqueued in blocks (4, 4, 8, 16, ...); between blocks
 * the call synchronises `stream` and reads the workspace's done word, so it
 * returns once the fixed point has been seen or max_iterations are enqueued,
 * with at most one block of (immediately returning) passes after the fixed
 * point.  It therefore cannot be captured into a HIP graph.  The number of
 * iterations comes from ggdt_workspace_iterations.  out then equals
 * ggdt2d/ggdt3d with that many iterations (with max_iterations when it did not
 * converge). */
int ggdt2d_converge(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int max_iterations, float* out, int C, int H, int W, void* workspace,
                    size_t workspace_bytes, hipStream_t stream);
int ggdt3d_converge(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int max_iterations, float* out, int C, int D, int H, int W, void* workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* After a ggdt{2,3}d_converge call on `stream` with this workspace: synchronises
 * the stream and stores in *iterations the number of iterations that lowered
 * some value (the fixed point was confirmed by the next one), or -1 if
 * max_iterations passed without reaching it.  GGDT_ERR_WATCHDOG if an
 * inter-workgroup wait of the call expired. */
int ggdt_workspace_iterations(const void* workspace, hipStream_t stream, int* iterations);

/* ------------------------------------------------------------------ backward
 * The paper defines the forward transform only.  The argmin records and the
 * reverse pass below are this library's addition for training use: gradients
 * of a loss of D with respect to the image and the soft mask, obtained by
 * running the recorded minimisations of the forward schedule in reverse. */

/* Bytes of device workspace the backward entry points use: the forward's
 * minimal workspace plus one fp32 adjoint buffer of prod(dims) values, plus,
 * for single-channel volumes, scan-major copies (image, two adjoint volumes,
 * dL/dI, two passes' records) on which the reverses of the passes along the
 * last axis run as strided passes.  ggdt_backward_workspace_min_bytes is the
 * smallest size accepted (without the copies those reverse passes run in
 * place, more slowly).  0 for invalid shapes.  1 <= C <= 8 for the backward. */
size_t ggdt_backward_workspace_bytes(int ndim, const int* dims, int C);
size_t ggdt_backward_workspace_min_bytes(int ndim, const int* dims, int C);

/* Backward: exact reverse of the recorded schedule.  Given dL/dD (grad_out) and
 * the records of the forward with the same image, spacing, v, lambda and
 * iterations, writes dL/dI (grad_image, shape of image) and dL/dM (grad_softmask,
 * shape of softmask).  Where w = 0 the derivative of w is taken as 0.  The
 * adjoint is carried pass by pass in grad_softmask and the workspace's adjoint
 * buffer; outputs must not overlap the inputs or each other.  Records from a
 * different schedule give unspecified gradients (never out-of-bounds accesses). */
int ggdt2d_backward(const float* image, const uint8_t* records, const float* grad_out,
                    const float* spacing, float v, float lambda, int iterations, float* grad_image,
                    float* grad_softmask, int C, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);
int ggdt3d_backward(const float* image, const uint8_t* records, const float* grad_out,
                    const float* spacing, float v, float lambda, int iterations, float* grad_image,
                    float* grad_softmask, int C, int D, int H, int W, void* workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------ signed distance and GSF
 * The paper lists a signed geodesic distance and the geodesic symmetric filter
 * (GSF, after Criminisi et al. 2008) among what the software computes (sections
 * "Statement of need" and "Implementation") but does not define them.  This
 * library's reading, composed from the transform above (same schedule and FP32
 * arithmetic) and FP32 pointwise steps:
 *   S(M)  = D(I; M) - D(I; 1 - M)      negative where M marks the object (M = 0)
 *   obj(S, t) = mask of {x : S(x) < t}  (0 on the set, 1 elsewhere)
 *   GSF   = (S(obj(S0, theta_d)) + S(obj(S0, -theta_e))) + (theta_e - theta_d),
 *           S0 = S(M): the closing (dilate by theta_d, erode by theta_e) and the
 *           opening (erode, then dilate) merged through their signed distances;
 *           the filtered object is {GSF < 0}.
 * theta_e - theta_d is rounded to FP32 once.  Shapes, layouts, streams and
 * errors as ggdt2d/ggdt3d; out must not overlap image, softmask or the
 * workspace.  theta_d, theta_e must be finite and >= 0 (else
 * GGDT_ERR_BAD_PARAM). */

/* Workspace bytes: the transform's minimal workspace plus 2 (signed) or 4
 * (GSF) fp32 buffers of prod(dims) values, plus, for single-channel volumes,
 * the scan-major area described at ggdt_workspace_bytes (with less room, the
 * passes along the last axis run in place).  0 for invalid shapes. */
size_t ggdt_signed_workspace_bytes(int ndim, const int* dims, int C);
size_t ggdt_gsf_workspace_bytes(int ndim, const int* dims, int C);

/* out = S(M) with `iterations` iterations for both transforms. */
int ggdt2d_signed(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                  int iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
                  hipStream_t stream);
int ggdt3d_signed(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                  int iterations, float* out, int C, int D, int H, int W, void* workspace,
                  size_t workspace_bytes, hipStream_t stream);

/* out = GSF (six transforms, `iterations` iterations each). */
int ggdt2d_gsf(const float* image, const float* softmask, const float* spacing, float theta_d, float theta_e,
               float v, float lambda, int iterations, float* out, int C, int H, int W, void* workspace,
               size_t workspace_bytes, hipStream_t stream);
int ggdt3d_gsf(const float* image, const float* softmask, const float* spacing, float theta_d, float theta_e,
               float v, float lambda, int iterations, float* out, int C, int D, int H, int W, void* workspace,
               size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------- Toivanen's raster scan
 * The paper's software ships Toivanen's sequential raster scan as the
 * single-thread comparison method (section "Implementation"); it names the
 * method without describing it.  Reading: one iteration is a forward sweep over
 * the voxels in raster order (array order, every axis ascending) and then a
 * backward sweep in the reverse order; each voxel x in turn takes
 * min(D(x), D(y) + w(x, y)) over the neighbours y of its 8 (2D) / 26 (3D)
 * neighbourhood that precede it in the sweep (4 / 13 of them), updating D in
 * place, with the edge cost and FP32 operation sequence of the passes.  Here
 * the sweeps run on the GPU by hyperplanes t = 4z + 2y + x (every preceding
 * neighbour lies on an earlier hyperplane), which gives the sequential sweep's
 * values bit for bit.  D0 = v * softmask; iterations = 0 writes v * softmask.
 * Arguments, workspace (ggdt_workspace_min_bytes suffices), aliasing rules and
 * status codes as ggdt2d / ggdt3d.  One persistent launch for all iterations:
 * row blocks (slabs of whole planes of a volume, bands of image rows) run as a
 * pipeline, each waiting, bounded, for its one neighbour's progress
 * (GGDT_ERR_WATCHDOG via ggdt_workspace_status if a wait expires); returns
 * GGDT_ERR_UNSUPPORTED if the blocks cannot all be co-resident. */
int ggdt2d_toivanen(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int iterations, float* out, int C, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);
int ggdt3d_toivanen(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                    int iterations, float* out, int C, int D, int H, int W, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/* ------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory, not even a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): ggdt3d without the workspace arguments.  Its inter-workgroup
 * scratch lives in a fixed device array of GGDT_NOALLOC_SCRATCH_BYTES inside
 * the library (one per GPU, kept until the process ends); the call allocates
 * nothing; the passes run in place (no scan-major copies).  Problems whose
 * scratch exceeds it (ggdt_workspace_min_bytes above
 * GGDT_NOALLOC_SCRATCH_BYTES: planes of about 512 x 512 voxels and larger)
 * return GGDT_ERR_WORKSPACE_TOO_SMALL before anything is enqueued.  Every
 * call on one GPU uses that GPU's array, so calls that overlap in time on one
 * GPU (different streams, threads) race; calls on one stream are ordered.
 * Arguments, results, streams and errors otherwise as ggdt3d; the watchdog
 * word cannot be queried for this entry. */
#define GGDT_NOALLOC_SCRATCH_BYTES ((size_t)4 * 1024 * 1024 + 4096)
int ggdt3d_noalloc(const float* image, const float* softmask, const float* spacing, float v, float lambda,
                   int iterations, float* out, int C, int D, int H, int W, hipStream_t stream);

/* After the stream has finished a call, report whether its inter-workgroup waits
 * all completed: synchronises `stream`, returns GGDT_OK or GGDT_ERR_WATCHDOG (the
 * results of that call are then invalid).  `workspace` is the one the call used. */
int ggdt_workspace_status(const void* workspace, hipStream_t stream);

/* Debug knob: upper bound on polls of one inter-workgroup wait before the
 * watchdog fires (default 2^21).  Process-wide; 0 restores the default. */
void ggdt_set_spin_limit(unsigned long long polls);

/* Profiling (process-wide, not thread-safe).  After ggdt_profile_begin(n) the
 * forward and backward entry points record a HIP event pair on their stream
 * around each of their next n directional-pass kernel launches.
 * ggdt_profile_end synchronises those events, writes up to `capacity` launch
 * durations in milliseconds to `ms` (host) and returns how many launches were
 * recorded (or a negative status); it also ends profiling.  Begin allocates host
 * event objects only. */
int ggdt_profile_begin(int n);
int ggdt_profile_end(float* ms, int capacity);

/* ------------------------------------------------------------------ batched
 * Not from the paper, which runs one image or volume per call: this library's
 * addition for training use.  Many instances of uneven size, each with its own
 * spacing, v, lambda and iterations, run in one persistent launch with the
 * same schedule and FP32 arithmetic as the plain entries (outputs equal theirs
 * bit for bit). */

/* One instance of a ragged batch.  Same meaning and layout as the plain entry
 * points; dims[2] is ignored for ndim = 2; records may be NULL (then the backward
 * cannot run for this instance).  grad_* are used only by
 * ggdt_batched_backward and may be NULL otherwise. */
typedef struct ggdt_instance {
  int ndim;
  int C;
  int dims[3];
  const float* image;
  const float* softmask;
  float* out;
  float spacing[3];
  float v;
  float lambda;
  int iterations;
  uint8_t* records;
  const float* grad_out;
  float* grad_image;
  float* grad_softmask;
} ggdt_instance;

typedef struct ggdt_plan ggdt_plan;

/* Build a plan for n instances: validates every instance, splits the device's
 * resident workgroup slots among them and lays out the device descriptor table.
 * `tuning` (nullable) overrides tile geometry: see ggdt_tuning.  Writes the
 * workspace size the plan needs.  The plan (host object) is owned by the library
 * until ggdt_plan_destroy.  Errors are those of the plain entries, for the first
 * offending instance. */
typedef struct ggdt_tuning {
  int tile_p;      /* 3D plane tile side: 0 or 16 (default), or 24 (single-channel batches only; 24 x 24
                      tiles with chunk 4: less halo arithmetic for more exchanges); other values
                      GGDT_ERR_BAD_PARAM */
  int tile_q;      /* same as tile_p (either selects the side) */
  int chunk;       /* scan steps between inter-workgroup syncs: 0 (default), 8 or 32 (single-channel
                      kernels), 4 or 16 (kernels for up to 4 channels); 0 or 4 with tile side 24 */
  int wg_per_cu;   /* resident workgroups per compute unit to plan for (0 = default) */
} ggdt_tuning;

int ggdt_batched_plan(const ggdt_instance* instances, int n, const ggdt_tuning* tuning, ggdt_plan** plan,
                      size_t* workspace_bytes);

/* Run every instance's forward (records written where non-NULL) in one
 * persistent launch on `stream`.  Performs no host synchronisation and no
 * allocation, so it can be captured into a HIP graph; the plan's device table is
 * uploaded by ggdt_batched_plan. */
int ggdt_batched_run(const ggdt_plan* plan, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Run every instance's backward in one persistent launch (all instances need
 * records, grad_out, grad_image and grad_softmask).  GGDT_ERR_UNSUPPORTED when
 * the plan holds no reverse tables: some instance lacks those buffers, or the
 * batch's channel count exceeds what one reverse workgroup's LDS holds (2D
 * images: C <= 2, volumes: C <= 3; the per-instance backward has no such limit
 * below C = 8). */
int ggdt_batched_backward(const ggdt_plan* plan, void* workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* Shape of a plan, for diagnostics and tuning reports (any pointer may be NULL):
 * instances, forward grid, backward grid (0 if the plan has no backward),
 * dynamic LDS bytes of the forward and backward launches. */
int ggdt_plan_info(const ggdt_plan* plan, int* n, int* grid, int* bwd_grid, size_t* lds, size_t* bwd_lds);

void ggdt_plan_destroy(ggdt_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* GGDT_H_ */
