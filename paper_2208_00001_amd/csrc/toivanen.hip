// Toivanen's raster scan on the GPU, by hyperplanes.
//
// The paper's software ships Toivanen's sequential raster scan as the
// single-thread comparison method (section "Implementation").  One iteration
// is a forward sweep over the voxels in raster order (every axis ascending)
// and a backward sweep in the reverse order; a voxel takes the minimum of its
// own value and D(y) + w(x, y) over the neighbours y of its 8 (2D) / 26 (3D)
// neighbourhood that precede it in the sweep, in place, so it sees the values
// lowered earlier in the same sweep.
//
// The preceding neighbours of (z, y, x) in the forward order are the offsets
// whose first non-zero component is negative: (-1, *, *), (0, -1, *) and
// (0, 0, -1).  On the hyperplane t = 4z + 2y + x each of them lies at a
// smaller t (by 4 - 2|dy| - |dx| >= 1, 2 - |dx| >= 1 or 1), so every voxel of
// one hyperplane depends only on earlier hyperplanes: sweeping the hyperplanes
// in order and the voxels of one hyperplane in parallel gives exactly the
// values of the sequential sweep (the backward sweep takes the hyperplanes in
// reverse).  A 2D image is the volume with one plane.
//
// Each workgroup owns a block of rows (z, y), all x, and steps through the
// hyperplanes; hyperplane t meets row (z, y) at x = t - 4z - 2y.  A volume is
// cut into slabs of whole planes (all rows y), an image into bands of rows:
// either way the rows a block reads outside its own lie in the block just
// before it (forward sweep) or just after it (backward sweep), at hyperplanes
// up to t - 1, so a block waits for that one neighbour's progress, never for
// the whole grid, and the blocks run as a pipeline.  (Blocks cut along y as
// well would read each other both ways through the offsets (-1, +1, *) and
// (0, -1, *), a cycle.)  Progress is the number of steps (hyperplanes) a block
// has completed since the launch, published every few steps and at the end of
// each sweep (release at agent scope by one thread, after a workgroup
// barrier); a block that needs more than it has seen polls and acquires.  A
// block skips the hyperplanes that miss all its rows.  The same waits order
// the sweeps: a block's first step of a sweep needs its neighbour to have
// finished the previous sweep, and that neighbour is the one block that read
// this block's rows during it.  The dependencies are acyclic (lower blocks
// first in a forward sweep, upper blocks first in a backward one), so with
// every block resident the pipeline always advances; the waits are bounded
// like every other.
//
// Two forms share this plan: the ring form keeps the recent steps of a
// block's rows in LDS (one row per thread, up to 3 channels); the general form
// reads every candidate from global memory and serves the rest (more channels,
// blocks whose rings would not fit).
#include "ggdt.h"
#include "pass_device.h"
#include "toivanen.h"

namespace ggdt {

namespace {
using namespace dev;

// Thread 0: wait until the neighbour block `dep` has completed `need` steps
// (polls its progress word; `known` keeps the last count seen), then acquire.
// Bounded like every wait; false if it gave up or another wait did.
__device__ __forceinline__ bool wait_progress(unsigned long long* prog, int dep, unsigned long long need,
                                              unsigned long long& known, unsigned* words,
                                              unsigned long long limit) {
  if (known >= need) return true;
  unsigned long long polls = 0;
  for (;;) {
    known = __hip_atomic_load(prog + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (known >= need) break;
    if (ld_relaxed(words + kWordAbort) != 0u) return false;
    if (++polls > limit) {
      __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Thread 0, after a workgroup barrier that drained every wave's stores:
// publish the block's completed steps.
__device__ __forceinline__ void publish_progress(unsigned long long* prog, int b, unsigned long long steps) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(prog + b, steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One voxel's update in a sweep (dir +1 forward, -1 backward): its value
// and those of its preceding neighbours are all loaded before the arithmetic,
// so a step costs one memory round trip per channel rather than one per
// neighbour; the candidates are then taken in the offsets' order with a
// strict <.
template <int NOFF>
__device__ __forceinline__ void toivanen_voxel(const ToivDesc& d, const gmem<const float>& I, const gmem<float>& D,
                                               int z, int y, int x, int dir) {
  const int Z = d.dims[0], H = d.dims[1], W = d.dims[2];
  const long long i = ((long long)z * H + y) * W + x;
  long long yi[NOFF];
  bool ok[NOFF];
#pragma unroll
  for (int k = 0; k < NOFF; ++k) {
    const int zz = z + dir * d.off[k][0], yy = y + dir * d.off[k][1], xx = x + dir * d.off[k][2];
    ok[k] = zz >= 0 && zz < Z && yy >= 0 && yy < H && xx >= 0 && xx < W;
    yi[k] = ok[k] ? ((long long)zz * H + yy) * W + xx : i;  // an absent neighbour reads the voxel itself
  }
  float dv[NOFF], g[NOFF];
  const float di = D[i];
#pragma unroll
  for (int k = 0; k < NOFF; ++k) dv[k] = D[yi[k]];
  {
    const float ii = I[i];
    float iv[NOFF];
#pragma unroll
    for (int k = 0; k < NOFF; ++k) iv[k] = I[yi[k]];
#pragma unroll
    for (int k = 0; k < NOFF; ++k) {
      const float d0 = ii - iv[k];
      g[k] = d0 * d0;
    }
  }
  for (int c = 1; c < d.C; ++c) {
    const long long o = (long long)c * d.N;
    const float ii = I[o + i];
    float iv[NOFF];
#pragma unroll
    for (int k = 0; k < NOFF; ++k) iv[k] = I[o + yi[k]];
#pragma unroll
    for (int k = 0; k < NOFF; ++k) {
      const float dc = ii - iv[k];
      g[k] = fmaf(dc, dc, g[k]);
    }
  }
  float best = di;
#pragma unroll
  for (int k = 0; k < NOFF; ++k) {
    const float cand = dv[k] + sqrtf(fmaf(d.lam, g[k], d.A[k]));
    if (ok[k] && cand < best) best = cand;
  }
  D[i] = best;
}

// General form: 1024 threads, rows strided over them, every candidate read
// from global memory; a workgroup barrier between steps.
template <int NOFF>
__global__ __launch_bounds__(kToivThreads) void toivanen_kernel(ToivDesc d, unsigned* words,
                                                                unsigned long long limit) {
  __shared__ int s_ok;
  const gmem<const float> I = to_gmem(d.image);
  const gmem<float> D = to_gmem(d.D);
  const int Z = d.dims[0], H = d.dims[1], W = d.dims[2];
  const int b = blockIdx.x;
  const bool image = Z == 1;
  const int z0 = image ? 0 : b * d.bz, z1 = image ? 1 : min(Z, z0 + d.bz);  // volume slab
  const int y0 = image ? b * d.by : 0, y1 = image ? min(H, y0 + d.by) : H;  // image band
  const int nry = y1 - y0, nrows = (z1 - z0) * nry;
  // hyperplanes meeting the block's rows
  const int t_lo = 4 * z0 + 2 * y0, t_hi = 4 * (z1 - 1) + 2 * (y1 - 1) + (W - 1);
  // progress words (steps completed since the launch) of every block, after the header
  unsigned long long* prog = reinterpret_cast<unsigned long long*>(words + kHeaderWords);
  for (int it = 0; it < d.iterations; ++it) {
    for (int sweep = 0; sweep < 2; ++sweep) {
      const int dir = sweep == 0 ? 1 : -1;
      const unsigned long long base = (unsigned long long)(2 * it + sweep) * (unsigned long long)d.T;
      const int dep = b - dir;  // the block whose rows this one reads in this sweep
      const bool has_dep = dep >= 0 && dep < d.nb;
      const int j_lo = dir > 0 ? t_lo : d.T - 1 - t_hi, j_hi = dir > 0 ? t_hi : d.T - 1 - t_lo;
      unsigned long long known = 0;  // progress seen of the neighbour (thread 0)
      for (int j = j_lo; j <= j_hi; ++j) {
        const int t = dir > 0 ? j : d.T - 1 - j;
        // the neighbour must have completed every step before this one
        const unsigned long long need = base + (unsigned long long)j;
        if (threadIdx.x == 0) s_ok = !has_dep || wait_progress(prog, dep, need, known, words, limit);
        __syncthreads();
        if (!s_ok) return;
        for (int r = threadIdx.x; r < nrows; r += kToivThreads) {
          const int rz = r / nry;
          const int z = z0 + rz, y = y0 + (r - rz * nry);
          const int x = t - 4 * z - 2 * y;
          if (x >= 0 && x < W) toivanen_voxel<NOFF>(d, I, D, z, y, x, dir);
        }
        __syncthreads();
        if (threadIdx.x == 0 && (j + 1 - j_lo) % d.publish == 0 && j < j_hi) publish_progress(prog, b, need + 1ull);
      }
      // the whole sweep (the hyperplanes after the block's last are no-ops)
      __syncthreads();
      if (threadIdx.x == 0) publish_progress(prog, b, base + (unsigned long long)d.T);
    }
  }
}

// Ring form (one row per thread, at most 3 channels).  A block keeps the
// last S steps of its rows' values of D and of the image in LDS rings (slot =
// step mod S; a preceding neighbour lies at most 7 steps back in a volume, 3
// in an image), and the neighbour block's rows it reads, its ghost rows, in
// rings of their own.  A voxel's candidates then come from LDS; the only
// global accesses of a step are loads issued one step ahead (the row's own D
// from the previous sweep and its image value, and one ghost voxel per ghost
// row) and the store of the result.  Steps meet at an LDS barrier; every
// `publish` steps a full workgroup barrier drains the stores before the
// progress is published.  Thread 0 waits, at the end of each step, for the
// neighbour's progress that the next step's ghost load needs.  The offsets and
// the sweep direction are compile-time constants, so a candidate costs its
// two LDS reads and its arithmetic; the ring slot of an offset is the same
// for every thread.

// The preceding neighbours in the forward raster order, in the order the
// host's edge constants A_j follow: (-1, *, *), (0, -1, *), (0, 0, -1).
__device__ constexpr int kRingOff3[13][3] = {{-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0},
                                            {-1, 0, 1},   {-1, 1, -1},  {-1, 1, 0},  {-1, 1, 1},  {0, -1, -1},
                                            {0, -1, 0},   {0, -1, 1},   {0, 0, -1}};
__device__ constexpr int kRingOff2[4][3] = {{0, -1, -1}, {0, -1, 0}, {0, -1, 1}, {0, 0, -1}};

template <int NOFF>
__device__ constexpr int ring_off(int k, int a) {
  return NOFF == 13 ? kRingOff3[k][a] : kRingOff2[k][a];
}

// The part of a block's state the sweeps share.
struct RingBlock {
  int b, r, z0, z1, y0, y1, nry, t_lo, t_hi, z, y, t0;
  bool has_row;
  long long row0;
};

// One sweep (DIR +1 forward, -1 backward) of a block; false if a wait gave up.
template <int NOFF, int C, int NT, int DIR, int MODE>
__device__ __forceinline__ bool ring_sweep(const ToivDesc& d, const RingBlock& k0, float* lds, int* s_ok,
                                           unsigned* words, unsigned long long limit, unsigned long long base) {
  constexpr int S = NOFF == 13 ? 8 : 4;
  constexpr int R = NT;
  // offsets 0..KG-1 leave the block through its boundary face (dz != 0 in a
  // volume slab, dy != 0 in an image band); the others stay inside
  constexpr int KG = NOFF == 13 ? 9 : 3;
  // Ring rows of R1 = R + 1 (ghost: G1 = G + 1) columns: column r holds row r
  // of the block, the last column +inf, read in place of a neighbour outside
  // the domain.  A row idle at a step writes +inf into its slot, the rings
  // start every sweep at +inf, and the ghost loader writes +inf where the
  // ghost voxel does not exist: a missing neighbour's candidate is then +inf
  // (or NaN) and never passes the strict <, as if it were skipped.
  constexpr int R1 = R + 1;
  const int G = d.ng, G1 = G + 1;
  const float inf = __builtin_inff();
  float* rD = lds;               // [S][R1]    D of the block's rows
  float* rI = rD + S * R1;       // [C][S][R1] their image values
  float* gD = rI + C * S * R1;   // [S][G1]    D of the ghost rows
  float* gI = gD + S * G1;       // [C][S][G1]
  const int gbase = (1 + C) * S * R1;  // gD's offset in the LDS
  const gmem<const float> I = to_gmem(d.image);
  const gmem<float> D = to_gmem(d.D);
  const gmem<float> sink = to_gmem(reinterpret_cast<float*>(words + kWordSink));
  unsigned long long* prog = reinterpret_cast<unsigned long long*>(words + kHeaderWords);
  const int Z = d.dims[0], H = d.dims[1], W = d.dims[2], T = d.T;
  const long long N = d.N;
  const bool image = Z == 1;
  const int b = k0.b, r = k0.r, z = k0.z, y = k0.y, t0 = k0.t0;
  const bool has_row = k0.has_row;
  const long long row0 = k0.row0;
  const unsigned long long end = base + (unsigned long long)T;
  const int dep = b - DIR;
  const bool has_dep = dep >= 0 && dep < d.nb;
  const int u_lo = DIR > 0 ? k0.t_lo : T - 1 - k0.t_hi, u_hi = DIR > 0 ? k0.t_hi : T - 1 - k0.t_lo;
  // ghost rows: the plane before (forward) or after (backward) the slab, row
  // y' loaded by thread y'; the row before or after an image band, loaded by
  // thread 0
  const int zg = image ? 0 : (DIR > 0 ? k0.z0 - 1 : k0.z1);
  const int yg = image ? (DIR > 0 ? k0.y0 - 1 : k0.y1) : r;
  const bool loader = has_dep && (image ? r == 0 : r < H);
  const int gcol = image ? 0 : r;
  const long long grow0 = ((long long)zg * H + yg) * W;
  const int tg0 = 4 * zg + 2 * yg;
  // whether this row's boundary-face offsets reach the ghost rows, and each
  // candidate's column (ring offset at slot 0) and ring stride
  const bool edge = image ? (y == (DIR > 0 ? k0.y0 : k0.y1 - 1)) : (z == (DIR > 0 ? k0.z0 : k0.z1 - 1));
  const int estride = edge ? G1 : R1;  // stride of the offsets 0..KG-1
  int col[NOFF];
#pragma unroll
  for (int k = 0; k < NOFF; ++k) {
    const int dz = DIR * ring_off<NOFF>(k, 0), dy = DIR * ring_off<NOFF>(k, 1);
    const int zz = z + dz, yy = y + dy;
    const bool there = has_row && zz >= 0 && zz < Z && yy >= 0 && yy < H;
    if (k < KG && edge)
      col[k] = gbase + (there ? (image ? 0 : yy) : G);
    else
      col[k] = there ? r + dz * k0.nry + dy : R;
  }
  unsigned long long known = 0;
  // the neighbour's steps up to u_lo + 1: the ghosts of the first step and the first ghost load
  if (r == 0) {
    const unsigned long long need = base + (unsigned long long)(u_lo + 2);
    s_ok[0] = !has_dep || wait_progress(prog, dep, need < end ? need : end, known, words, limit);
  }
  // the rings' D at +inf (the last columns stay so)
  for (int i = r; i < S * R1; i += NT) rD[i] = inf;
  for (int i = r; i < S * G1; i += NT) gD[i] = inf;
  __syncthreads();
  if (!s_ok[0]) return false;
  float pD = 0.0f, pI[C];  // the loader's ghost voxel of the current step
  int px = -1;
#pragma unroll
  for (int c = 0; c < C; ++c) pI[c] = 0.0f;
  if (loader) {
#pragma unroll 1
    for (int q = 1 - S; q <= 0; ++q) {
      const int ug = u_lo + q;
      const int xg = (DIR > 0 ? ug : T - 1 - ug) - tg0;
      if (ug < 0 || xg < 0 || xg >= W) continue;
      const float vD = D[grow0 + xg];
      float vI[C];
#pragma unroll
      for (int c = 0; c < C; ++c) vI[c] = I[c * N + grow0 + xg];
      if (q == 0) {
        pD = vD;
#pragma unroll
        for (int c = 0; c < C; ++c) pI[c] = vI[c];
        px = xg;
      } else {
        const int slot = ug & (S - 1);
        gD[slot * G1 + gcol] = vD;
#pragma unroll
        for (int c = 0; c < C; ++c) gI[(c * S + slot) * G1 + gcol] = vI[c];
      }
    }
  }
  float cD = 0.0f, cI[C];  // the row's own D (previous sweep) and image at the current step
#pragma unroll
  for (int c = 0; c < C; ++c) cI[c] = 0.0f;
  {
    const int x = (DIR > 0 ? u_lo : T - 1 - u_lo) - t0;
    if (has_row && x >= 0 && x < W) {
      cD = D[row0 + x];
#pragma unroll
      for (int c = 0; c < C; ++c) cI[c] = I[c * N + row0 + x];
    }
  }
  // complete the loads above, so that a step's wait for its operands counts
  // only the memory operations of the step before
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll 1
  for (int u = u_lo; u <= u_hi; ++u) {
    const int t = DIR > 0 ? u : T - 1 - u;
    const bool more = u < u_hi;
    // the ghost voxel of this step into its slot (loaded a step ago), +inf
    // where there is none
    if (loader) {
      const int slot = u & (S - 1);
      gD[slot * G1 + gcol] = px >= 0 ? pD : inf;
#pragma unroll
      for (int c = 0; c < C; ++c) gI[(c * S + slot) * G1 + gcol] = pI[c];
    }
    // the next step's loads, issued by every thread at a clamped index
    // (their values unused where the voxel does not exist), so that no wait
    // before this step's arithmetic has to include them
    const int xn = t + DIR - t0, xg = t + DIR - tg0;
    const long long on = row0 + min(max(xn, 0), W - 1);
    const long long gn = (loader ? grow0 : row0) + min(max(xg, 0), W - 1);
    const float nD = D[on], qD = D[gn];
    float nI[C], qI[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      nI[c] = I[c * N + on];
      qI[c] = I[c * N + gn];
    }
    const int x = t - t0;
    const bool active = has_row && x >= 0 && x < W;
    float best = cD;
#pragma unroll
    for (int k = 0; k < NOFF; ++k) {
      // steps back to the neighbour's hyperplane, and its ring slot (uniform)
      const int a = -(4 * ring_off<NOFF>(k, 0) + 2 * ring_off<NOFF>(k, 1) + ring_off<NOFF>(k, 2));
      const int slot = (u - a) & (S - 1);
      const int stride = k < KG ? estride : R1;
      const int cs = S * stride;  // from D to the image values, and between channels
      const int offD = col[k] + slot * stride;
      const int offI = offD + cs;
      const float dv = lds[offD];
      const float d0 = cI[0] - lds[offI];
      float w;
      if (MODE == kModeLam1C1) {
        w = fabsf(d0);  // = sqrtf(fl(d0 * d0)) for the classified image (no tiny or huge values)
      } else {
        float g = d0 * d0;
#pragma unroll
        for (int c = 1; c < C; ++c) {
          const float dc = cI[c] - lds[offI + c * cs];
          g = fmaf(dc, dc, g);
        }
        w = general_root<MODE>(fmaf(d.lam, g, d.A[k]));
      }
      const float cand = dv + w;
      if (cand < best) best = cand;
    }
    {
      const int slot = u & (S - 1);
      rD[slot * R1 + r] = active ? best : inf;
#pragma unroll
      for (int c = 0; c < C; ++c) rI[(c * S + slot) * R1 + r] = cI[c];
    }
    // the result, stored by every thread (idle ones to the sink word)
    *(active ? &D[row0 + x] : sink) = best;
    cD = nD;
    pD = qD;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cI[c] = nI[c];
      pI[c] = qI[c];
    }
    px = loader && more && xg >= 0 && xg < W ? xg : -1;
    // the neighbour's progress the next step's ghost load needs
    if (r == 0) {
      const unsigned long long need = base + (unsigned long long)(u + 3);
      s_ok[u & 1] = !(has_dep && more) || wait_progress(prog, dep, need < end ? need : end, known, words, limit);
    }
    if ((u + 1 - u_lo) % d.publish == 0 && more) {
      __syncthreads();
      if (r == 0) publish_progress(prog, b, base + (unsigned long long)(u + 1));
    } else {
      lds_barrier();
    }
    if (!s_ok[u & 1]) return false;
  }
  __syncthreads();
  if (r == 0) publish_progress(prog, b, end);
  return true;
}

// The sweeps of one edge-cost form.
template <int NOFF, int C, int NT, int MODE>
__device__ __forceinline__ void ring_iterations(const ToivDesc& d, const RingBlock& k0, float* lds, int* s_ok,
                                                unsigned* words, unsigned long long limit) {
  for (int it = 0; it < d.iterations; ++it) {
    const unsigned long long base = (unsigned long long)(2 * it) * (unsigned long long)d.T;
    if (!ring_sweep<NOFF, C, NT, 1, MODE>(d, k0, lds, s_ok, words, limit, base)) return;
    if (!ring_sweep<NOFF, C, NT, -1, MODE>(d, k0, lds, s_ok, words, limit, base + (unsigned long long)d.T)) return;
  }
}

// RMODE: the form the host requested (kModeLam1C1 or kModeGeneral); the image
// classification decides on the device whether its fast form applies, as for
// the passes.
template <int NOFF, int C, int NT, int RMODE>
__global__ __launch_bounds__(NT) void toivanen_ring_kernel(ToivDesc d, unsigned* words, unsigned long long limit) {
  extern __shared__ __align__(16) float lds[];
  __shared__ int s_ok[2];
  const int Z = d.dims[0], H = d.dims[1], W = d.dims[2];
  const bool image = Z == 1;
  RingBlock k0;
  k0.b = blockIdx.x;
  k0.r = threadIdx.x;
  k0.z0 = image ? 0 : k0.b * d.bz;  // volume slab
  k0.z1 = image ? 1 : min(Z, k0.z0 + d.bz);
  k0.y0 = image ? k0.b * d.by : 0;  // image band
  k0.y1 = image ? min(H, k0.y0 + d.by) : H;
  k0.nry = k0.y1 - k0.y0;
  const int nrows = (k0.z1 - k0.z0) * k0.nry;
  k0.t_lo = 4 * k0.z0 + 2 * k0.y0;
  k0.t_hi = 4 * (k0.z1 - 1) + 2 * (k0.y1 - 1) + (W - 1);
  k0.has_row = k0.r < nrows;
  const int rz = k0.has_row ? k0.r / k0.nry : 0;
  k0.z = k0.z0 + rz;
  k0.y = k0.y0 + (k0.has_row ? k0.r - rz * k0.nry : 0);
  k0.row0 = ((long long)k0.z * H + k0.y) * W;  // voxel index of x = 0
  k0.t0 = 4 * k0.z + 2 * k0.y;                 // its hyperplane
  const unsigned cls = ld_relaxed(words + kWordClass);
  if (RMODE == kModeLam1C1 && fast_mode_ok(kModeLam1C1, cls))
    ring_iterations<NOFF, C, NT, kModeLam1C1>(d, k0, lds, s_ok, words, limit);
  else if (RMODE == kModeGeneral && general_n_ok(d.sqrt_normal, words + kWordClass))
    ring_iterations<NOFF, C, NT, kModeGeneralN>(d, k0, lds, s_ok, words, limit);
  else
    ring_iterations<NOFF, C, NT, kModeGeneral>(d, k0, lds, s_ok, words, limit);
}

}  // namespace

namespace {

template <int NOFF, int NT>
const void* ring_fn_c(int C, int mode) {
  if (mode == kModeLam1C1) return C == 1 ? (const void*)toivanen_ring_kernel<NOFF, 1, NT, kModeLam1C1> : nullptr;
  if (C == 1) return (const void*)toivanen_ring_kernel<NOFF, 1, NT, kModeGeneral>;
  if (C == 2) return (const void*)toivanen_ring_kernel<NOFF, 2, NT, kModeGeneral>;
  if (C == 3) return (const void*)toivanen_ring_kernel<NOFF, 3, NT, kModeGeneral>;
  return nullptr;
}

// The block sizes the plan picks: image bands of up to 256 rows; volume slabs
// of up to 512 rows, or one plane of up to 1024.
const void* ring_fn(int noff, int C, int nt, int mode) {
  if (noff == 4 && nt == 256) return ring_fn_c<4, 256>(C, mode);
  if (noff == 13 && nt == 512) return ring_fn_c<13, 512>(C, mode);
  if (noff == 13 && nt == 1024) return ring_fn_c<13, 1024>(C, mode);
  return nullptr;
}

const void* general_fn(int noff) {
  if (noff == 13) return (const void*)toivanen_kernel<13>;
  if (noff == 4) return (const void*)toivanen_kernel<4>;
  return nullptr;
}

// Co-resident workgroups of a kernel with `lds` bytes of dynamic LDS (0 on error).
int capacity(const void* fn, int threads, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (lds > 0 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

// Dynamic LDS of the ring form: rings of S steps of D and C image channels for
// the block's rows (one per thread) and its ghost rows.
size_t ring_lds(const ToivDesc& d) {
  const size_t S = d.noff == 13 ? 8 : 4;
  return (size_t)(1 + d.C) * S * (size_t)(d.threads + 1 + d.ng + 1) * sizeof(float);
}

}  // namespace

// The ring form takes blocks of a few hundred rows, one per thread (bands of
// kToivRowsImage image rows, slabs of kToivRowsVolume / H planes; a volume with
// more rows per plane takes slabs of one plane, up to 1024 rows), when they fit: at
// most 3 channels, the rings within the LDS, every block co-resident.  Smaller
// blocks spread a hyperplane's voxels over more compute units; a block trails
// its neighbour by a few steps (the ghost load a step ahead, the publication
// period), and starts 4 bz (volume) or 2 by (image) hyperplanes after it:
// publishing every half of that keeps the pipeline near full speed.
// Otherwise the general form, 1024 threads per block, with blocks grown while
// there are more of them than co-resident workgroups.
int toivanen_plan(ToivDesc* d, long long words) {
  const int Z = d->dims[0], H = d->dims[1];
  const bool image = Z == 1;
  d->ng = image ? 1 : H;
  d->ring = 0;
  auto set_blocks = [&](int bz, int by) {
    const long long nb = image ? (H + by - 1) / by : (Z + bz - 1) / bz;
    const int lead = image ? 2 * by : 4 * bz;
    d->bz = bz;
    d->by = by;
    d->nb = (int)(nb < 0x7fffffffLL ? nb : 0x7fffffffLL);
    d->publish = lead / 2 < 1 ? 1 : (lead / 2 > 16 ? 16 : lead / 2);
    return nb;
  };
  {
    const int bz = image ? 1 : (H >= kToivRowsVolume ? 1 : kToivRowsVolume / H);
    const int by = image ? (H < kToivRowsImage ? H : kToivRowsImage) : H;
    const long long rows = image ? by : (long long)bz * H;
    const int nt = image ? 256 : (rows <= 512 ? 512 : 1024);
    const long long nb = set_blocks(bz, by);
    d->threads = nt;
    const void* fn = ring_fn(d->noff, d->C, nt, d->mode);
    const size_t lds = ring_lds(*d);
    if (fn && rows <= 1024 && lds <= 160 * 1024 && nb <= words) {
      const int cap = capacity(fn, nt, lds);
      if (cap <= 0) return GGDT_ERR_HIP;
      if (nb <= cap) {
        d->ring = 1;
        d->lds = lds;
        return GGDT_OK;
      }
    }
  }
  d->threads = kToivThreads;
  d->lds = 0;
  const int cap = capacity(general_fn(d->noff), kToivThreads, 0);
  if (cap <= 0) return GGDT_ERR_HIP;
  int bz = image ? 1 : (H >= kToivThreads ? 1 : kToivThreads / H);
  int by = image ? (H < kToivThreads ? H : kToivThreads) : H;
  for (;;) {
    const long long nb = set_blocks(bz, by);
    if (nb <= cap && nb <= words) return GGDT_OK;
    if (image ? by >= H : bz >= Z) return GGDT_ERR_UNSUPPORTED;
    if (image) by = by < H / 2 ? by * 2 : H;
    else bz = bz < Z / 2 ? bz * 2 : Z;
  }
}

hipError_t launch_toivanen(const ToivDesc& d, unsigned* words, unsigned long long spin_limit, hipStream_t stream) {
  const int grid = d.nb;
  if (grid <= 0) return hipErrorInvalidConfiguration;
  const void* fn = d.ring ? ring_fn(d.noff, d.C, d.threads, d.mode) : general_fn(d.noff);
  if (!fn) return hipErrorInvalidValue;
  void* args[] = {(void*)&d, (void*)&words, (void*)&spin_limit};
  return hipLaunchKernel(fn, dim3(grid), dim3(d.threads), args, d.lds, stream);
}

}  // namespace ggdt
