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
#include "pass_device.h"
#include "toivanen.h"

namespace ggdt {

namespace {
using namespace dev;

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
        if (threadIdx.x == 0) {
          int ok = 1;
          if (has_dep && known < need) {
            unsigned long long polls = 0;
            for (;;) {
              known = __hip_atomic_load(prog + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (known >= need) break;
              if (ld_relaxed(words + kWordAbort) != 0u) {
                ok = 0;
                break;
              }
              if (++polls > limit) {
                __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
              }
              __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          }
          s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) return;
        for (int r = threadIdx.x; r < nrows; r += kToivThreads) {
          const int rz = r / nry;
          const int z = z0 + rz, y = y0 + (r - rz * nry);
          const int x = t - 4 * z - 2 * y;
          if (x >= 0 && x < W) toivanen_voxel<NOFF>(d, I, D, z, y, x, dir);
        }
        __syncthreads();
        if (threadIdx.x == 0 && (j + 1 - j_lo) % d.publish == 0 && j < j_hi) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(prog + b, need + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // the whole sweep (the hyperplanes after the block's last are no-ops)
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(prog + b, base + (unsigned long long)d.T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

}  // namespace

int toivanen_capacity() {
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)toivanen_kernel<13>, kToivThreads, 0) !=
        hipSuccess)
      return 0;
    cap = per_cu * cus;
  }
  return cap;
}

// Row blocks of about one row per thread (slabs of 1024 / H planes, bands of
// 1024 image rows), grown while there are more blocks than co-resident
// workgroups or progress words.  A block trails its neighbour by the steps
// between publications, and starts 4 bz (volume) or 2 by (image) hyperplanes
// after it: publishing every half of that keeps the pipeline at full speed.
bool toivanen_blocks(ToivDesc* d, int cap, long long words) {
  const int Z = d->dims[0], H = d->dims[1];
  const bool image = Z == 1;
  int bz = image ? 1 : (H >= kToivThreads ? 1 : kToivThreads / H);
  int by = image ? (H < kToivThreads ? H : kToivThreads) : H;
  for (;;) {
    const long long nb = image ? (H + by - 1) / by : (Z + bz - 1) / bz;
    if (nb <= cap && nb <= words) {
      const int lead = image ? 2 * by : 4 * bz;
      d->bz = bz;
      d->by = by;
      d->nb = (int)nb;
      d->publish = lead / 2 < 1 ? 1 : (lead / 2 > 16 ? 16 : lead / 2);
      return true;
    }
    if (image ? by >= H : bz >= Z) return false;
    if (image) by = by < H / 2 ? by * 2 : H;
    else bz = bz < Z / 2 ? bz * 2 : Z;
  }
}

hipError_t launch_toivanen(const ToivDesc& d, unsigned* words, unsigned long long spin_limit, hipStream_t stream) {
  const int grid = d.nb;
  if (grid <= 0) return hipErrorInvalidConfiguration;
  if (d.noff == 13)
    hipLaunchKernelGGL(toivanen_kernel<13>, dim3(grid), dim3(kToivThreads), 0, stream, d, words, spin_limit);
  else if (d.noff == 4)
    hipLaunchKernelGGL(toivanen_kernel<4>, dim3(grid), dim3(kToivThreads), 0, stream, d, words, spin_limit);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ggdt
