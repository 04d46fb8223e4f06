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
// reverse).  A 2D image is the volume with one plane.  The voxels of one
// hyperplane are spread over the threads of a persistent grid, and the
// hyperplanes are separated by a grid barrier (a workgroup barrier when the
// grid is one workgroup).
#include "grid_sync.h"
#include "toivanen.h"

namespace ggdt {

namespace {
using namespace dev;

__global__ __launch_bounds__(kToivThreads) void toivanen_kernel(ToivDesc d, unsigned* words,
                                                                unsigned long long limit) {
  const gmem<const float> I = to_gmem(d.image);
  const gmem<float> D = to_gmem(d.D);
  const int Z = d.dims[0], H = d.dims[1], W = d.dims[2];
  const long long P = (long long)Z * H;  // rows (z, y); hyperplane t meets row (z, y) at x = t - 4z - 2y
  const long long nthr = (long long)gridDim.x * blockDim.x;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(words + kWordToivCounter);
  unsigned long long target = 0;
  for (int it = 0; it < d.iterations; ++it) {
    for (int sweep = 0; sweep < 2; ++sweep) {
      const int dir = sweep == 0 ? 1 : -1;
      for (int s = 0; s < d.T; ++s) {
        const int t = dir > 0 ? s : d.T - 1 - s;
        for (long long k = gid; k < P; k += nthr) {
          const int z = (int)(k / H), y = (int)(k - (long long)z * H);
          const int x = t - 4 * z - 2 * y;
          if (x < 0 || x >= W) continue;
          const long long i = ((long long)z * H + y) * W + x;
          float best = D[i];
          for (int j = 0; j < d.noff; ++j) {
            const int zz = z + dir * d.off[j][0], yy = y + dir * d.off[j][1], xx = x + dir * d.off[j][2];
            if (zz < 0 || zz >= Z || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const long long yi = ((long long)zz * H + yy) * W + xx;
            const float d0 = I[i] - I[yi];
            float g = d0 * d0;
            for (int c = 1; c < d.C; ++c) {
              const float dc = I[(long long)c * d.N + i] - I[(long long)c * d.N + yi];
              g = fmaf(dc, dc, g);
            }
            const float cand = D[yi] + sqrtf(fmaf(d.lam, g, d.A[j]));
            if (cand < best) best = cand;
          }
          D[i] = best;
        }
        if (gridDim.x == 1) {
          __syncthreads();
        } else {
          target += gridDim.x;
          if (!counter_barrier<unsigned long long>(ctr, target, words, limit)) return;
        }
      }
    }
  }
}

}  // namespace

int toivanen_grid(const ToivDesc& d) {
  const long long rows = (long long)d.dims[0] * d.dims[1];
  // A row holds at most one voxel of a hyperplane: up to 4 rows per thread in
  // one workgroup (no grid barrier), else about two rows per thread (on the
  // 256^3 volume: 32 workgroups, 44 ms per iteration, against 49 ms with one
  // row per thread and 70 ms with four).
  if (rows <= 4LL * kToivThreads) return 1;
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)toivanen_kernel, kToivThreads, 0) !=
        hipSuccess)
      return 0;
    cap = per_cu * cus;
  }
  long long g = (rows + 2LL * kToivThreads - 1) / (2LL * kToivThreads);
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_toivanen(const ToivDesc& d, unsigned* words, unsigned long long spin_limit, hipStream_t stream) {
  const int grid = toivanen_grid(d);
  if (grid <= 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(toivanen_kernel, dim3(grid), dim3(kToivThreads), 0, stream, d, words, spin_limit);
  return hipGetLastError();
}

}  // namespace ggdt
