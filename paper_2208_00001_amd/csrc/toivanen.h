// Toivanen's raster scan by hyperplanes t = 4z + 2y + x (toivanen.hip); a 2D
// image is a volume of one plane (dims = {1, H, W}).
#pragma once

#include "ggdt_internal.h"

namespace ggdt {

constexpr int kToivThreads = 1024;  // threads per workgroup of the general form
constexpr int kToivRowsImage = 256;   // rows per block of the ring form (one per thread): image bands
constexpr int kToivRowsVolume = 512;  // volume slabs

struct ToivDesc {
  const float* image;  // (C, N)
  float* D;            // (N), holds v * M on entry
  long long N;
  int C;
  int dims[3];
  float lam;
  float A[13];     // (float)((1 - lambda) * |off_j|_s^2), the spatial term in double
  int off[13][3];  // offsets (dz, dy, dx) of the neighbours preceding a voxel in the forward sweep
  int noff;        // 4 (2D) or 13 (3D)
  int iterations;
  int T;           // hyperplanes per sweep: 4 (Z - 1) + 2 (H - 1) + (W - 1) + 1
  // Row blocks, one workgroup each: slabs of `bz` planes (all rows y) of a
  // volume, or bands of `by` rows of an image (Z = 1, bz = 1); `nb` blocks.
  int bz, by, nb;
  int publish;  // steps between progress publications
  int ng;       // ghost rows: the rows of the neighbouring block a block reads (H, image: 1)
  int mode;         // kModeLam1C1 (lambda 1, one channel) or kModeGeneral, as the passes request
  int sqrt_normal;  // kSqrtNormal*: when the general root may take its normal-range form
  int ring;     // 1: the LDS-ring form, 0: the general form
  int threads;  // threads per workgroup
  size_t lds;   // dynamic LDS bytes of the launch
};

// Pick the form and row blocks of a problem (one workgroup each, all
// co-resident, at most `words` progress words): GGDT_OK, GGDT_ERR_UNSUPPORTED
// if none fits, GGDT_ERR_HIP if the device cannot be queried.
int toivanen_plan(ToivDesc* d, long long words);
hipError_t launch_toivanen(const ToivDesc& d, unsigned* words, unsigned long long spin_limit, hipStream_t stream);

}  // namespace ggdt
