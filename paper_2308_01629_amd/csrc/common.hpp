// Shared device-side definitions of the upsampling library (gfx950).
//
// The whole library is compiled with -ffp-contract=off: every a*b+c below is
// two rounded operations unless it is written as an explicit fmaf.  The grid
// keys and the membership predicate depend on that (they are a bit-exact
// contract); the weights use explicit fmaf where it pays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/upsample.h"

namespace ups {

constexpr int kBlock = 256;            // threads per block for streaming kernels
constexpr int kScanItems = 8;          // cells per thread in the cell scan
constexpr int kScanChunk = kBlock * kScanItems;

// Grid and step constants passed by value to kernels (kernarg -> SGPRs).
struct GridConst {
  float lo[3];
  float inv_cs;
  int dims[3];
  float cs;       // fl32(cell size): bounds of cell boxes
  int reach;
  float h2;       // fl32(9 r^2): membership threshold
  float inv_h2;   // fl32(1 / (9 r^2)): weight scale
};

struct StepConst {
  float c1, c2, dt, r_hr;
  float g[3];
  int n_walls;
  int has_rigid;  // 0: every LR particle is granular (rigid rule is moot)
};

// Walls travel in the kernel arguments: 32 x 12 floats = 1.5 KB.
struct WallTable {
  float w[UPSAMPLE_MAX_WALLS * UPSAMPLE_WALL_FLOATS];
};

// One LR particle in sorted order: 32 bytes, two 16-byte loads.
//   p = (x, y, z, rigid ? 1 : 0), v = (vx, vy, vz, original index as bits)
struct __align__(16) LRPoint {
  float4 p;
  float4 v;
};

// Cell coordinate along one axis: clamp(floor(fl32(fl32(x - lo) * inv_cs)), 0, G-1).
__device__ __forceinline__ int cell_coord(float x, float lo, float inv_cs, int G) {
  float t = (x - lo) * inv_cs;              // two rounded ops (no contraction)
  float f = floorf(t);
  f = fminf(fmaxf(f, 0.0f), (float)(G - 1));
  return (int)f;
}

// Squared distance with each operation rounded separately.
__device__ __forceinline__ float sq_dist(float ax, float ay, float az, float bx, float by, float bz) {
  float dx = ax - bx, dy = ay - by, dz = az - bz;
  float sx = dx * dx, sy = dy * dy, sz = dz * dz;
  return (sx + sy) + sz;
}

}  // namespace ups
