// The upsampling step proper (Section 4): per HR particle, a walk over the
// (2R+1)^3 cell stencil of the LR grid accumulating the kernel-weighted sums,
// then the blend parameter, the gravity blend, symplectic Euler and the walls,
// all in one kernel so each HR particle is read once and written once.
//
// HR state is structure-of-arrays float32 [3][n]: lanes of a wave read and
// write consecutive floats (six fully coalesced 256-byte accesses per wave
// each way).  Along x the cells of one (y, z) row of the stencil are adjacent
// keys, so each row is one contiguous range of the sorted LR copy.
#include <type_traits>

#include "kernels.hpp"
#include "tile.hpp"

namespace ups {
namespace {

struct Sums {
  float S, Ux, Uy, Uz, M;
  bool gran;
  uint32_t count;
  uint32_t arg;  // TAPE: original index of the largest weight (ties: smallest index)
  uint32_t count_w;  // DEBUG: candidates whose computed weight is > 0
  float wdis;        // DEBUG: largest weight where that test and membership disagree
};

// Weight of squared distance s in the direct form, each operation rounded
// separately: the debug exports' reference for entries on which the kernel's
// weight test and the exact membership predicate disagree.
__device__ __forceinline__ float direct_weight(float s, float inv_h2) {
  const float t = fmaxf(1.0f - s * inv_h2, 0.0f);
  return (t * t) * t;
}

// Walk the stencil of HR position (x, y, z) and accumulate the weighted sums
// over candidates of positive weight.  The float32 membership predicate
// s < h2 decides the rigid rule; DEBUG also records the member ids.
// RIGID: the scene has rigid LR particles, so their contributions are dropped
// when no granular LR particle is in the support.
template <bool DEBUG, bool RIGID, bool TAPE = false>
__device__ __forceinline__ Sums gather(const GridConst& gc, const LRPoint* __restrict__ lr,
                                       const uint32_t* __restrict__ cell_start, float x, float y,
                                       float z, uint32_t* ids, int64_t max_k) {
  Sums r{0.f, 0.f, 0.f, 0.f, 0.f, false, 0u, 0xffffffffu, 0u, 0.f};
  const int R = gc.reach;
  const int cx = cell_coord(x, gc.lo[0], gc.inv_cs, gc.dims[0]);
  const int cy = cell_coord(y, gc.lo[1], gc.inv_cs, gc.dims[1]);
  const int cz = cell_coord(z, gc.lo[2], gc.inv_cs, gc.dims[2]);
  const int x0 = max(cx - R, 0), x1 = min(cx + R, gc.dims[0] - 1);
  const int y0 = max(cy - R, 0), y1 = min(cy + R, gc.dims[1] - 1);
  const int z0 = max(cz - R, 0), z1 = min(cz + R, gc.dims[2] - 1);
  for (int zz = z0; zz <= z1; ++zz) {
    for (int yy = y0; yy <= y1; ++yy) {
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      const uint32_t b = cell_start[row + (uint32_t)x0];
      const uint32_t e = cell_start[row + (uint32_t)x1 + 1u];
      for (uint32_t j = b; j < e; ++j) {
        const float4 P = lr[j].p;
        // the candidate order and zero test of the wave-tiled path and its
        // direct-form weight arithmetic (bit-identical to the tiled path for
        // waves wider than 2h and for rigid scenes; the dot-product form of
        // compact waves differs by rounding)
        const float dx = P.x - x, dy = P.y - y, dz = P.z - z;
        const float sq = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float t = fmaxf(fmaf(-sq, gc.inv_h2, 1.0f), 0.0f);
        const float w = t * t * t;
        if (DEBUG) r.count_w += w > 0.0f ? 1u : 0u;
        if (t > 0.0f) {
          const float4 V = lr[j].v;
          r.S += w;
          r.Ux = fmaf(w, V.x, r.Ux);
          r.Uy = fmaf(w, V.y, r.Uy);
          r.Uz = fmaf(w, V.z, r.Uz);
          if (TAPE) {
            const uint32_t id = __float_as_uint(V.w);
            if (w > r.M || (w == r.M && id < r.arg)) r.arg = id;
          }
          r.M = fmaxf(r.M, w);
        }
        // support membership (the exact predicate) decides the rigid rule
        // and the neighbour lists
        if (DEBUG || (RIGID && !r.gran && P.w == 0.0f)) {
          const float s = sq_dist(P.x, P.y, P.z, x, y, z);
          if (s < gc.h2) {
            r.gran |= (P.w == 0.0f);
            if (DEBUG) {
              if (ids != nullptr && (int64_t)r.count < max_k) ids[r.count] = __float_as_uint(lr[j].v.w);
              r.count += 1u;
            }
          }
          if (DEBUG && ((s < gc.h2) != (w > 0.0f))) r.wdis = fmaxf(r.wdis, fmaxf(w, direct_weight(s, gc.inv_h2)));
        }
      }
    }
  }
  // Rigid LR particles count only next to a granular one (Section 4).
  if (RIGID && !r.gran) {
    r.S = 0.f;
    r.Ux = r.Uy = r.Uz = 0.f;
    r.M = 0.f;
    r.arg = 0xffffffffu;
  }
  return r;
}

// Element o of the array at p, addressed as a base pointer (uniform across
// the wave, so in scalar registers) plus a 32-bit lane offset, instead of a
// 64-bit address per lane.
__device__ __forceinline__ const float* col(const float* p, uint32_t o) {
  return reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + (uint32_t)(o * 4u));
}
__device__ __forceinline__ float* col(float* p, uint32_t o) {
  return reinterpret_cast<float*>(reinterpret_cast<char*>(p) + (uint32_t)(o * 4u));
}

// A copy of *p for a wave-uniform p into data that stays unchanged for the
// whole kernel, read through the constant address space: the compiler then
// issues scalar loads and keeps the values in scalar registers.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  typedef const __attribute__((address_space(4))) uint32_t* ConstDword;
  const ConstDword q = (ConstDword)(const void*)p;
  T out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = q[k];
  return out;
}

// WP: a pointer to the wall table, generic or in the constant address space.
// need: the walls the wave tests (bit k: wall k); a wall whose bit is clear
// has its plane at least r_hr from every lane's position, so its test would
// fail for all of them.  A push moves a particle off the position those bits
// were cleared for, so after one every later wall is tested.
template <class WP>
__device__ __forceinline__ void apply_walls(WP walls, int n_walls, uint32_t need, float r_hr,
                                            float ox, float oy, float oz, float& x, float& y, float& z,
                                            float& vx, float& vy, float& vz) {
  for (int k = 0; k < n_walls; ++k) {
    if (((need >> k) & 1u) == 0u) continue;
    const auto w = walls + k * UPSAMPLE_WALL_FLOATS;
    bool pushed = false;
    const float nx = w[0], ny = w[1], nz = w[2], d = w[3];
    const float pen = fmaf(nz, z, fmaf(ny, y, nx * x)) - d;
    if (pen < r_hr) {  // rare: most particles are clear of most walls
      const float ax = w[4], ay = w[5], az = w[6], b = w[7];
      const float px = w[8], py = w[9], pz = w[10], R = w[11];
      bool act = fmaf(az, z, fmaf(ay, y, ax * x)) >= b;
      if (R > 0.0f) {
        // in-plane distance from the hole centre >= R, compared squared
        const float rx = x - px, ry = y - py, rz = z - pz;
        const float rn = fmaf(nz, rz, fmaf(ny, ry, nx * rx));
        const float ix = fmaf(-rn, nx, rx), iy = fmaf(-rn, ny, ry), iz = fmaf(-rn, nz, rz);
        act = act && (fmaf(iz, iz, fmaf(iy, iy, ix * ix)) >= R * R);
      }
      act = act && (fmaf(nz, oz, fmaf(ny, oy, nx * ox)) - d >= 0.0f);
      if (act) {
        const float push = r_hr - pen;
        x = fmaf(push, nx, x);
        y = fmaf(push, ny, y);
        z = fmaf(push, nz, z);
        const float vn = fmaf(nz, vz, fmaf(ny, vy, nx * vx));
        if (vn < 0.0f) {
          vx = fmaf(-vn, nx, vx);
          vy = fmaf(-vn, ny, vy);
          vz = fmaf(-vn, nz, vz);
        }
        pushed = true;
      }
    }
    if (need != ~0u && __ballot(pushed) != 0ull) need = ~0u;
  }
}

// The walls a wave tests: those flagged in the mask of cell c (uniform
// values), valid for particles inside that cell's neighbourhood; mask ~0
// when there is no mask table or the wave's box is too wide.  The region's
// bounds are formed only where they are used, so that nothing but scalar
// registers is held across the candidate walk.
struct WallCull {
  uint32_t mask;
  int c[3];
};
__device__ __forceinline__ WallCull all_walls() { return WallCull{~0u, {0, 0, 0}}; }

// Cull for a wave whose box corners lie in cells (x0, y0, z0) .. (x1, y1, z1)
// (uniform values): the mask table covers the neighbourhood of reach + 1
// cells around each cell, so for a box of at most two cells per axis the
// mask of its first cell serves (one scalar load), with the region running
// reach + 1 cells beyond that cell on each side.
__device__ __forceinline__ WallCull wall_cull(const GridConst& gc, const uint32_t* __restrict__ wall_mask,
                                              int x0, int x1, int y0, int y1, int z0, int z1) {
  WallCull wc = all_walls();
  if (wall_mask == nullptr) return wc;
  x0 = __builtin_amdgcn_readfirstlane(x0);
  x1 = __builtin_amdgcn_readfirstlane(x1);
  y0 = __builtin_amdgcn_readfirstlane(y0);
  y1 = __builtin_amdgcn_readfirstlane(y1);
  z0 = __builtin_amdgcn_readfirstlane(z0);
  z1 = __builtin_amdgcn_readfirstlane(z1);
  if (x1 - x0 > 1 || y1 - y0 > 1 || z1 - z0 > 1) return wc;
  const uint32_t sy = (uint32_t)gc.dims[0], sz = sy * (uint32_t)gc.dims[1];
  wc.mask = load_uniform(wall_mask + ((uint32_t)x0 + sy * (uint32_t)y0 + sz * (uint32_t)z0));
  wc.c[0] = x0;
  wc.c[1] = y0;
  wc.c[2] = z0;
  return wc;
}

// Shepard average, blend, symplectic Euler and walls for one HR particle, the
// particle first + o (first uniform).
template <class WP>
__device__ __forceinline__ void finish(const AdvanceArgs& a, WP walls, int64_t first, uint32_t o, float x,
                                      float y, float z, float vx, float vy, float vz, float S,
                                      float Ux, float Uy, float Uz, float M, bool* A_out,
                                      const WallCull& wc = all_walls()) {
  // Shepard average and blend parameter (Section 4); empty support -> v~ = 0, alpha = 1.
  float tx = 0.f, ty = 0.f, tz = 0.f;
  bool A = true;
  if (S > 0.0f) {
    const float r = __builtin_amdgcn_rcpf(S);  // 1 ulp; the adjoint's replay uses the same
    tx = Ux * r;
    ty = Uy * r;
    tz = Uz * r;
    A = (M <= a.sc.c1) || (M * r >= a.sc.c2);
  }
  const float alpha = A ? 1.0f - M : 0.0f;
  const float dt = a.sc.dt;
  const float fx = fmaf(dt, a.sc.g[0], vx), fy = fmaf(dt, a.sc.g[1], vy), fz = fmaf(dt, a.sc.g[2], vz);
  float nvx = fmaf(alpha, fx - tx, tx), nvy = fmaf(alpha, fy - ty, ty), nvz = fmaf(alpha, fz - tz, tz);
  float nx = fmaf(dt, nvx, x), ny = fmaf(dt, nvy, y), nz = fmaf(dt, nvz, z);
  uint32_t need = ~0u;
  if (wc.mask != ~0u) {
    // the culled set holds if every (live) lane's new position lies in the
    // neighbourhood of cells c - reach - 1 .. c + reach + 1
    const GridConst& gc = a.gc;
    const int M = gc.reach + 1;
    const bool in = nx >= fmaf((float)(wc.c[0] - M), gc.cs, gc.lo[0]) &&
                    nx <= fmaf((float)(wc.c[0] + M + 1), gc.cs, gc.lo[0]) &&
                    ny >= fmaf((float)(wc.c[1] - M), gc.cs, gc.lo[1]) &&
                    ny <= fmaf((float)(wc.c[1] + M + 1), gc.cs, gc.lo[1]) &&
                    nz >= fmaf((float)(wc.c[2] - M), gc.cs, gc.lo[2]) &&
                    nz <= fmaf((float)(wc.c[2] + M + 1), gc.cs, gc.lo[2]);
    if (__ballot(!in) == 0ull) need = wc.mask;
  }
  apply_walls(walls, a.sc.n_walls, need, a.sc.r_hr, x, y, z, nx, ny, nz, nvx, nvy, nvz);
  const int64_t n = a.ld;
  float* const px = a.hx_out + first;
  float* const pv = a.hv_out + first;
  *col(px, o) = nx;
  *col(px + n, o) = ny;
  *col(px + 2 * n, o) = nz;
  *col(pv, o) = nvx;
  *col(pv + n, o) = nvy;
  *col(pv + 2 * n, o) = nvz;
  *A_out = A;
}

// Per-lane walk (exact predicate): debug exports and waves whose particles are
// too spread out for a shared candidate list.
template <bool DEBUG>
__global__ __launch_bounds__(kBlock) void k_advance(AdvanceArgs a, WallTable wt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.ld;
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  uint32_t* ids = (DEBUG && a.dbg_ids != nullptr) ? a.dbg_ids + i * a.dbg_max_k : nullptr;
  const Sums s = gather<DEBUG, true>(a.gc, a.lr, a.cell_start, x, y, z, ids, a.dbg_max_k);
  bool A;
  finish(a, wt.w, (int64_t)blockIdx.x * kBlock, threadIdx.x, x, y, z, vx, vy, vz, s.S, s.Ux, s.Uy, s.Uz, s.M, &A);
  if (DEBUG) {
    if (a.dbg_count != nullptr) a.dbg_count[i] = s.count;
    if (a.dbg_branch != nullptr)
      a.dbg_branch[i] = (uint8_t)((A ? 1 : 0) | (s.gran ? 2 : 0) | (s.S > 0.0f ? 4 : 0));
  }
}

// Wave-tiled gather (tile.hpp): every lane walks its group's LDS candidate
// list,   d = X_j - x_i,  t = 1 - |d|^2 / h^2,  w = max(t, 0)^3,
// accumulating S, U, M; the per-lane stencil walk covers spread-out waves.
constexpr int kGatherListEntries = 128;  // per wave, split over the G group lists
constexpr uint32_t kLaneWalkShare = 4;  // see advance_tile
constexpr int kGatherRows = 64;

// The single-scene step kernel runs blocks of one wave: a block's LDS is
// released only when its slowest wave ends, so one-wave blocks leave no slot
// idle behind a long wave (the batched kernel runs its kBlock-particle tiles
// as one-wave blocks too).
constexpr int kGatherThreads = 64;
template <int G, int W = kWaves>
using GatherLDS = TileLDS<G, (kGatherListEntries / G > 64 ? kGatherListEntries / G : 64), kGatherRows, W>;

// The cull of a one-group wave in centred form: candidates are tested on
// q = X - c against the wave box's centre c and half-extents (tile_visit),
// and the list keeps their absolute positions.  Lanes then evaluate the
// weight in the direct form d = X_j - x_i, 1 - |d|^2 / h^2, whose argument
// is accurate to a few float32 units of 1.  (An expanded dot-product form,
// (1 - |p|^2/h^2) - |q|^2/h^2 + 2 p.q / h^2 relative to the box centre, saves
// three operations per entry but cancels terms as large as 12 for boxes 2h
// wide, with errors of several 1e-6 in the argument: more than the per-step
// velocity tolerance allows in dense supports.)
struct CentredCull : PlainStage {
  static constexpr bool kCentred = true;
  float cx, cy, cz;
  float hx, hy, hz;  // half-extents of the wave box
  __device__ __forceinline__ float4 centred(float4 P, uint32_t bits) const { return (*this)(P, bits); }
};

// Velocity entries (V_j, 1): with them the sums (Ux, Uy, Uz, S) of a wave are
// one matrix product, weights (64 lanes x entries) times entries (entries x 4).
template <class Base>
struct WithOnes : Base {
  __device__ __forceinline__ float4 vel(float4 V, uint32_t /*bits*/) const { return make_float4(V.x, V.y, V.z, 1.0f); }
};

// Debug twin of a stage: the velocity entry keeps the candidate's sorted
// index in .w (padding: all ones), so that the walk can look up the
// candidate's absolute position for the exact predicate.  Culling and the
// position entries are the base stage's.
template <class Base>
struct WithSortedIndex : Base {
  __device__ __forceinline__ float4 vel(float4 V, uint32_t bits) const {
    return make_float4(V.x, V.y, V.z, __uint_as_float(bits & 0x7fffffffu));
  }
  __device__ __forceinline__ float4 pad_vel() const { return make_float4(0.f, 0.f, 0.f, __uint_as_float(~0u)); }
};

// Member accounting of the debug instance of the step kernel, per lane.
struct DebugWalk {
  uint32_t* ids;  // this lane's id row, or null (idle lanes, no id export)
  int64_t max_k;
  uint32_t count, count_w;
  float wdis;
  // One list entry: w as the kernel computed it, the candidate's absolute
  // position P and original index.
  __device__ __forceinline__ void see(float w, float px, float py, float pz, uint32_t orig, float x, float y,
                                      float z, const GridConst& gc) {
    const float s = sq_dist(px, py, pz, x, y, z);
    const bool member = s < gc.h2;
    const bool pos = w > 0.0f;
    if (member) {
      if (ids != nullptr && (int64_t)count < max_k) ids[count] = orig;
      count += 1u;
    }
    count_w += pos ? 1u : 0u;
    if (member != pos) wdis = fmaxf(wdis, fmaxf(w, direct_weight(s, gc.inv_h2)));
  }
};

typedef float v4f __attribute__((ext_vector_type(4)));



// One list entry of the matrix-core accumulation (v_mfma_f32_4x4x1f32, 16
// blocks of 4 lanes): lane l supplies its weight w (A) and component l mod 4
// of the entry's (Vx, Vy, Vz, 1) (B); register r of lane l accumulates
// sum_c w(particle 4 floor(l/4) + r, c) * V_c[l mod 4].
__device__ __forceinline__ v4f mfma_entry(float w, float b, v4f acc) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(w, b, acc, 0, 0, 0);
}

// max(u, 0)^3 for u <= 1 (the kernel's argument never exceeds 1 but by
// rounding): (u u) u clamped to [0, 1], the clamp folded into the multiply.
__device__ __forceinline__ float cube01(float u) {
  return __builtin_amdgcn_fmed3f((u * u) * u, 0.0f, 1.0f);
}

// Value of v at lane n of each quad (DPP quad_perm [n, n, n, n]; every lane
// has a valid source).
template <int N>
__device__ __forceinline__ float quad_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), N * 0x55, 0xf, 0xf, true));
}

// Register i of lane 4q + n, for the lane 4q + i that calls it (flat selects,
// no branches).
template <int N>
__device__ __forceinline__ float quad_pick(v4f acc, bool i1, bool i2, bool i3) {
  float o = quad_lane<N>(acc[0]);
  const float t1 = quad_lane<N>(acc[1]), t2 = quad_lane<N>(acc[2]), t3 = quad_lane<N>(acc[3]);
  o = i1 ? t1 : o;
  o = i2 ? t2 : o;
  o = i3 ? t3 : o;
  return o;
}

// Transpose of each quad's 4 x 4 block: lane 4q + i receives register i of
// lanes 4q + 0..3, i.e. (Ux, Uy, Uz, S) of its own particle.
__device__ __forceinline__ void quad_sums(v4f acc, int lane, float& Ux, float& Uy, float& Uz, float& S) {
  const int i = lane & 3;
  const bool i1 = i == 1, i2 = i == 2, i3 = i == 3;
  Ux = quad_pick<0>(acc, i1, i2, i3);
  Uy = quad_pick<1>(acc, i1, i2, i3);
  Uz = quad_pick<2>(acc, i1, i2, i3);
  S = quad_pick<3>(acc, i1, i2, i3);
}

// The same transpose through the wave's LDS list (free once its walk is
// done): lane 4q + n stores register r at float 16q + 4r + n, so particle
// 4q + r's four sums sit at floats 4(4q + r) .. +3, one 16-byte read per lane.
// Data movement only: the sums are those of quad_sums bit for bit.
__device__ __forceinline__ void lds_quad_sums(v4f acc, int lane, float4* scratch, float& Ux, float& Uy,
                                              float& Uz, float& S) {
  float* t = reinterpret_cast<float*>(scratch) + 16 * (lane >> 2) + (lane & 3);
  t[0] = acc[0];
  t[4] = acc[1];
  t[8] = acc[2];
  t[12] = acc[3];
  wave_lds_sync();
  const float4 r = scratch[lane];
  Ux = r.x;
  Uy = r.y;
  Uz = r.z;
  S = r.w;
  wave_lds_sync();  // the read is done before the wave writes the list again
}

// The lane's particle within the tile at first: threadIdx.x, or the tile's
// last particle for idle lanes past n.
__device__ __forceinline__ uint32_t lane_offset(const AdvanceArgs& a, int64_t first) {
  const int64_t last = a.n - 1 - first;
  const uint32_t lastc = (uint32_t)(last < kBlock - 1 ? last : kBlock - 1);
  return min((uint32_t)threadIdx.x, lastc);
}

// One lane's HR state: the particle first + threadIdx.x, or the last particle
// for idle lanes past n.
struct HRLane {
  float x, y, z, vx, vy, vz;
};
__device__ __forceinline__ HRLane load_lane(const AdvanceArgs& a, int64_t first) {
  const int64_t n = a.ld;
  const uint32_t o = lane_offset(a, first);
  const float* const px = a.hx + first;
  const float* const pv = a.hv + first;
  return HRLane{*col(px, o), *col(px + n, o), *col(px + 2 * n, o),
                *col(pv, o), *col(pv + n, o), *col(pv + 2 * n, o)};
}

// One block of HR particles first .. first + blockDim.x - 1, one wave each 64
// (those below a.n are live; the rest shadow the last particle and write
// nothing).
// TAPE: also record (S, Ux, Uy, Uz, M, argmax) per particle for the adjoint.
// DBG: the same arithmetic, plus per-lane member exports (AdvanceArgs dbg_*):
// the exact predicate on every list entry (or stencil candidate), the count
// of entries of positive computed weight and the largest weight on which the
// two disagree.
template <bool RIGID, int G, bool TAPE = false, bool DBG = false, class WP, class LDS>
__device__ __forceinline__ void advance_tile(const AdvanceArgs& a, WP walls,
                                             LDS& lds, int64_t first, const HRLane& st) {
  static_assert(!(TAPE && DBG), "the debug instance records no tape");
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool live = first + (int64_t)threadIdx.x < a.n;  // idle lanes shadow the last particle
  const float x = st.x, y = st.y, z = st.z;
  const float vx = st.vx, vy = st.vy, vz = st.vz;
  const GridConst& gc = a.gc;

  float S = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, M = 0.f;
  uint32_t arg = 0xffffffffu;
  // TAPE: (weight bits << 32 | ~index) -- its unsigned maximum is the largest
  // weight and, among equal weights, the smallest index
  uint64_t key = 0ull;
  WallCull wc = all_walls();
  DebugWalk dw{nullptr, 0, 0u, 0u, 0.0f};
  if (DBG && live && a.dbg_ids != nullptr) {
    dw.ids = a.dbg_ids + (first + (int64_t)threadIdx.x) * a.dbg_max_k;
    dw.max_k = a.dbg_max_k;
  }
  const TileSetup<G> ts = tile_setup<G>(gc, a.cell_start, x, y, z, lane, wid, lds);
  // The per-lane walk: for waves whose rows overflow the LDS, and for waves
  // streaming more than tile_max candidates whose lanes' own stencils hold
  // fewer than 1 / kLaneWalkShare of them (spread-out waves).  A compact wave
  // in dense LR keeps the shared list: its lanes would each walk nearly all
  // of the candidates one dependent load at a time.  tile_max 0 sends every
  // wave with candidates to the per-lane walk.
  bool per_lane = ts.nrows > lds.kRows;
  if (!per_lane && ts.total > (uint32_t)a.tile_max)
    per_lane = a.tile_max == 0 || kLaneWalkShare * lane_walk_max(gc, a.cell_start, x, y, z) < ts.total;
  if (per_lane) {
    // every lane walks its own stencil
    const Sums s = gather<DBG, RIGID, TAPE>(gc, a.lr, a.cell_start, x, y, z, dw.ids, dw.max_k);
    S = s.S; Ux = s.Ux; Uy = s.Uy; Uz = s.Uz; M = s.M; arg = s.arg;
    if (DBG) {
      dw.count = s.count;
      dw.count_w = s.count_w;
      dw.wdis = s.wdis;
    }
  } else {
    const float inv_h2 = gc.inv_h2;
    bool gran = !RIGID;
    // the wave's box (union of its groups)
    float lo0 = ts.gb[0].lo[0], lo1 = ts.gb[0].lo[1], lo2 = ts.gb[0].lo[2];
    float hi0 = ts.gb[0].hi[0], hi1 = ts.gb[0].hi[1], hi2 = ts.gb[0].hi[2];
#pragma unroll
    for (int g = 1; g < G; ++g) {
      lo0 = fminf(lo0, ts.gb[g].lo[0]); lo1 = fminf(lo1, ts.gb[g].lo[1]); lo2 = fminf(lo2, ts.gb[g].lo[2]);
      hi0 = fmaxf(hi0, ts.gb[g].hi[0]); hi1 = fmaxf(hi1, ts.gb[g].hi[1]); hi2 = fmaxf(hi2, ts.gb[g].hi[2]);
    }
    wc = wall_cull(gc, a.wall_mask, ts.bx0, ts.bx1, ts.by0, ts.by1, ts.bz0, ts.bz1);
    {
      // weights in the vector unit, sums on the matrix cores
      v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
      const int comp = lane & 3;
      // M as the integer maximum of the weights' bits: exact for w >= 0 (a
      // -0 weight sorts lowest) and free of the NaN canonicalisation of fmaxf
      int Mb = 0;
      // one list entry: lvf points at the velocity list as floats.  Without a
      // tape the entries are (V_j, 1); with one they keep the index bits in
      // .w for the argmax, and lanes of component 3 use 1 instead.
      auto take = [&](float w, const float* lvf, uint32_t c) {
        float b = lvf[4 * c + comp];
        if (DBG) {
          b = comp == 3 ? 1.0f : b;
          const uint32_t jb = __float_as_uint(lvf[4 * c + 3]);
          if (jb != ~0u) {
            const LRPoint& P = a.lr[jb];
            dw.see(w, P.p.x, P.p.y, P.p.z, __float_as_uint(P.v.w), x, y, z, gc);
          }
        }
        if (TAPE) {
          b = comp == 3 ? 1.0f : b;
          const uint32_t id = __float_as_uint(lvf[4 * c + 3]);
          const uint64_t k = ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(~id);
          key = k > key ? k : key;
        } else {
          Mb = max(Mb, __float_as_int(w));
        }
        acc = mfma_entry(w, b, acc);
      };
      auto walk = [&](uint32_t nc, const float4* lp, const float4* lv) {
        const float* lvf = reinterpret_cast<const float*>(lv);
        auto step = [&](uint32_t c) {
          const float4 Q = lp[c];
          const float dx = Q.x - x, dy = Q.y - y, dz = Q.z - z;
          const float sq = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          take(cube01(fmaf(-sq, inv_h2, 1.0f)), lvf, c);
        };
        uint32_t c0 = 0;
        if (RIGID) {
          // With rigid particles a lane must learn whether a granular LR
          // particle is its member: the squared distance rounded operation
          // by operation (the exact predicate; padding entries are far)
          // decides, and the weight is taken from it too.  Once every lane
          // of the wave has met one, the rest of the list takes the plain
          // walk.  Four entries per trip.
          auto step_rigid = [&](uint32_t c) {
            const float4 Q = lp[c];
            const float dx = Q.x - x, dy = Q.y - y, dz = Q.z - z;
            const float sq = (dx * dx + dy * dy) + dz * dz;
            gran |= ((__float_as_uint(Q.w) & 0x80000000u) == 0u) & (sq < gc.h2);
            take(cube01(fmaf(-sq, inv_h2, 1.0f)), lvf, c);
          };
          for (; c0 + 4u <= nc; c0 += 4u) {
            if (__builtin_amdgcn_ballot_w64(!gran) == 0ull) break;
#pragma unroll
            for (int k = 0; k < 4; ++k) step_rigid(c0 + (uint32_t)k);
          }
        }
        // eight entries per trip (one address update), then a last four
        for (; c0 + 8u <= nc; c0 += 8u) {
#pragma unroll
          for (int k = 0; k < 8; ++k) step(c0 + (uint32_t)k);
        }
        if (c0 < nc) {
#pragma unroll
          for (int k = 0; k < 4; ++k) step(c0 + (uint32_t)k);
        }
      };
      if (G == 1) {
        const CentredCull cc{{}, 0.5f * (lo0 + hi0), 0.5f * (lo1 + hi1), 0.5f * (lo2 + hi2),
                             0.5f * (hi0 - lo0), 0.5f * (hi1 - lo1), 0.5f * (hi2 - lo2)};
        using Stage = std::conditional_t<DBG, WithSortedIndex<CentredCull>,
                                         std::conditional_t<TAPE, CentredCull, WithOnes<CentredCull>>>;
        tile_visit<G, 4>(ts, gc, a.lr, lane, wid, lds, walk, SortedTag(), Stage{cc});
      } else {
        using Stage = std::conditional_t<DBG, WithSortedIndex<PlainStage>,
                                         std::conditional_t<TAPE, PlainStage, WithOnes<PlainStage>>>;
        tile_visit<G, 4>(ts, gc, a.lr, lane, wid, lds, walk, SortedTag(), Stage{});
      }
      if (!TAPE) M = __int_as_float(Mb);
      lds_quad_sums(acc, lane, &lds.p[wid][0][0], Ux, Uy, Uz, S);
    }
    if (TAPE) {
      M = __uint_as_float((uint32_t)(key >> 32));
      arg = ~(uint32_t)key;  // meaningful only when M > 0
    }
    if (RIGID && !gran) {
      S = Ux = Uy = Uz = M = 0.f;
      arg = 0xffffffffu;
    }
  }
  if (live) {
    bool A;
    const uint32_t o = threadIdx.x;
    finish(a, walls, first, o, x, y, z, vx, vy, vz, S, Ux, Uy, Uz, M, &A, wc);
    if (DBG) {
      const int64_t i = first + (int64_t)o;
      if (a.dbg_count != nullptr) a.dbg_count[i] = dw.count;
      if (a.dbg_count_w != nullptr) a.dbg_count_w[i] = dw.count_w;
      if (a.dbg_wdis != nullptr) a.dbg_wdis[i] = dw.wdis;
    }
    if (TAPE) {
      const int64_t m = a.n;
      float* const pt = a.tape + first;
      *col(pt, o) = S;
      *col(pt + m, o) = Ux;
      *col(pt + 2 * m, o) = Uy;
      *col(pt + 3 * m, o) = Uz;
      *col(pt + 4 * m, o) = M;
      *col(pt + 5 * m, o) = __uint_as_float(arg);
    }
  }
}

// Seven waves per SIMD asked of the register allocator; with four lane groups
// the LDS lists (35 KB per block) allow four.
template <bool RIGID, int G, bool TAPE = false, bool DBG = false>
__global__ __launch_bounds__(kGatherThreads, G == 4 ? 4 : 7) void k_advance_tiled(AdvanceArgs a, WallTable wt) {
  __shared__ GatherLDS<G, kGatherThreads / 64> lds;
  const int64_t first = (int64_t)blockIdx.x * kGatherThreads;
  advance_tile<RIGID, G, TAPE, DBG>(a, wt.w, lds, first, load_lane(a, first));
}

// Batched step over the (scene, first particle) tile table; each tile reads
// its scene's constants from the scene table.  A kBlock-particle tile is run
// by four one-wave blocks.  Blocks go to the 8 XCDs round robin and the tile
// table is laid out so that tile position p runs on XCD p mod 8: block q
// takes wave (q / 8) mod 4 of position 8 (q / 32) + q mod 8, which keeps each
// tile on its XCD and its four waves within 32 consecutive blocks.  The
// waves are those of the single-scene kernel, so the results are
// bit-identical to it.  Seven waves per SIMD: 72 VGPRs without spills (the
// scene constants are in scalar registers).
constexpr int kTileWaves = kBlock / kGatherThreads;
static_assert(kTileWaves == 4, "the block-to-wave map assumes four waves per tile");
template <bool RIGID>
__global__ __launch_bounds__(kGatherThreads, 7) void k_advance_batched(BatchAdvanceArgs b) {
  __shared__ GatherLDS<1, kGatherThreads / 64> lds;
  const int64_t total = (b.n_tiles + 7) / 8 * 32;
  for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
    const int64_t pos = (q >> 5) * 8 + (q & 7);
    if (pos >= b.n_tiles) continue;  // block-uniform
    const BatchTile tile = load_uniform(b.tiles + pos);
    const BatchScene sc = load_uniform(b.scenes + tile.scene);
    const int64_t first = (int64_t)tile.first + ((q >> 3) & 3) * kGatherThreads;
    if (first >= sc.n_hr) continue;  // past the scene's last particle (block-uniform)
    AdvanceArgs a;
    a.gc = sc.gc;
    a.sc = sc.sc;
    a.lr = b.lr;
    a.cell_start = b.cell_start + sc.cell_base;
    a.hx = b.hx + sc.hr_off;
    a.hv = b.hv + sc.hr_off;
    a.hx_out = b.hx_out + sc.hr_off;
    a.hv_out = b.hv_out + sc.hr_off;
    a.n = sc.n_hr;
    a.ld = b.ld;
    a.dbg_count = nullptr;
    a.dbg_ids = nullptr;
    a.dbg_max_k = 0;
    a.dbg_branch = nullptr;
    a.dbg_count_w = nullptr;
    a.dbg_wdis = nullptr;
    a.wall_mask = nullptr;
    a.groups = 1;
    a.tile_max = b.tile_max;
    a.tape = nullptr;
    typedef const __attribute__((address_space(4))) float* ConstFloat;  // scalar loads of the scene's walls
    advance_tile<RIGID, 1>(a, (ConstFloat)(const void*)(b.walls + sc.wall_off), lds, first, load_lane(a, first));
  }
}

}  // namespace

hipError_t launch_advance(const AdvanceArgs& a, const WallTable& walls, int debug, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n + kBlock - 1) / kBlock);
  const unsigned tblocks = (unsigned)((a.n + kGatherThreads - 1) / kGatherThreads);
  if (debug == 1)
    hipLaunchKernelGGL(k_advance<true>, dim3(blocks), dim3(kBlock), 0, st, a, walls);
  else if (debug == 2 && a.sc.has_rigid)
    hipLaunchKernelGGL((k_advance_tiled<true, 1, false, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (debug == 2 && a.groups == 4)
    hipLaunchKernelGGL((k_advance_tiled<false, 4, false, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (debug == 2 && a.groups == 2)
    hipLaunchKernelGGL((k_advance_tiled<false, 2, false, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (debug == 2)
    hipLaunchKernelGGL((k_advance_tiled<false, 1, false, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (a.tape != nullptr && a.sc.has_rigid)
    hipLaunchKernelGGL((k_advance_tiled<true, 1, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (a.tape != nullptr)
    hipLaunchKernelGGL((k_advance_tiled<false, 1, true>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (a.sc.has_rigid)
    hipLaunchKernelGGL((k_advance_tiled<true, 1>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (a.groups == 4)
    hipLaunchKernelGGL((k_advance_tiled<false, 4>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else if (a.groups == 2)
    hipLaunchKernelGGL((k_advance_tiled<false, 2>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  else
    hipLaunchKernelGGL((k_advance_tiled<false, 1>), dim3(tblocks), dim3(kGatherThreads), 0, st, a, walls);
  return hipGetLastError();
}

hipError_t launch_advance_batched(const BatchAdvanceArgs& b, int grid, hipStream_t st) {
  if (b.n_tiles == 0) return hipSuccess;
  const dim3 blocks((unsigned)((grid + 7) / 8 * 32));
  if (b.rigid)
    hipLaunchKernelGGL(k_advance_batched<true>, blocks, dim3(kGatherThreads), 0, st, b);
  else
    hipLaunchKernelGGL(k_advance_batched<false>, blocks, dim3(kGatherThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace ups
