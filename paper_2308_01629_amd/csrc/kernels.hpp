// Host-side launchers of the library's kernels (one translation unit each)
// and the device helpers that several of them share.
#pragma once

#include <string>

#include "common.hpp"

namespace ups {

// Key of the cell holding a position: x fastest, coordinates clamped into the
// grid.
__device__ __forceinline__ uint32_t cell_key(const GridConst& gc, float x, float y, float z) {
  int cx = cell_coord(x, gc.lo[0], gc.inv_cs, gc.dims[0]);
  int cy = cell_coord(y, gc.lo[1], gc.inv_cs, gc.dims[1]);
  int cz = cell_coord(z, gc.lo[2], gc.inv_cs, gc.dims[2]);
  return (uint32_t)cx + (uint32_t)gc.dims[0] * ((uint32_t)cy + (uint32_t)gc.dims[1] * (uint32_t)cz);
}

// Arrival slot of key k inside its bin.  Lanes whose key equals the key of the
// lane before them join that lane's run; the first lane of each run claims
// the whole run with one atomic add.  Nearly sorted input (the HR reorder)
// then costs a handful of atomics per wave instead of 64.  Every lane of the
// wave calls it (invalid lanes with valid = false): it shuffles and votes
// across the whole wave.
__device__ __forceinline__ uint32_t claim_slot(uint32_t k, bool valid, uint32_t* counts) {
  const int lane = threadIdx.x & 63;
  const uint32_t kk = valid ? k : 0xffffffffu;
  const uint32_t prev = __shfl_up(kk, 1, 64);
  const bool head = (lane == 0) || (prev != kk);
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll(heads & upto);
  const uint64_t above = heads & ~upto;
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  uint32_t base = 0u;
  if (head && valid) base = atomicAdd(&counts[kk], (uint32_t)(next - lane));
  base = __shfl(base, start, 64);
  return base + (uint32_t)(lane - start);
}

// Scratch of one grid build (device pointers, owned by a handle).
struct GridScratch {
  uint32_t* keys;        // [max_lr] cell key per LR (original order)
  uint32_t* slot;        // [max_lr] arrival slot inside the cell (unstable)
  uint32_t* tmp;         // [max_lr] unstable cell order
  uint32_t* perm;        // [max_lr] stable cell order: original index per sorted slot
  uint32_t* counts;      // [n_cells] per-cell count; zero between builds
  uint32_t* local;       // [n_cells] exclusive scan inside each scan chunk
  uint32_t* chunk_sum;   // [n_chunks + 1] chunk totals, then exclusive chunk offsets
  uint32_t* cell_start;  // [n_cells + 1]
  LRPoint* lr_sorted;    // [max_lr]
};

// a2..a5: keys + counts, chunked scan, unstable scatter, stable fix + LR reorder.
hipError_t launch_build_grid(const GridConst& gc, const float* lr_x, const float* lr_v,
                             const uint8_t* lr_rigid, int64_t n_lr, int64_t n_cells,
                             const GridScratch& s, hipStream_t st);
// A build over positions alone (x [3][n]) without the stable fix: the sorted
// copy holds x and an int32 tag per particle (as bits; 0 without a tag
// array) in p, the index in v.w, and inside a cell its order varies from
// run to run.  Leaves perm and
// tmp untouched.  keys_ready: a kernel before it on the stream has already
// written s.keys and s.slot and counted into s.counts (claim_slot on the
// cell_key of these same positions), so the build starts at the scan.
hipError_t launch_build_grid_points(const GridConst& gc, const float* x, const int32_t* tag, int64_t n,
                                    int64_t n_cells, const GridScratch& s, hipStream_t st,
                                    bool keys_ready = false);
// The same build of the LR state between two frames: x0 + theta (x1 - x0)
// (and v alike), each float32 operation rounded separately, fused into the
// keys and the sorted copy.
hipError_t launch_build_grid_lerp(const GridConst& gc, const float* x0, const float* v0, const float* x1,
                                  const float* v1, float theta, const uint8_t* lr_rigid, int64_t n_lr,
                                  int64_t n_cells, const GridScratch& s, hipStream_t st);

// Exclusive scan of n_bins counts (zeroed behind): local[b] + chunk_sum[b /
// kScanChunk] is bin b's offset, chunk_sum[n_chunks] the total.
hipError_t launch_scan_bins(uint32_t* counts, int64_t n_bins, uint32_t* local, uint32_t* chunk_sum,
                            hipStream_t st);

// The sorted LR copy as [3][n] positions and velocities (either may be null).
hipError_t launch_unpack_sorted(const LRPoint* lr, int64_t n, float* x, float* v, hipStream_t st);

// HR reorder by a space-filling key of fine cells (grid cells split into sub^3
// sub-cells: Hilbert index, global Morton code, or cell then Morton order),
// so that a wave's 64 consecutive particles sit in a compact box and
// neighbouring waves are neighbours in space.
struct HRSortScratch {
  uint32_t* keys;       // [max_hr]
  uint32_t* slot;       // [max_hr]
  uint32_t* src;        // [max_hr] source index of each (key, slot) entry
  float* x;             // [3][max_hr]
  float* v;             // [3][max_hr]
  int32_t* perm;        // [max_hr]
  uint32_t* counts;     // [n_bins], zero between sorts
  uint32_t* local;      // [n_bins]
  uint32_t* chunk_sum;  // [n_bins / kScanChunk + 2]
  int64_t n_cells;      // grid cells
  int64_t n_bins;       // bins allocated in counts / local
  int max_sub;          // largest sub-cell count per axis the bins are sized for (4, 2 or 1)
};

// Significant bits of a fine coordinate in [0, n).
inline int sort_bits(int64_t n) {
  int b = 0;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}
// Bins of the HR reorder for a sub-cell count: mode 1 (global Morton code of
// fine cells) 2^(bx + by + bz); mode 0 (grid cell, then Morton order of its
// sub-cells) n_cells * sub^3; mode 2 (global Hilbert index of fine cells, on
// a cube of 2^max(bx, by, bz) cells per axis) 2^(3 max(bx, by, bz)).
// Index of fine cell (x0, x1, x2) along a 3-D Hilbert curve over a cube of
// 2^b cells per axis, by Skilling's transpose method ("Programming the Hilbert
// curve", AIP Conf. Proc. 707, 2004): undo the excess work of each level from
// the top bit down, Gray-encode, then interleave the bits with axis 0 most
// significant.  Consecutive indices are face-neighbouring cells, so runs of
// particles in this order fill compact boxes (no Z-order jumps).
__host__ __device__ inline uint32_t hilbert3(uint32_t x0, uint32_t x1, uint32_t x2, int b) {
  for (int k = b - 1; k > 0; --k) {
    const uint32_t q = 1u << k, p = q - 1u;
    x0 = (x0 & q) ? (x0 ^ p) : x0;
    {
      const uint32_t t = (x0 ^ x1) & p;
      const bool hit = (x1 & q) != 0u;
      x0 = hit ? (x0 ^ p) : (x0 ^ t);
      x1 = hit ? x1 : (x1 ^ t);
    }
    {
      const uint32_t t = (x0 ^ x2) & p;
      const bool hit = (x2 & q) != 0u;
      x0 = hit ? (x0 ^ p) : (x0 ^ t);
      x2 = hit ? x2 : (x2 ^ t);
    }
  }
  x1 ^= x0;
  x2 ^= x1;
  uint32_t t = 0u;
  for (int k = b - 1; k > 0; --k) {
    const uint32_t q = 1u << k;
    if (x2 & q) t ^= q - 1u;
  }
  x0 ^= t;
  x1 ^= t;
  x2 ^= t;
  uint32_t key = 0u;
  for (int k = b - 1; k >= 0; --k)
    key = (key << 3) | (((x0 >> k) & 1u) << 2) | (((x1 >> k) & 1u) << 1) | ((x2 >> k) & 1u);
  return key;
}

inline int64_t sort_bins(const int dims[3], int sub, int mode) {
  if (mode == 0) return (int64_t)dims[0] * dims[1] * dims[2] * sub * sub * sub;
  int b = 0, m = 0;
  for (int a = 0; a < 3; ++a) {
    const int ba = sort_bits((int64_t)dims[a] * sub);
    b += ba;
    m = ba > m ? ba : m;
  }
  if (mode == 2) return (int64_t)1 << (3 * m);
  return (int64_t)1 << b;
}
// out_x / out_v may alias hr_x / hr_v (then the permuted copy goes through scratch).
// ld: the stride between the components of hr_x / hr_v (n_hr if negative); a
// strided state is sorted in place, and perm_out receives perm_base + the old
// column.  rank (mode 2 only, else ignored): the Hilbert ranks of the grid's
// fine cells at this sub (launch_hilbert_ranks), which sort the same order on
// one bin per fine cell.
hipError_t launch_sort_hr(const GridConst& gc, const float* hr_x, const float* hr_v, float* out_x,
                          float* out_v, int64_t n_hr, int sub, int mode, const HRSortScratch& s,
                          int32_t* perm_out, hipStream_t st, int64_t ld = -1, int32_t perm_base = 0,
                          const uint32_t* rank = nullptr);

// One scene of a batched HR reorder: its grid, sub-cells per axis, fine grid
// dims (dims * sub) and first bin (also its offset in the rank table).
struct HrRankScene {
  GridConst gc;
  int sub;
  int fdims[3];
  uint32_t base;
};
// Hilbert rank of every fine cell of a grid of fdims fine cells (row-major,
// x fastest) among all of them: rank (uint32 [fx fy fz]); cube, local (uint32
// [2^(3 bits)], cube zero on entry and on exit) and chunk_sum are scratch.
hipError_t launch_hilbert_ranks(const int fdims[3], uint32_t* rank, uint32_t* cube, uint32_t* local,
                                uint32_t* chunk_sum, hipStream_t st);
// Reorder of the columns [0, n) of a batch (scene s owns start[s] ..
// start[s + 1]) in place: key = base + rank[base + fine cell] per scene, one
// counting sort over n_bins bins for all scenes.  perm_out (or null) receives
// the old column of each new column.
hipError_t launch_sort_hr_batched(float* hr_x, float* hr_v, int64_t n, const int64_t* start,
                                  int n_scenes, const HrRankScene* sc, const uint32_t* rank, int64_t n_bins,
                                  const HRSortScratch& s, int32_t* perm_out, hipStream_t st);

// a6: fused gather + blend + integrate + walls.
struct AdvanceArgs {
  GridConst gc;
  StepConst sc;
  const LRPoint* lr;
  const uint32_t* cell_start;
  const float* hx;
  const float* hv;
  float* hx_out;
  float* hv_out;
  int64_t n;
  int64_t ld;  // component stride of the HR arrays ([3][ld]; n for one scene)
  // debug outputs (all may be null)
  uint32_t* dbg_count;
  uint32_t* dbg_ids;
  int64_t dbg_max_k;
  uint8_t* dbg_branch;
  uint32_t* dbg_count_w;  // tiled debug: entries whose computed weight is > 0
  float* dbg_wdis;        // tiled debug: largest weight where that test and membership disagree
  // [n_cells] per cell, bit k set when wall k can come within r_hr of the
  // cell's neighbourhood (cells c - reach - 1 .. c + reach + 1); null: every
  // wave tests every wall
  const uint32_t* wall_mask;
  int groups;    // lane groups per wave in the tiled gather: 1, 2 or 4 (a tuning knob)
  int tile_max;  // a spread-out wave streaming more LR candidates than this walks per lane
  float* tape;   // [6][n] (S, Ux, Uy, Uz, M, argmax bits) or null
};
// debug: 0 the step kernel, 1 the per-lane walk with member exports, 2 the
// step kernel's own template instance with member exports (same arithmetic)
hipError_t launch_advance(const AdvanceArgs& a, const WallTable& walls, int debug, hipStream_t st);

// a9: batched step over many scenes in concatenated buffers.
struct BatchScene {
  GridConst gc;
  StepConst sc;
  int64_t hr_off, n_hr;   // caller's HR columns
  int64_t lr_off, n_lr;   // caller's LR columns
  int64_t lr_int;         // first internal (concatenated) LR index of the scene
  uint32_t cell_base;     // first global cell of the scene
  uint32_t n_cells;
  int32_t wall_off;       // first float of the scene's walls in the wall table
  int32_t pad;
};
struct BatchTile {
  uint32_t scene;
  uint32_t first;  // first particle of the tile inside its scene
};
struct BatchAdvanceArgs {
  const BatchScene* scenes;
  const BatchTile* tiles;  // one per kBlock HR particles of each scene
  int64_t n_tiles;
  const float* walls;
  const LRPoint* lr;           // every scene's sorted LR copy, scene after scene
  const uint32_t* cell_start;  // global cells
  const float* hx;
  const float* hv;
  float* hx_out;
  float* hv_out;
  int64_t ld;  // component stride of the caller's HR arrays
  int tile_max;
  int rigid;
};
hipError_t launch_advance_batched(const BatchAdvanceArgs& b, int grid, hipStream_t st);

// Batched grid rebuild: one key / count / scan / scatter / stable pass over
// the LR particles of every scene (keys offset by the scene's cell base).
struct BatchGridArgs {
  const BatchScene* scenes;
  const BatchTile* lr_blocks;  // one per kBlock LR particles of each scene
  int64_t n_lr_blocks;
  const float* lr_x;
  const float* lr_v;
  const uint8_t* lr_rigid;
  int64_t ld;          // component stride of the caller's LR arrays
  int64_t n_int;       // LR particles of all scenes
  int64_t n_cells;     // cells of all scenes
  uint16_t* scene_of;  // [n_int] scene of each internal LR index
};
hipError_t launch_build_grid_batched(const BatchGridArgs& b, const GridScratch& s, hipStream_t st);

// Host: validate one scene's parameters and compute its grid (runtime.hip).
int check_scene_params(const upsample_params* p, upsample_grid_info* gi, std::string* why);
// Host: the kernels' constants of a scene (runtime.hip).
GridConst make_grid_const(const upsample_grid_info& gi);
StepConst make_step_const(const upsample_params& p, bool has_rigid);
WallTable make_wall_table(const float* walls, int n_walls);

// a7: adjoint step.
struct AdjointArgs {
  GridConst gc;
  StepConst sc;
  const LRPoint* lr;
  const uint32_t* cell_start;
  const float* hx;
  const float* hv;
  const float* gx_out;
  const float* gv_out;
  float* gx_in;
  float* gv_in;
  float* g_lr_x;
  float* g_lr_v;
  // [6][n_lr] LR gradients by sorted index (dL/dV, then dL/dX), zero between
  // calls: the tiled kernel's block flush adds here, where the slots of one
  // row are consecutive addresses; launch_adjoint then adds it into g_lr_v /
  // g_lr_x by original index and zeroes it again
  float* g_sorted;
  int64_t n;
  int64_t n_lr;
  int tiled;     // 1: wave-tiled kernel (non-rigid scenes), 0: one particle per lane
  int tile_max;  // a spread-out wave streaming more LR candidates than this walks per lane
  const float* tape;  // forward record [6][n] (skips the recomputation of the sums) or null
  // deterministic LR gradients (all null otherwise): per HR particle its
  // adjoint coefficients [7][n] (dL/dU, dL/dS, dL/dM, argmax bits; row 6:
  // dL/dM by sorted slot), and the HR particles sorted by the same cells
  float* det_coef;
  const uint32_t* hr_cell_start;  // set by launch_adjoint from hr_grid
  const LRPoint* hr_sorted;
};
// With a.det_coef set (and hr_grid, scratch for max_hr particles over the
// same cells): the HR pass writes the coefficients instead of adding LR
// gradients, the HR grid is built into *hr_grid, and one wave per LR particle
// sums its HR neighbours' terms in a fixed order (no atomics).
hipError_t launch_adjoint(const AdjointArgs& a, const WallTable& walls, hipStream_t st,
                          const GridScratch* hr_grid = nullptr);

// VALIDATE flag: sets *flag to 1 if any of the n floats is NaN or Inf.
hipError_t launch_check_finite(const float* p, int64_t n, uint32_t* flag, hipStream_t st);
// perm_io[i] <- perm_io[p[i]] through tmp (n entries of scratch).
hipError_t launch_compose_perm(int32_t* perm_io, const int32_t* p, int64_t n, uint32_t* tmp, hipStream_t st);
hipError_t launch_permute(const float* a, const float* b, float* ao, float* bo, int64_t n, const int32_t* perm,
                          int scatter, uint32_t* bad, hipStream_t st);

}  // namespace ups
