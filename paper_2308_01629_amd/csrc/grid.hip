// Uniform-grid rebuild of the LR guide particles: the neighbour search the
// paper runs with a compact-hashing library (Section 5.1), as five streaming
// kernels over structure-of-arrays input:
//
//   k_keys_count  cell key per LR particle, per-cell counts by atomic add
//                 (the returned old count is the particle's arrival slot)
//   k_scan_chunks exclusive scan of the counts in 2048-cell chunks (counts are
//   k_scan_totals re-zeroed), then one block scans the chunk totals (grids
//                 of at most 256 chunks skip it: every scatter block scans them)
//   k_scatter     cell_start[] and an arrival-order placement per cell
//   k_stable      rank inside the cell by original index (stable order), then
//                 writes perm[] and the LR copy in sorted order (32 B / particle)
//
// The same key / count / scan machinery reorders HR particles by cell.
#include <algorithm>

#include "kernels.hpp"

namespace ups {
namespace {

// An LR frame at the HR time level: frame a, or with a second frame b the
// linear interpolation a + theta (b - a) in time, each operation rounded
// separately (the boundary's float32 arithmetic; the key and the sorted copy
// compute it identically).
struct FramePair {
  const float* x0;
  const float* v0;
  const float* x1;  // null: the frame is x0, v0 itself
  const float* v1;
  float theta;
};
__device__ __forceinline__ float frame_at(const float* a, const float* b, float theta, int64_t k) {
  if (b == nullptr) return a[k];
  const float a0 = a[k];
  const float d = b[k] - a0;
  const float p = theta * d;
  return a0 + p;
}

__global__ __launch_bounds__(kBlock) void k_keys_count(GridConst gc, FramePair f,
                                                       int64_t n, uint32_t* __restrict__ keys,
                                                       uint32_t* __restrict__ slot,
                                                       uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const uint32_t k = valid ? cell_key(gc, frame_at(f.x0, f.x1, f.theta, i), frame_at(f.x0, f.x1, f.theta, n + i),
                                      frame_at(f.x0, f.x1, f.theta, 2 * n + i))
                           : 0u;
  const uint32_t sl = claim_slot(k, valid, counts);
  if (valid) {
    keys[i] = k;
    slot[i] = sl;
  }
}

// Inclusive wave64 scan with ds_swizzle-free shuffles.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread; *total receives the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    uint32_t s = wsum[w];
    off += (w < wid) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Scan of the counts, first step: each block scans one 2048-bin chunk (eight
// consecutive bins per thread, two 16-byte loads where the chunk is whole),
// writes the chunk-local exclusive offsets, zeroes the counts for the next
// build and publishes the chunk total.  The chunk totals are scanned by the
// next launch; the kernel boundary orders the two, so no block waits on
// another and no device-scope fence is needed.
__global__ __launch_bounds__(kBlock) void k_scan_chunks(uint32_t* __restrict__ counts, int64_t n_cells,
                                                        uint32_t* __restrict__ local,
                                                        uint32_t* __restrict__ chunk_sum) {
  static_assert(kScanItems == 8, "two 16-byte loads per thread");
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  const bool whole = base + kScanItems <= n_cells;
  if (whole) {
    uint4* c4 = reinterpret_cast<uint4*>(counts + base);
    const uint4 lo = c4[0], hi = c4[1];
    v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
    v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
    c4[0] = make_uint4(0u, 0u, 0u, 0u);  // ready for the next build
    c4[1] = make_uint4(0u, 0u, 0u, 0u);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t c = base + k;
      v[k] = 0u;
      if (c < n_cells) {
        v[k] = counts[c];
        counts[c] = 0u;
      }
    }
  }
  uint32_t ex[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    ex[k] = sum;
    sum += v[k];
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan(sum, &total);
  if (whole) {
    uint4* l4 = reinterpret_cast<uint4*>(local + base);
    l4[0] = make_uint4(ex[0] + off, ex[1] + off, ex[2] + off, ex[3] + off);
    l4[1] = make_uint4(ex[4] + off, ex[5] + off, ex[6] + off, ex[7] + off);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t c = base + k;
      if (c < n_cells) local[c] = ex[k] + off;
    }
  }
  if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

// Second step, one block: exclusive scan of the chunk totals in tiles of
// kBlock; chunk_sum[n_chunks] receives the grand total.
__global__ __launch_bounds__(kBlock) void k_scan_totals(uint32_t* __restrict__ chunk_sum, int n_chunks) {
  uint32_t carry = 0;
  for (int b0 = 0; b0 < n_chunks; b0 += kBlock) {
    const int b = b0 + (int)threadIdx.x;
    const uint32_t v = b < n_chunks ? chunk_sum[b] : 0u;
    uint32_t tile;
    const uint32_t e = block_exclusive_scan(v, &tile);
    if (b < n_chunks) chunk_sum[b] = carry + e;
    carry += tile;
  }
  if (threadIdx.x == 0) chunk_sum[n_chunks] = carry;
}

__device__ __forceinline__ uint32_t cell_offset(const uint32_t* local, const uint32_t* chunk_sum,
                                                uint32_t k) {
  return local[k] + chunk_sum[k / (uint32_t)kScanChunk];
}

// SCAN_TOTALS: chunk_sum holds the chunks' raw totals (at most kBlock
// chunks), and every block scans them in LDS itself, which saves the
// one-block launch over the totals on small grids.
template <bool SCAN_TOTALS>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ slot, int64_t n,
                                                    const uint32_t* __restrict__ local,
                                                    const uint32_t* __restrict__ chunk_sum,
                                                    int64_t n_cells, int n_chunks,
                                                    uint32_t* __restrict__ tmp,
                                                    uint32_t* __restrict__ cell_start) {
  __shared__ uint32_t offs[SCAN_TOTALS ? kBlock + 1 : 1];
  const uint32_t* csum = chunk_sum;
  if (SCAN_TOTALS) {
    const uint32_t v = (int)threadIdx.x < n_chunks ? chunk_sum[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t e = block_exclusive_scan(v, &total);
    offs[threadIdx.x] = e;
    if (threadIdx.x == 0) offs[n_chunks] = total;
    __syncthreads();
    csum = offs;
  }
  int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n_cells) cell_start[t] = cell_offset(local, csum, (uint32_t)t);
  if (t == n_cells) cell_start[t] = csum[n_chunks];
  if (t < n) {
    const uint32_t pos = cell_offset(local, csum, keys[t]) + slot[t];
    if (pos < (uint64_t)n) tmp[pos] = (uint32_t)t;  // always true when counts started at zero
  }
}

// The scatter of a build over positions alone that writes the sorted copy
// itself: position, the caller's int32 tag (as bits) in p.w, the particle's
// index in v.w.  Inside a cell the particles keep the order of their slot
// claims, which varies from run to run; a caller of this grid build makes its
// results independent of that order.
template <bool SCAN_TOTALS>
__global__ __launch_bounds__(kBlock) void k_scatter_points(const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ slot, int64_t n,
                                                           const uint32_t* __restrict__ local,
                                                           const uint32_t* __restrict__ chunk_sum,
                                                           int64_t n_cells, int n_chunks,
                                                           const float* __restrict__ x,
                                                           const int32_t* __restrict__ tag,
                                                           LRPoint* __restrict__ out,
                                                           uint32_t* __restrict__ cell_start) {
  __shared__ uint32_t offs[SCAN_TOTALS ? kBlock + 1 : 1];
  const uint32_t* csum = chunk_sum;
  if (SCAN_TOTALS) {
    const uint32_t v = (int)threadIdx.x < n_chunks ? chunk_sum[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t e = block_exclusive_scan(v, &total);
    offs[threadIdx.x] = e;
    if (threadIdx.x == 0) offs[n_chunks] = total;
    __syncthreads();
    csum = offs;
  }
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n_cells) cell_start[t] = cell_offset(local, csum, (uint32_t)t);
  if (t == n_cells) cell_start[t] = csum[n_chunks];
  if (t < n) {
    const uint32_t pos = cell_offset(local, csum, keys[t]) + slot[t];
    if (pos < (uint64_t)n) {  // always true when counts started at zero
      LRPoint o;
      o.p = make_float4(x[t], x[n + t], x[2 * n + t], tag != nullptr ? __int_as_float(tag[t]) : 0.0f);
      o.v = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float((uint32_t)t));
      out[pos] = o;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_stable(const uint32_t* __restrict__ tmp,
                                                   const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ cell_start, int64_t n,
                                                   FramePair f,
                                                   const uint8_t* __restrict__ rigid,
                                                   uint32_t* __restrict__ perm,
                                                   LRPoint* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const uint32_t i = tmp[p];
  if (i >= (uint64_t)n) return;  // defensive: tmp is a permutation of [0, n)
  const uint32_t k = keys[i];
  const uint32_t b = cell_start[k], e = cell_start[k + 1];
  if (e > (uint64_t)n || b > e) return;
  uint32_t rank = 0;
  // independent loads: unrolled, several are in flight at once (HR cells of
  // the deterministic backward hold hundreds of particles)
#pragma unroll 16
  for (uint32_t q = b; q < e; ++q) rank += (tmp[q] < i) ? 1u : 0u;
  const uint32_t dst = b + rank;
  if (dst >= e) return;
  perm[dst] = i;
  const float flag = (rigid != nullptr && rigid[i] != 0) ? 1.0f : 0.0f;
  LRPoint o;
  o.p = make_float4(frame_at(f.x0, f.x1, f.theta, i), frame_at(f.x0, f.x1, f.theta, n + i),
                    frame_at(f.x0, f.x1, f.theta, 2 * n + i), flag);
  o.v = make_float4(frame_at(f.v0, f.v1, f.theta, i), frame_at(f.v0, f.v1, f.theta, n + i),
                    frame_at(f.v0, f.v1, f.theta, 2 * n + i), __uint_as_float(i));
  out[dst] = o;
}

// HR reorder: scatter (x, v) by cell into scratch, remember the old index.
// One block per block of k_hr_keys_count: it stages that block's particles in
// LDS with coalesced reads, then walks its (key, slot, source) entries in their
// block-local order, so that consecutive threads write consecutive
// destinations of one bin.
constexpr int kHrItems = 4;
constexpr int kHrSpan = kHrItems * kBlock;  // particles per block of the HR reorder

// Blocks are dispatched to the 8 XCDs round robin (block p on XCD p mod 8).
// Renumber them so that XCD x runs a contiguous range of logical blocks: the
// bin segments that neighbouring blocks share at their edges then meet in one
// L2 instead of being written back in part from two.  A bijection on
// [0, gridDim.x) for any grid size.
constexpr uint32_t kXcdCount = 8;
__device__ __forceinline__ uint32_t xcd_contiguous_block() {
  const uint32_t p = blockIdx.x, nb = gridDim.x;
  const uint32_t x = p % kXcdCount, base = nb / kXcdCount, rem = nb % kXcdCount;
  return x * base + min(x, rem) + p / kXcdCount;
}
// SCAN_TOTALS: chunk_sum holds the chunks' raw totals (n_chunks <= kBlock),
// and every block scans them in LDS itself (no one-block launch over them).
template <bool SCAN_TOTALS>
__global__ __launch_bounds__(kBlock) void k_hr_scatter(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ slot,
                                                       const uint32_t* __restrict__ src, int64_t n,
                                                       const uint32_t* __restrict__ local,
                                                       const uint32_t* __restrict__ chunk_sum, int n_chunks,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ v, int64_t ld,
                                                       float* __restrict__ xs, float* __restrict__ vs,
                                                       int32_t* __restrict__ perm) {
  __shared__ float stage[6][kHrSpan];
  __shared__ uint32_t offs[SCAN_TOTALS ? kBlock : 1];
  const uint32_t* csum = chunk_sum;
  if (SCAN_TOTALS) {
    const uint32_t t = (int)threadIdx.x < n_chunks ? chunk_sum[threadIdx.x] : 0u;
    uint32_t total;
    offs[threadIdx.x] = block_exclusive_scan(t, &total);
    csum = offs;  // read after the barrier that follows the staging below
  }
  const int64_t block0 = (int64_t)xcd_contiguous_block() * kHrSpan;
#pragma unroll
  for (int j = 0; j < kHrItems; ++j) {
    const int l = j * kBlock + threadIdx.x;
    const int64_t i = block0 + l;
    if (i < n) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        stage[a][l] = x[a * ld + i];
        stage[3 + a][l] = v[a * ld + i];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kHrItems; ++j) {
    const int64_t q = block0 + j * kBlock + threadIdx.x;
    if (q >= n) continue;
    const uint32_t i = src[q];
    const uint32_t l = (uint32_t)((int64_t)i - block0);
    const uint32_t dst = cell_offset(local, csum, keys[q]) + slot[q];
    // defensive: counts started at zero, sources stay inside the block
    if (dst >= (uint64_t)n || i >= (uint64_t)n || l >= (uint32_t)kHrSpan) continue;
    if (perm != nullptr) perm[dst] = (int32_t)i;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xs[a * n + dst] = stage[a][l];
      vs[a * n + dst] = stage[3 + a][l];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_back(const float* __restrict__ xs,
                                                      const float* __restrict__ vs,
                                                      const int32_t* __restrict__ perm, int64_t n,
                                                      float* __restrict__ x, float* __restrict__ v, int64_t ld,
                                                      int32_t* __restrict__ perm_out, int32_t perm_base) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a * ld + i] = xs[a * n + i];
    v[a * ld + i] = vs[a * n + i];
  }
  if (perm_out != nullptr) perm_out[i] = perm[i] + perm_base;
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const float* __restrict__ p, int64_t n,
                                                         uint32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && !isfinite(p[i])) atomicOr(flag, 1u);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Fine coordinate of one axis: cell * sub + sub-cell index, from the same
// float32 arithmetic as the cell coordinate.
__device__ __forceinline__ uint32_t fine_coord(float x, float lo, float inv_cs, int G, int sub) {
  const float t = (x - lo) * inv_cs;
  const float c = fminf(fmaxf(floorf(t), 0.0f), (float)(G - 1));
  const float f = fminf(fmaxf(floorf((t - c) * (float)sub), 0.0f), (float)(sub - 1));
  return (uint32_t)c * (uint32_t)sub + (uint32_t)f;
}

// Morton (Z-order) code of fine coordinates with bx, by, bz significant bits
// per axis: bit b of each axis that has one, x first, low bits first.
__device__ __forceinline__ uint32_t morton3(uint32_t fx, uint32_t fy, uint32_t fz, int bx, int by, int bz) {
  uint32_t key = 0u;
  int pos = 0;
  const int bmax = max(bx, max(by, bz));
  for (int b = 0; b < bmax; ++b) {
    if (b < bx) key |= ((fx >> b) & 1u) << pos++;
    if (b < by) key |= ((fy >> b) & 1u) << pos++;
    if (b < bz) key |= ((fz >> b) & 1u) << pos++;
  }
  return key;
}

__device__ __forceinline__ uint32_t morton_sub(uint32_t a, uint32_t b, uint32_t c) {
  return (a & 1u) | ((b & 1u) << 1) | ((c & 1u) << 2) | ((a & 2u) << 2) | ((b & 2u) << 3) | ((c & 2u) << 4);
}

// HR reorder keys and slots, with the bin claims aggregated over blocks of
// kHrItems * kBlock consecutive particles.  Each wave first joins runs of equal
// keys (as claim_slot does); the first lane of each run then enters the key in
// an LDS hash table of the block's distinct keys and adds the run length to
// that entry.  One global atomic add per distinct key then claims the block's
// slots of that bin, so a bin receives one atomic per block instead of one per
// wave run.  The block writes (key, slot, source index) in block-local order:
// the particles of one key together, in slot order, so that consecutive
// threads of the scatter write consecutive destinations.  Keys are below 2^24,
// so all-ones marks an empty entry.  The table holds twice the block's particle
// count: a linear probe meets its key or an empty entry within one sweep, and
// the global-atomic path for a run that finds neither is never taken.
constexpr int kHrTableBits = 11;
constexpr int kHrTable = 1 << kHrTableBits;
constexpr int kHrPerThread = kHrTable / kBlock;
static_assert(kHrTable >= 2 * kHrSpan, "HR key table must stay at most half full");
static_assert(kHrTable % kBlock == 0, "HR key table entries per thread");
constexpr uint32_t kNoKey = 0xffffffffu;

// The reorder key of HR particle i of one scene: mode 2 the Hilbert index of
// its fine cell, mode 1 the Z-order code, mode 0 the grid cell then the
// Z-order of its sub-cells.
struct SceneHrKey {
  GridConst gc;
  const float* x;
  int64_t ld;
  int sub, mode, bx, by, bz;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    const uint32_t fx = fine_coord(x[i], gc.lo[0], gc.inv_cs, gc.dims[0], sub);
    const uint32_t fy = fine_coord(x[ld + i], gc.lo[1], gc.inv_cs, gc.dims[1], sub);
    const uint32_t fz = fine_coord(x[2 * ld + i], gc.lo[2], gc.inv_cs, gc.dims[2], sub);
    if (mode == 2) return hilbert3(fx, fy, fz, max(bx, max(by, bz)));
    if (mode == 1) return morton3(fx, fy, fz, bx, by, bz);
    // sub is 1, 2 or 4: divide and take remainders by shifts
    const uint32_t sh = (uint32_t)(__ffs(sub) - 1), m = (uint32_t)sub - 1u;
    const uint32_t cell = (fx >> sh) + (uint32_t)gc.dims[0] * ((fy >> sh) + (uint32_t)gc.dims[1] * (fz >> sh));
    return (cell << (3u * sh)) + morton_sub(fx & m, fy & m, fz & m);
  }
};

// The reorder key of HR particle i of one scene by rank table: the Hilbert
// rank of its fine cell among the grid's fine cells (the order of mode 2 on
// F bins instead of a padded 2^(3b) cube).
struct RankHrKey {
  GridConst gc;
  const float* x;
  int64_t ld;
  int sub;
  int fdims[3];
  const uint32_t* rank;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    const uint32_t fx = fine_coord(x[i], gc.lo[0], gc.inv_cs, gc.dims[0], sub);
    const uint32_t fy = fine_coord(x[ld + i], gc.lo[1], gc.inv_cs, gc.dims[1], sub);
    const uint32_t fz = fine_coord(x[2 * ld + i], gc.lo[2], gc.inv_cs, gc.dims[2], sub);
    return rank[fx + (uint32_t)fdims[0] * (fy + (uint32_t)fdims[1] * fz)];
  }
};

// The key of column i of a batch whose scenes own consecutive column ranges
// (start[s] .. start[s + 1]): the scene's first bin plus the Hilbert rank of
// the particle's fine cell among all fine cells of that scene's grid, so the
// bins of all scenes together number their fine cells, not padded cubes.
struct BatchHrKey {
  const float* x;
  int64_t ld;
  const int64_t* start;
  int n_scenes;
  const HrRankScene* sc;
  const uint32_t* rank;
  __device__ __forceinline__ uint32_t operator()(int64_t i) const {
    int lo = 0, hi = n_scenes;  // the scene s with start[s] <= i < start[s + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (start[mid] <= i) lo = mid; else hi = mid;
    }
    const HrRankScene& d = sc[lo];
    const uint32_t fx = fine_coord(x[i], d.gc.lo[0], d.gc.inv_cs, d.gc.dims[0], d.sub);
    const uint32_t fy = fine_coord(x[ld + i], d.gc.lo[1], d.gc.inv_cs, d.gc.dims[1], d.sub);
    const uint32_t fz = fine_coord(x[2 * ld + i], d.gc.lo[2], d.gc.inv_cs, d.gc.dims[2], d.sub);
    const uint32_t f = fx + (uint32_t)d.fdims[0] * (fy + (uint32_t)d.fdims[1] * fz);
    return d.base + rank[d.base + f];
  }
};

template <class KeyFn>
__global__ __launch_bounds__(kBlock) void k_hr_keys_count(KeyFn kf, int64_t n,
                                                          uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ slot,
                                                          uint32_t* __restrict__ src,
                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t tkey[kHrTable];  // key of the entry, then its first block-local position
  __shared__ uint32_t tval[kHrTable];  // particle count of the entry, then its first slot
  __shared__ uint32_t n_direct;        // particles whose run claimed its slots directly
  for (int t = threadIdx.x; t < kHrTable; t += kBlock) {
    tkey[t] = kNoKey;
    tval[t] = 0u;
  }
  if (threadIdx.x == 0) n_direct = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t block0 = (int64_t)xcd_contiguous_block() * kHrSpan;
  uint32_t key[kHrItems], rank[kHrItems], drank[kHrItems];
  int ent[kHrItems];
#pragma unroll
  for (int j = 0; j < kHrItems; ++j) {
    const int64_t i = block0 + (int64_t)j * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int64_t ii = valid ? i : 0;
    const uint32_t k = kf(ii);
    const uint32_t kk = valid ? k : kNoKey;
    const uint32_t prev = __shfl_up(kk, 1, 64);
    const bool head = (lane == 0) || (prev != kk);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int start = 63 - __clzll(heads & upto);
    const uint64_t above = heads & ~upto;
    const int next = above ? (__ffsll((long long)above) - 1) : 64;
    int e = -1;
    uint32_t r = 0u, dr = 0u;
    if (head && valid) {
      const uint32_t len = (uint32_t)(next - lane);
      uint32_t h = (kk * 2654435761u) >> (32 - kHrTableBits);
      for (int probe = 0; probe < kHrTable; ++probe) {
        const uint32_t old = atomicCAS(&tkey[h], kNoKey, kk);
        if (old == kNoKey || old == kk) {
          e = (int)h;
          break;
        }
        h = (h + 1u) & (uint32_t)(kHrTable - 1);
      }
      if (e >= 0) {
        r = atomicAdd(&tval[e], len);
      } else {
        r = atomicAdd(&counts[kk], len);
        dr = atomicAdd(&n_direct, len);
      }
    }
    const uint32_t off = (uint32_t)(lane - start);
    ent[j] = __shfl(e, start, 64);
    rank[j] = __shfl(r, start, 64) + off;
    drank[j] = __shfl(dr, start, 64) + off;
    key[j] = kk;
  }
  __syncthreads();
  // claim each key's slots, and lay the entries out one after another: thread
  // t owns entries t, t + kBlock, ... and places them consecutively
  uint32_t cnt[kHrPerThread], sum = 0u;
#pragma unroll
  for (int q = 0; q < kHrPerThread; ++q) {
    const int t = q * kBlock + threadIdx.x;
    const uint32_t k = tkey[t];
    cnt[q] = tval[t];
    if (k != kNoKey) tval[t] = atomicAdd(&counts[k], cnt[q]);
    sum += cnt[q];
  }
  uint32_t in_table = 0u;
  uint32_t pos = block_exclusive_scan(sum, &in_table);
#pragma unroll
  for (int q = 0; q < kHrPerThread; ++q) {
    tkey[q * kBlock + threadIdx.x] = pos;
    pos += cnt[q];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kHrItems; ++j) {
    const int64_t i = block0 + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) {
      const bool tab = ent[j] >= 0;
      const int e = tab ? ent[j] : 0;
      const int64_t dst = block0 + (tab ? (int64_t)tkey[e] + rank[j] : (int64_t)in_table + drank[j]);
      keys[dst] = key[j];
      slot[dst] = tab ? tval[e] + rank[j] : rank[j];
      src[dst] = (uint32_t)i;
    }
  }
}

// Batched grid: keys of every scene's LR particles, offset by the scene's
// first global cell; the internal index of a particle is its scene's first
// internal index plus its index inside the scene.
__global__ __launch_bounds__(kBlock) void k_keys_count_batched(BatchGridArgs b, uint32_t* __restrict__ keys,
                                                               uint32_t* __restrict__ slot,
                                                               uint32_t* __restrict__ counts) {
  const BatchTile blk = b.lr_blocks[blockIdx.x];
  const BatchScene& sc = b.scenes[blk.scene];
  const int64_t e = (int64_t)blk.first + threadIdx.x;
  const bool valid = e < sc.n_lr;
  uint32_t k = 0u;
  if (valid) {
    const int64_t src = sc.lr_off + e;
    k = sc.cell_base + cell_key(sc.gc, b.lr_x[src], b.lr_x[b.ld + src], b.lr_x[2 * b.ld + src]);
  }
  const uint32_t sl = claim_slot(k, valid, counts);
  if (valid) {
    const int64_t q = sc.lr_int + e;
    keys[q] = k;
    slot[q] = sl;
    b.scene_of[q] = (uint16_t)blk.scene;
  }
}

// Stable rank inside the cell and the sorted LR copy, as k_stable; the id
// bits hold the particle's index inside its scene.
__global__ __launch_bounds__(kBlock) void k_stable_batched(const uint32_t* __restrict__ tmp,
                                                           const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ cell_start,
                                                           BatchGridArgs b, uint32_t* __restrict__ perm,
                                                           LRPoint* __restrict__ out) {
  const int64_t n = b.n_int;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const uint32_t i = tmp[p];
  if (i >= (uint64_t)n) return;  // defensive: tmp is a permutation of [0, n)
  const uint32_t k = keys[i];
  const uint32_t c0 = cell_start[k], c1 = cell_start[k + 1];
  if (c1 > (uint64_t)n || c0 > c1) return;
  uint32_t rank = 0;
  for (uint32_t q = c0; q < c1; ++q) rank += (tmp[q] < i) ? 1u : 0u;
  const uint32_t dst = c0 + rank;
  if (dst >= c1) return;
  perm[dst] = i;
  const BatchScene& sc = b.scenes[b.scene_of[i]];
  const int64_t local = (int64_t)i - sc.lr_int;
  const int64_t src = sc.lr_off + local;
  const float flag = (b.lr_rigid != nullptr && b.lr_rigid[src] != 0) ? 1.0f : 0.0f;
  LRPoint o;
  o.p = make_float4(b.lr_x[src], b.lr_x[b.ld + src], b.lr_x[2 * b.ld + src], flag);
  o.v = make_float4(b.lr_v[src], b.lr_v[b.ld + src], b.lr_v[2 * b.ld + src], __uint_as_float((uint32_t)local));
  out[dst] = o;
}

hipError_t scan_bins(uint32_t* counts, int64_t n_bins, uint32_t* local, uint32_t* chunk_sum, hipStream_t st) {
  const int n_chunks = (int)((n_bins + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(k_scan_chunks, dim3(n_chunks), dim3(kBlock), 0, st, counts, n_bins, local, chunk_sum);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, st, chunk_sum, n_chunks);
  return hipGetLastError();
}

}  // namespace

static hipError_t build_grid(const GridConst& gc, const FramePair& f, const uint8_t* lr_rigid, int64_t n_lr,
                             int64_t n_cells, const GridScratch& s, hipStream_t st) {
  if (n_lr > 0) {
    hipLaunchKernelGGL(k_keys_count, dim3(blocks_for(n_lr)), dim3(kBlock), 0, st, gc, f, n_lr,
                       s.keys, s.slot, s.counts);
  }
  int n_chunks = (int)((n_cells + kScanChunk - 1) / kScanChunk);
  int64_t span = n_lr > n_cells + 1 ? n_lr : n_cells + 1;
  if (n_chunks <= kBlock) {
    // small grid: the chunk scan, then the scatter scans the chunk totals itself
    hipLaunchKernelGGL(k_scan_chunks, dim3(n_chunks), dim3(kBlock), 0, st, s.counts, n_cells, s.local,
                       s.chunk_sum);
    hipLaunchKernelGGL(k_scatter<true>, dim3(blocks_for(span)), dim3(kBlock), 0, st, s.keys, s.slot, n_lr,
                       s.local, s.chunk_sum, n_cells, n_chunks, s.tmp, s.cell_start);
  } else {
    hipError_t e = scan_bins(s.counts, n_cells, s.local, s.chunk_sum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter<false>, dim3(blocks_for(span)), dim3(kBlock), 0, st, s.keys, s.slot, n_lr,
                       s.local, s.chunk_sum, n_cells, n_chunks, s.tmp, s.cell_start);
  }
  if (n_lr > 0) {
    hipLaunchKernelGGL(k_stable, dim3(blocks_for(n_lr)), dim3(kBlock), 0, st, s.tmp, s.keys,
                       s.cell_start, n_lr, f, lr_rigid, s.perm, s.lr_sorted);
  }
  return hipGetLastError();
}

hipError_t launch_build_grid(const GridConst& gc, const float* lr_x, const float* lr_v,
                             const uint8_t* lr_rigid, int64_t n_lr, int64_t n_cells,
                             const GridScratch& s, hipStream_t st) {
  return build_grid(gc, FramePair{lr_x, lr_v, nullptr, nullptr, 0.0f}, lr_rigid, n_lr, n_cells, s, st);
}

hipError_t launch_build_grid_points(const GridConst& gc, const float* x, const int32_t* tag, int64_t n,
                                    int64_t n_cells, const GridScratch& s, hipStream_t st, bool keys_ready) {
  if (n > 0 && !keys_ready)
    hipLaunchKernelGGL(k_keys_count, dim3(blocks_for(n)), dim3(kBlock), 0, st, gc,
                       FramePair{x, x, nullptr, nullptr, 0.0f}, n, s.keys, s.slot, s.counts);
  const int n_chunks = (int)((n_cells + kScanChunk - 1) / kScanChunk);
  const int64_t span = n > n_cells + 1 ? n : n_cells + 1;
  if (n_chunks <= kBlock) {
    hipLaunchKernelGGL(k_scan_chunks, dim3(n_chunks), dim3(kBlock), 0, st, s.counts, n_cells, s.local,
                       s.chunk_sum);
    hipLaunchKernelGGL(k_scatter_points<true>, dim3(blocks_for(span)), dim3(kBlock), 0, st, s.keys, s.slot, n,
                       s.local, s.chunk_sum, n_cells, n_chunks, x, tag, s.lr_sorted, s.cell_start);
  } else {
    const hipError_t e = scan_bins(s.counts, n_cells, s.local, s.chunk_sum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_points<false>, dim3(blocks_for(span)), dim3(kBlock), 0, st, s.keys, s.slot, n,
                       s.local, s.chunk_sum, n_cells, n_chunks, x, tag, s.lr_sorted, s.cell_start);
  }
  return hipGetLastError();
}

// The sorted LR copy as structure-of-arrays [3][n] (debug export).
__global__ __launch_bounds__(kBlock) void k_unpack_sorted(const LRPoint* __restrict__ lr, int64_t n,
                                                          float* __restrict__ x, float* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const LRPoint q = lr[j];
  if (x != nullptr) {
    x[j] = q.p.x;
    x[n + j] = q.p.y;
    x[2 * n + j] = q.p.z;
  }
  if (v != nullptr) {
    v[j] = q.v.x;
    v[n + j] = q.v.y;
    v[2 * n + j] = q.v.z;
  }
}

hipError_t launch_unpack_sorted(const LRPoint* lr, int64_t n, float* x, float* v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_unpack_sorted, dim3(blocks_for(n)), dim3(kBlock), 0, st, lr, n, x, v);
  return hipGetLastError();
}

hipError_t launch_scan_bins(uint32_t* counts, int64_t n_bins, uint32_t* local, uint32_t* chunk_sum,
                            hipStream_t st) {
  return scan_bins(counts, n_bins, local, chunk_sum, st);
}

hipError_t launch_build_grid_lerp(const GridConst& gc, const float* x0, const float* v0, const float* x1,
                                  const float* v1, float theta, const uint8_t* lr_rigid, int64_t n_lr,
                                  int64_t n_cells, const GridScratch& s, hipStream_t st) {
  return build_grid(gc, FramePair{x0, v0, x1, v1, theta}, lr_rigid, n_lr, n_cells, s, st);
}

hipError_t launch_build_grid_batched(const BatchGridArgs& b, const GridScratch& s, hipStream_t st) {
  if (b.n_lr_blocks > 0) {
    hipLaunchKernelGGL(k_keys_count_batched, dim3((unsigned)b.n_lr_blocks), dim3(kBlock), 0, st, b, s.keys,
                       s.slot, s.counts);
  }
  hipError_t e = scan_bins(s.counts, b.n_cells, s.local, s.chunk_sum, st);
  if (e != hipSuccess) return e;
  const int n_chunks = (int)((b.n_cells + kScanChunk - 1) / kScanChunk);
  const int64_t span = b.n_int > b.n_cells + 1 ? b.n_int : b.n_cells + 1;
  hipLaunchKernelGGL(k_scatter<false>, dim3(blocks_for(span)), dim3(kBlock), 0, st, s.keys, s.slot, b.n_int, s.local,
                     s.chunk_sum, b.n_cells, n_chunks, s.tmp, s.cell_start);
  if (b.n_int > 0) {
    hipLaunchKernelGGL(k_stable_batched, dim3(blocks_for(b.n_int)), dim3(kBlock), 0, st, s.tmp, s.keys,
                       s.cell_start, b, s.perm, s.lr_sorted);
  }
  return hipGetLastError();
}

// The scan of the HR reorder's bins and the scatter: with at most kBlock
// scan chunks the scatter's blocks scan the chunk totals themselves.
static hipError_t launch_hr_scatter(const HRSortScratch& s, int64_t n, int64_t n_bins, const float* x,
                                    const float* v, int64_t ld, float* xs, float* vs, int32_t* perm,
                                    hipStream_t st) {
  const int n_chunks = (int)((n_bins + kScanChunk - 1) / kScanChunk);
  const unsigned nb = (unsigned)((n + kHrSpan - 1) / kHrSpan);
  if (n_chunks <= kBlock) {
    hipLaunchKernelGGL(k_scan_chunks, dim3(n_chunks), dim3(kBlock), 0, st, s.counts, n_bins, s.local, s.chunk_sum);
    hipLaunchKernelGGL(k_hr_scatter<true>, dim3(nb), dim3(kBlock), 0, st, s.keys, s.slot, s.src, n, s.local,
                       s.chunk_sum, n_chunks, x, v, ld, xs, vs, perm);
  } else {
    const hipError_t e = scan_bins(s.counts, n_bins, s.local, s.chunk_sum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hr_scatter<false>, dim3(nb), dim3(kBlock), 0, st, s.keys, s.slot, s.src, n, s.local,
                       s.chunk_sum, n_chunks, x, v, ld, xs, vs, perm);
  }
  return hipGetLastError();
}

hipError_t launch_sort_hr(const GridConst& gc, const float* hr_x, const float* hr_v, float* out_x,
                          float* out_v, int64_t n_hr, int sub, int mode, const HRSortScratch& s,
                          int32_t* perm_out, hipStream_t st, int64_t ld, int32_t perm_base,
                          const uint32_t* rank) {
  if (n_hr == 0) return hipSuccess;
  if (ld < 0) ld = n_hr;
  // a strided state is sorted in place only (through the scratch copy)
  if (ld != n_hr && (out_x != hr_x || out_v != hr_v)) return hipErrorInvalidValue;
  int bits[3];
  for (int a = 0; a < 3; ++a) bits[a] = sort_bits((int64_t)gc.dims[a] * sub);
  int64_t n_bins = sort_bins(gc.dims, sub, mode);
  const unsigned nb = (unsigned)((n_hr + kHrSpan - 1) / kHrSpan);
  if (mode == 2 && rank != nullptr) {
    const RankHrKey kf{gc, hr_x, ld, sub, {gc.dims[0] * sub, gc.dims[1] * sub, gc.dims[2] * sub}, rank};
    n_bins = (int64_t)kf.fdims[0] * kf.fdims[1] * kf.fdims[2];
    hipLaunchKernelGGL(k_hr_keys_count<RankHrKey>, dim3(nb), dim3(kBlock), 0, st, kf, n_hr, s.keys, s.slot, s.src,
                       s.counts);
  } else {
    const SceneHrKey kf{gc, hr_x, ld, sub, mode, bits[0], bits[1], bits[2]};
    hipLaunchKernelGGL(k_hr_keys_count<SceneHrKey>, dim3(nb), dim3(kBlock), 0, st, kf, n_hr, s.keys, s.slot, s.src,
                       s.counts);
  }
  const bool in_place = out_x == hr_x || out_v == hr_v;
  // the old index of each new position is written only when it is asked for
  int32_t* perm = perm_out == nullptr ? nullptr : (in_place ? s.perm : perm_out);
  hipError_t e = launch_hr_scatter(s, n_hr, n_bins, hr_x, hr_v, ld, in_place ? s.x : out_x,
                                   in_place ? s.v : out_v, perm, st);
  if (e != hipSuccess) return e;
  if (in_place) {
    hipLaunchKernelGGL(k_copy_back, dim3(blocks_for(n_hr)), dim3(kBlock), 0, st, s.x, s.v, s.perm,
                       n_hr, out_x, out_v, ld, perm_out, perm_base);
  }
  return hipGetLastError();
}

// Hilbert ranks of one scene's fine cells: mark the Hilbert index of every
// fine cell of the box in a cube of 2^(3 bits) bins, scan, and give each fine
// cell the number of box cells before it along the curve.
__global__ __launch_bounds__(kBlock) void k_rank_mark(int fx, int fy, int fz, int bits, uint32_t* __restrict__ cube) {
  const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (f >= (int64_t)fx * fy * fz) return;
  const uint32_t x = (uint32_t)(f % fx), y = (uint32_t)((f / fx) % fy), z = (uint32_t)(f / ((int64_t)fx * fy));
  cube[hilbert3(x, y, z, bits)] = 1u;
}

__global__ __launch_bounds__(kBlock) void k_rank_fill(int fx, int fy, int fz, int bits,
                                                      const uint32_t* __restrict__ local,
                                                      const uint32_t* __restrict__ chunk_sum,
                                                      uint32_t* __restrict__ rank) {
  const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (f >= (int64_t)fx * fy * fz) return;
  const uint32_t x = (uint32_t)(f % fx), y = (uint32_t)((f / fx) % fy), z = (uint32_t)(f / ((int64_t)fx * fy));
  rank[f] = cell_offset(local, chunk_sum, hilbert3(x, y, z, bits));
}

hipError_t launch_hilbert_ranks(const int fdims[3], uint32_t* rank, uint32_t* cube, uint32_t* local,
                                uint32_t* chunk_sum, hipStream_t st) {
  int bits = 0;
  for (int a = 0; a < 3; ++a) bits = std::max(bits, sort_bits(fdims[a]));
  const int64_t F = (int64_t)fdims[0] * fdims[1] * fdims[2];
  const int64_t n_cube = (int64_t)1 << (3 * bits);
  if (F == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rank_mark, dim3(blocks_for(F)), dim3(kBlock), 0, st, fdims[0], fdims[1], fdims[2], bits, cube);
  hipError_t e = scan_bins(cube, n_cube, local, chunk_sum, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_fill, dim3(blocks_for(F)), dim3(kBlock), 0, st, fdims[0], fdims[1], fdims[2], bits,
                     local, chunk_sum, rank);
  return hipGetLastError();
}

hipError_t launch_sort_hr_batched(float* hr_x, float* hr_v, int64_t n, const int64_t* start,
                                  int n_scenes, const HrRankScene* sc, const uint32_t* rank, int64_t n_bins,
                                  const HRSortScratch& s, int32_t* perm_out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const BatchHrKey kf{hr_x, n, start, n_scenes, sc, rank};
  const unsigned nb = (unsigned)((n + kHrSpan - 1) / kHrSpan);
  hipLaunchKernelGGL(k_hr_keys_count<BatchHrKey>, dim3(nb), dim3(kBlock), 0, st, kf, n, s.keys, s.slot, s.src,
                     s.counts);
  const hipError_t e = launch_hr_scatter(s, n, n_bins, hr_x, hr_v, n, s.x, s.v,
                                         perm_out != nullptr ? s.perm : nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_back, dim3(blocks_for(n)), dim3(kBlock), 0, st, s.x, s.v, s.perm, n,
                     hr_x, hr_v, n, perm_out, 0);
  return hipGetLastError();
}

// Permute up to two [3][n] arrays: gather (dst[:, i] = src[:, perm[i]]) or
// scatter (dst[:, perm[i]] = src[:, i]); indices outside [0, n) are skipped
// and raise *bad.
template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_permute(const float* __restrict__ a, const float* __restrict__ b,
                                                    float* __restrict__ ao, float* __restrict__ bo, int64_t n,
                                                    const int32_t* __restrict__ perm, uint32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t p = perm[i];
  if (p < 0 || (int64_t)p >= n) {
    atomicOr(bad, 1u);
    return;
  }
  const int64_t src = SCATTER ? i : (int64_t)p;
  const int64_t dst = SCATTER ? (int64_t)p : i;
  for (int c = 0; c < 3; ++c) ao[c * n + dst] = a[c * n + src];
  if (b != nullptr)
    for (int c = 0; c < 3; ++c) bo[c * n + dst] = b[c * n + src];
}

hipError_t launch_permute(const float* a, const float* b, float* ao, float* bo, int64_t n, const int32_t* perm,
                          int scatter, uint32_t* bad, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (scatter)
    hipLaunchKernelGGL(k_permute<true>, dim3(blocks_for(n)), dim3(kBlock), 0, st, a, b, ao, bo, n, perm, bad);
  else
    hipLaunchKernelGGL(k_permute<false>, dim3(blocks_for(n)), dim3(kBlock), 0, st, a, b, ao, bo, n, perm, bad);
  return hipGetLastError();
}

// tmp[i] = perm_io[p[i]]: the original index of each position after a reorder
// whose permutation is p, given perm_io before it.
__global__ __launch_bounds__(kBlock) void k_compose_perm(const int32_t* __restrict__ perm_io,
                                                         const int32_t* __restrict__ p, int64_t n,
                                                         int32_t* __restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t q = p[i];
  if (q < 0 || (int64_t)q >= n) return;  // defensive: p is a permutation of [0, n)
  tmp[i] = perm_io[q];
}

hipError_t launch_compose_perm(int32_t* perm_io, const int32_t* p, int64_t n, uint32_t* tmp, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int32_t* t = reinterpret_cast<int32_t*>(tmp);
  hipLaunchKernelGGL(k_compose_perm, dim3(blocks_for(n)), dim3(kBlock), 0, st, perm_io, p, n, t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(perm_io, t, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
  return e;
}

hipError_t launch_check_finite(const float* p, int64_t n, uint32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n, flag);
  return hipGetLastError();
}

}  // namespace ups
