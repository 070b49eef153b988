// Randomized volume sampling of initial particle states (Section 4, the
// sampling paragraph): the bounding box is cut into cubic cells of side
// 2 r / sqrt(3) -- a cell's diagonal is 2 r, so two non-overlapping
// particles never share a cell -- random candidates inside the hull are
// assigned to their cells, and each cell takes one of its candidates that
// overlaps no position sampled before it.
//
// The paper leaves the order of the cells open.  Cells are taken here in 27
// colour phases, colour (cx mod 3) + 3 (cy mod 3) + 9 (cz mod 3): two cells
// of one colour differ by at least 3 in some axis, so their points are at
// least two sides (2.31 r) apart and cannot conflict.  Within a phase every
// cell chooses at once (one thread per cell), and the result is that of the
// sequential pass over the cells in (colour, key) order.  A conflict can only
// come from the 5 x 5 x 5 cells around a cell (2 r is 1.73 sides), and in
// phase k only from those of the k colours before it: cells of later colours
// are still empty, and the only cell of its own colour in the window is the
// cell itself.  Each phase therefore tests the offsets of earlier colours
// alone (none in the first phase, 62 on average), nearest first so that a
// candidate that conflicts is rejected early.
//
// Candidates go through the LR grid build over positions (keys, counting
// sort by cell; the order inside a cell is left as the slot claims give it,
// and each candidate carries its input index), so the whole routine is the
// grid machinery plus 27 launches of k_sample_phase and a compaction of the
// per-cell samples in key order.
#include <cmath>
#include <string>

#include "kernels.hpp"

namespace ups {
namespace {

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_zero_f4(float4* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The offsets one phase tests: (dx + 2) | (dy + 2) << 3 | (dz + 2) << 6.
struct PhaseOffsets {
  int n;
  uint32_t off[124];
};

// One colour phase: cells (a + 3 i, b + 3 j, c + 3 k).  A cell keeps, of its
// candidates whose separately rounded squared distance to every sample of
// the listed neighbour cells is >= d2 = fl(4 r^2), the one first in input
// order (the smallest index: whether a candidate fits does not depend on the
// cell's other candidates, so this is the sequential visit's choice).
__global__ __launch_bounds__(kBlock) void k_sample_phase(GridConst gc, const uint32_t* __restrict__ cell_start,
                                                         const LRPoint* __restrict__ cand, float4* __restrict__ smp,
                                                         int a, int b, int c, int ni, int nj, int nk, float d2,
                                                         PhaseOffsets po) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)ni * nj * nk) return;
  const int i = (int)(t % ni), j = (int)((t / ni) % nj), k = (int)(t / ((int64_t)ni * nj));
  const int cx = a + 3 * i, cy = b + 3 * j, cz = c + 3 * k;
  const int Gx = gc.dims[0], Gy = gc.dims[1], Gz = gc.dims[2];
  const uint32_t key = (uint32_t)cx + (uint32_t)Gx * ((uint32_t)cy + (uint32_t)Gy * (uint32_t)cz);
  const uint32_t e = cell_start[key + 1u];
  uint32_t best = 0xffffffffu;
  float4 pick = make_float4(0.f, 0.f, 0.f, 0.f);
  for (uint32_t q = cell_start[key]; q < e; ++q) {
    const LRPoint C = cand[q];
    const uint32_t idx = __float_as_uint(C.v.w);
    if (idx >= best) continue;  // an earlier candidate already fits
    const float4 P = C.p;
    bool ok = true;
    for (int o = 0; o < po.n; ++o) {
      const uint32_t w = po.off[o];
      const int x = cx + (int)(w & 7u) - 2, y = cy + (int)((w >> 3) & 7u) - 2, z = cz + (int)(w >> 6) - 2;
      if ((unsigned)x >= (unsigned)Gx || (unsigned)y >= (unsigned)Gy || (unsigned)z >= (unsigned)Gz) continue;
      const float4 S = smp[(uint32_t)x + (uint32_t)Gx * ((uint32_t)y + (uint32_t)Gy * (uint32_t)z)];
      if (S.w != 0.0f && sq_dist(P.x, P.y, P.z, S.x, S.y, S.z) < d2) {
        ok = false;
        break;
      }
    }
    if (ok) {
      best = idx;
      pick = make_float4(P.x, P.y, P.z, 1.0f);
    }
  }
  if (best != 0xffffffffu) smp[key] = pick;
}

// The neighbour offsets of phase (a, b, c) whose cells have an earlier
// colour, ordered by squared offset length.
PhaseOffsets phase_offsets(int a, int b, int c) {
  PhaseOffsets po{};
  const int col = a + 3 * b + 9 * c;
  for (int len = 1; len <= 12; ++len)
    for (int dz = -2; dz <= 2; ++dz)
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          if (dx * dx + dy * dy + dz * dz != len) continue;
          const int nc = (a + dx + 3) % 3 + 3 * ((b + dy + 3) % 3) + 9 * ((c + dz + 3) % 3);
          if (nc < col) po.off[po.n++] = (uint32_t)(dx + 2) | (uint32_t)(dy + 2) << 3 | (uint32_t)(dz + 2) << 6;
        }
  return po;
}

__global__ __launch_bounds__(kBlock) void k_sample_flags(const float4* __restrict__ smp, int64_t n,
                                                         uint32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) flags[i] = smp[i].w != 0.0f ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_sample_compact(const float4* __restrict__ smp, int64_t n,
                                                           const uint32_t* __restrict__ local,
                                                           const uint32_t* __restrict__ chunk_sum,
                                                           float* __restrict__ out, int64_t max_out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 S = smp[i];
  if (S.w == 0.0f) return;
  const int64_t pos = (int64_t)local[i] + chunk_sum[i / kScanChunk];
  if (pos >= max_out) return;
  out[pos] = S.x;
  out[max_out + pos] = S.y;
  out[2 * max_out + pos] = S.z;
}

template <typename T>
hipError_t alloc(T** p, int64_t n) {
  return hipMalloc((void**)p, (size_t)(n > 0 ? n : 1) * sizeof(T));
}

}  // namespace
}  // namespace ups

using namespace ups;

extern "C" int upsample_sample_volume(const float* cand, int64_t n_cand, float r, const float* lo,
                                      const float* hi, float* out, int64_t max_out, int64_t* n_out,
                                      void* stream) {
  if (n_out == nullptr || lo == nullptr || hi == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  *n_out = 0;
  if (n_cand < 0 || max_out < 0 || !(std::isfinite(r) && r > 0.0f)) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_cand >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_CAPACITY;
  if (n_cand > 0 && cand == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (max_out > 0 && out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  const double side = 2.0 * (double)r / std::sqrt(3.0);
  GridConst gc;
  int64_t n_cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (!(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] > lo[a])) return UPSAMPLE_ERR_INVALID_ARG;
    const double ext = ((double)hi[a] - (double)lo[a]) / side;
    if (!(ext < 1048576.0)) return UPSAMPLE_ERR_GRID_TOO_LARGE;
    int d = (int)std::ceil(ext);
    if (d < 1) d = 1;
    gc.dims[a] = d;
    gc.lo[a] = lo[a];
    n_cells *= d;
  }
  if (n_cells >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_GRID_TOO_LARGE;
  gc.inv_cs = (float)(1.0 / side);
  gc.cs = (float)side;
  gc.reach = 2;
  gc.h2 = (float)(4.0 * (double)r * (double)r);
  gc.inv_h2 = 0.0f;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UPSAMPLE_ERR_NO_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n_chunks = (n_cells + kScanChunk - 1) / kScanChunk;
  GridScratch g{};
  float4* smp = nullptr;
  uint32_t* flags = nullptr;
  uint32_t* local = nullptr;
  uint32_t* csum = nullptr;
  uint32_t* total_dev = nullptr;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n) \
  if (e == hipSuccess) e = alloc(&(ptr), (n));
  ALLOC(g.keys, n_cand)
  ALLOC(g.slot, n_cand)
  ALLOC(g.counts, n_cells)
  ALLOC(g.local, n_cells)
  ALLOC(g.chunk_sum, n_chunks + 1)
  ALLOC(g.cell_start, n_cells + 1)
  ALLOC(g.lr_sorted, n_cand)
  ALLOC(smp, n_cells)
  ALLOC(flags, n_cells)
  ALLOC(local, n_cells)
  ALLOC(csum, n_chunks + 1)
#undef ALLOC
  if (e == hipSuccess) e = hipMemsetAsync(g.counts, 0, sizeof(uint32_t) * (size_t)n_cells, st);
  if (e == hipSuccess) e = launch_build_grid_points(gc, cand, nullptr, n_cand, n_cells, g, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_zero_f4, dim3(blocks_of(n_cells)), dim3(kBlock), 0, st, smp, n_cells);
    e = hipGetLastError();
  }
  for (int col = 0; col < 27 && e == hipSuccess; ++col) {
    const int a = col % 3, b = (col / 3) % 3, c = col / 9;
    const int ni = (gc.dims[0] - a + 2) / 3, nj = (gc.dims[1] - b + 2) / 3, nk = (gc.dims[2] - c + 2) / 3;
    const int64_t cnt = (int64_t)ni * nj * nk;
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_sample_phase, dim3(blocks_of(cnt)), dim3(kBlock), 0, st, gc, g.cell_start, g.lr_sorted,
                       smp, a, b, c, ni, nj, nk, gc.h2, phase_offsets(a, b, c));
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sample_flags, dim3(blocks_of(n_cells)), dim3(kBlock), 0, st, smp, n_cells, flags);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_scan_bins(flags, n_cells, local, csum, st);
  if (e == hipSuccess && max_out > 0) {
    hipLaunchKernelGGL(k_sample_compact, dim3(blocks_of(n_cells)), dim3(kBlock), 0, st, smp, n_cells, local, csum,
                       out, max_out);
    e = hipGetLastError();
  }
  uint32_t total = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&total, csum + n_chunks, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  void* ptrs[] = {g.keys, g.slot, g.tmp, g.perm, g.counts, g.local, g.chunk_sum, g.cell_start, g.lr_sorted,
                  smp, flags, local, csum, total_dev};
  for (void* q : ptrs)
    if (q != nullptr) (void)hipFree(q);
  if (e == hipErrorOutOfMemory) return UPSAMPLE_ERR_OOM;
  if (e != hipSuccess) return UPSAMPLE_ERR_HIP;
  *n_out = (int64_t)total;
  return (int64_t)total > max_out ? UPSAMPLE_ERR_CAPACITY : UPSAMPLE_OK;
}
