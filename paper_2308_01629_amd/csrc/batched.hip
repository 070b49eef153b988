// Batched step over many independent scenes: the scene table, the tile
// tables, the shared scratch, HIP graph capture / replay and the
// upsample_batch_* entry points declared in include/upsample.h.
//
// Layout.  Scene s owns global cells [cell_base_s, cell_base_s + n_cells_s)
// and internal LR indices [lr_int_s, lr_int_s + n_lr_s), both assigned in
// scene order, so the one counting sort over all cells leaves the sorted LR
// copy of scene s in internal positions lr_int_s .. and its cell_start values
// are those of a single-scene build shifted by lr_int_s: every scene sees
// exactly the candidates, in exactly the order, of upsample_step.
//
// Launch.  Six kernels per step (LR keys, two scan steps, scatter, stable
// fix, gather over the tile table); counters are re-zeroed by the kernels
// that consume them, so a captured step needs no memset node.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace ups;

namespace {

constexpr int kGraphCache = 4;
constexpr int kXcds = 8;  // the HR tile table is split in this many contiguous ranges

struct GraphEntry {
  const void* key[7];
  hipGraph_t graph;
  hipGraphExec_t exec;
  uint64_t used;
};

}  // namespace

struct upsample_batch_s {
  int device;
  uint32_t flags;
  int32_t n_scenes;
  int64_t total_lr, total_hr, n_int, n_cells;
  int64_t n_lr_blocks, n_tiles;
  int grid_blocks;
  bool counts_dirty;
  BatchScene* d_scenes;
  BatchTile* d_lr_blocks;
  BatchTile* d_tiles;
  float* d_walls;
  uint16_t* d_scene_of;
  GridScratch g;
  hipStream_t cap;  // capture stream (default priority)
  GraphEntry graphs[kGraphCache];
  int n_graphs;
  uint64_t clock;
  int64_t captured;
  // HR reorder (upsample_batch_sort_hr): per-scene grid constants and sort
  // key, and the sort scratch, allocated at the first reorder
  std::vector<BatchScene> host_scenes;
  std::vector<int> sort_sub, sort_mode;
  HRSortScratch hsort;
  bool hsort_ready;
  bool sort_one_pass;        // one counting sort over all scenes (see upsample_batch_sort_hr)
  int64_t* d_sort_start;     // [n_scenes + 1] first column of each scene
  HrRankScene* d_rank_scenes;
  uint32_t* d_rank;          // Hilbert rank of each fine cell, per scene
  int64_t rank_bins;
  std::string last_error;
};

namespace {

int bfail(upsample_batch b, int code, const std::string& msg) {
  if (b != nullptr) b->last_error = msg;
  return code;
}

int bhip(upsample_batch b, hipError_t e, const char* where) {
  return bfail(b, UPSAMPLE_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename T>
hipError_t dalloc(T** p, int64_t count) {
  return hipMalloc((void**)p, (size_t)(count > 0 ? count : 1) * sizeof(T));
}

void release(upsample_batch b) {
  for (int k = 0; k < b->n_graphs; ++k) {
    (void)hipGraphExecDestroy(b->graphs[k].exec);
    (void)hipGraphDestroy(b->graphs[k].graph);
  }
  b->n_graphs = 0;
  void* ptrs[] = {b->d_scenes, b->d_lr_blocks, b->d_tiles, b->d_walls, b->d_scene_of, b->g.keys, b->g.slot,
                  b->g.tmp, b->g.perm, b->g.counts, b->g.local, b->g.chunk_sum,
                  b->g.cell_start, b->g.lr_sorted, b->hsort.keys, b->hsort.slot, b->hsort.src, b->hsort.x,
                  b->hsort.v, b->hsort.perm, b->hsort.counts, b->hsort.local, b->hsort.chunk_sum,
                  b->d_sort_start, b->d_rank_scenes, b->d_rank};
  for (void* q : ptrs)
    if (q != nullptr) (void)hipFree(q);
  if (b->cap != nullptr) (void)hipStreamDestroy(b->cap);
}

// Column ranges [off, off + n) of different scenes must not overlap.
bool disjoint(std::vector<std::pair<int64_t, int64_t>> r) {
  std::sort(r.begin(), r.end());
  for (size_t k = 1; k < r.size(); ++k)
    if (r[k].first < r[k - 1].first + r[k - 1].second) return false;
  return true;
}

// The step's launches on one stream.
hipError_t enqueue(upsample_batch b, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                   const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out, hipStream_t st) {
  BatchGridArgs ga;
  ga.scenes = b->d_scenes;
  ga.lr_blocks = b->d_lr_blocks;
  ga.n_lr_blocks = b->n_lr_blocks;
  ga.lr_x = lr_x;
  ga.lr_v = lr_v;
  ga.lr_rigid = lr_rigid;
  ga.ld = b->total_lr;
  ga.n_int = b->n_int;
  ga.n_cells = b->n_cells;
  ga.scene_of = b->d_scene_of;
  hipError_t e = launch_build_grid_batched(ga, b->g, st);
  if (e != hipSuccess) return e;
  BatchAdvanceArgs aa;
  aa.scenes = b->d_scenes;
  aa.tiles = b->d_tiles;
  aa.n_tiles = b->n_tiles;
  aa.walls = b->d_walls;
  aa.lr = b->g.lr_sorted;
  aa.cell_start = b->g.cell_start;
  aa.hx = hr_x;
  aa.hv = hr_v;
  aa.hx_out = hr_x_out;
  aa.hv_out = hr_v_out;
  aa.ld = b->total_hr;
  aa.tile_max = 512;
  aa.rigid = lr_rigid != nullptr ? 1 : 0;
  return launch_advance_batched(aa, b->grid_blocks, st);
}

}  // namespace

extern "C" {

int upsample_batch_init(const upsample_scene* scenes, int32_t n_scenes, uint32_t flags, upsample_batch* out) {
  if (out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  *out = nullptr;
  if (scenes == nullptr || n_scenes < 1 || n_scenes > UPSAMPLE_MAX_SCENES) return UPSAMPLE_ERR_INVALID_ARG;
  if ((flags & ~UPSAMPLE_BATCH_EAGER) != 0u) return UPSAMPLE_ERR_INVALID_ARG;

  // host tables
  std::vector<BatchScene> hs((size_t)n_scenes);
  std::vector<float> walls;
  std::vector<BatchTile> lr_blocks, tiles_by_scene;
  std::vector<std::pair<int64_t, int64_t>> lr_ranges, hr_ranges;
  int64_t total_lr = 0, total_hr = 0, n_int = 0, n_cells = 0;
  for (int32_t s = 0; s < n_scenes; ++s) {
    const upsample_scene& d = scenes[s];
    std::string why;
    upsample_grid_info gi;
    int rc = check_scene_params(&d.params, &gi, &why);
    if (rc != UPSAMPLE_OK) return rc;
    if (d.lr_offset < 0 || d.n_lr < 0 || d.hr_offset < 0 || d.n_hr < 0) return UPSAMPLE_ERR_INVALID_ARG;
    if (d.n_hr >= ((int64_t)1 << 31) || d.n_lr >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_INVALID_ARG;
    BatchScene& b = hs[(size_t)s];
    std::memset(&b, 0, sizeof(b));
    for (int a = 0; a < 3; ++a) {
      b.gc.lo[a] = gi.lo[a];
      b.gc.dims[a] = gi.dims[a];
      b.sc.g[a] = d.params.g[a];
    }
    b.gc.inv_cs = gi.inv_cell_size;
    b.gc.cs = (float)gi.cell_size;
    b.gc.reach = gi.reach;
    b.gc.h2 = gi.h2;
    b.gc.inv_h2 = gi.inv_h2;
    b.sc.c1 = d.params.c1;
    b.sc.c2 = d.params.c2;
    b.sc.dt = d.params.dt;
    b.sc.r_hr = d.params.r_hr;
    b.sc.n_walls = d.params.n_walls;
    b.sc.has_rigid = 0;  // the rigid rule is a kernel variant, chosen per step by lr_rigid
    b.hr_off = d.hr_offset;
    b.n_hr = d.n_hr;
    b.lr_off = d.lr_offset;
    b.n_lr = d.n_lr;
    b.lr_int = n_int;
    b.cell_base = (uint32_t)n_cells;
    b.n_cells = (uint32_t)gi.n_cells;
    b.wall_off = (int32_t)walls.size();
    for (int k = 0; k < d.params.n_walls * UPSAMPLE_WALL_FLOATS; ++k) walls.push_back(d.params.walls[k]);
    n_int += d.n_lr;
    n_cells += gi.n_cells;
    if (n_cells >= ((int64_t)1 << 31) - 1 || n_int >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_GRID_TOO_LARGE;
    total_lr = std::max(total_lr, d.lr_offset + d.n_lr);
    total_hr = std::max(total_hr, d.hr_offset + d.n_hr);
    if (d.n_lr > 0) lr_ranges.push_back({d.lr_offset, d.n_lr});
    if (d.n_hr > 0) hr_ranges.push_back({d.hr_offset, d.n_hr});
    for (int64_t f = 0; f < d.n_lr; f += kBlock) lr_blocks.push_back({(uint32_t)s, (uint32_t)f});
    for (int64_t f = 0; f < d.n_hr; f += kBlock) tiles_by_scene.push_back({(uint32_t)s, (uint32_t)f});
  }
  if (!disjoint(lr_ranges) || !disjoint(hr_ranges)) return UPSAMPLE_ERR_INVALID_ARG;
  // sanity of the per-scene stride products used on the device
  if (total_lr >= ((int64_t)1 << 40) || total_hr >= ((int64_t)1 << 40)) return UPSAMPLE_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return UPSAMPLE_ERR_NO_DEVICE;

  upsample_batch b = new (std::nothrow) upsample_batch_s();
  if (b == nullptr) return UPSAMPLE_ERR_OOM;
  b->flags = flags;
  b->n_scenes = n_scenes;
  b->total_lr = total_lr;
  b->total_hr = total_hr;
  b->n_int = n_int;
  b->n_cells = n_cells;
  b->n_lr_blocks = (int64_t)lr_blocks.size();
  b->n_tiles = (int64_t)tiles_by_scene.size();
  b->host_scenes = hs;
  // the HR reorder key of each scene: the single-scene handle's default
  // (Hilbert keys over cells split in 2 per axis when their bins fit)
  b->sort_sub.assign((size_t)n_scenes, 0);
  b->sort_mode.assign((size_t)n_scenes, 0);
  for (int32_t s = 0; s < n_scenes; ++s) {
    const int* dims = hs[(size_t)s].gc.dims;
    auto bins_for = [&](int sub) { return std::max(sort_bins(dims, sub, 0), sort_bins(dims, sub, 1)); };
    int max_sub = 4;
    while (max_sub > 1 && bins_for(max_sub) > ((int64_t)1 << 24)) max_sub /= 2;
    if (bins_for(max_sub) > ((int64_t)1 << 24)) continue;  // sub 0: this scene cannot be reordered
    const int sub = max_sub >= 2 ? 2 : 1;
    b->sort_sub[(size_t)s] = sub;
    b->sort_mode[(size_t)s] = sort_bins(dims, sub, 2) <= ((int64_t)1 << 24) ? 2 : 0;
  }
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return UPSAMPLE_ERR_NO_DEVICE;
  }
  // One launch position per tile (run as one one-wave block per 64 of its
  // particles): tiles differ in cost, and the hardware dispatcher balances
  // them better than a resident grid striding over the table (that was 9%
  // slower on the 64-scene workload).
  b->grid_blocks = (int)std::max<int64_t>(b->n_tiles, 1);

  // tile table in XCD order: block k runs on XCD k % kXcds and walks a
  // contiguous share of the tiles, so one XCD's L2 serves neighbouring tiles
  std::vector<BatchTile> tiles;
  tiles.reserve(tiles_by_scene.size());
  {
    const int64_t T = b->n_tiles;
    const int P = b->grid_blocks;
    const int X = P >= kXcds ? kXcds : 1;
    // block k takes tile positions k, k + P, ... (one position when P = T);
    // give XCD x (blocks k = x mod X) the range [T * x / X, T * (x + 1) / X)
    // in scene order
    std::vector<BatchTile> order((size_t)T);
    std::vector<int64_t> next((size_t)X);
    for (int x = 0; x < X; ++x) next[(size_t)x] = T * x / X;
    std::vector<int64_t> end((size_t)X);
    for (int x = 0; x < X; ++x) end[(size_t)x] = T * (x + 1) / X;
    // walk launch positions in order; position p belongs to block p % P,
    // hence XCD (p % P) % X
    for (int64_t p = 0; p < T; ++p) {
      const int x = (int)((p % P) % X);
      int64_t src;
      if (next[(size_t)x] < end[(size_t)x]) {
        src = next[(size_t)x]++;
      } else {
        // this XCD's share is used up: take the next tile of any other share
        int y = 0;
        while (y < X && next[(size_t)y] >= end[(size_t)y]) ++y;
        src = next[(size_t)y]++;
      }
      order[(size_t)p] = tiles_by_scene[(size_t)src];
    }
    tiles.swap(order);
  }

  hipError_t e = hipSuccess;
  const int64_t n_chunks = (n_cells + kScanChunk - 1) / kScanChunk;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  chk(dalloc(&b->d_scenes, n_scenes));
  chk(dalloc(&b->d_lr_blocks, b->n_lr_blocks));
  chk(dalloc(&b->d_tiles, b->n_tiles));
  chk(dalloc(&b->d_walls, (int64_t)walls.size()));
  chk(dalloc(&b->d_scene_of, n_int));
  chk(dalloc(&b->g.keys, n_int));
  chk(dalloc(&b->g.slot, n_int));
  chk(dalloc(&b->g.tmp, n_int));
  chk(dalloc(&b->g.perm, n_int));
  chk(dalloc(&b->g.counts, n_cells));
  chk(dalloc(&b->g.local, n_cells));
  chk(dalloc(&b->g.chunk_sum, n_chunks + 2));
  chk(dalloc(&b->g.cell_start, n_cells + 1));
  chk(dalloc(&b->g.lr_sorted, n_int));
  if (e != hipSuccess) {
    release(b);
    delete b;
    return UPSAMPLE_ERR_OOM;
  }
  chk(hipMemcpy(b->d_scenes, hs.data(), sizeof(BatchScene) * hs.size(), hipMemcpyHostToDevice));
  if (!lr_blocks.empty())
    chk(hipMemcpy(b->d_lr_blocks, lr_blocks.data(), sizeof(BatchTile) * lr_blocks.size(), hipMemcpyHostToDevice));
  if (!tiles.empty())
    chk(hipMemcpy(b->d_tiles, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice));
  if (!walls.empty())
    chk(hipMemcpy(b->d_walls, walls.data(), sizeof(float) * walls.size(), hipMemcpyHostToDevice));
  chk(hipMemset(b->g.counts, 0, sizeof(uint32_t) * (size_t)std::max<int64_t>(n_cells, 1)));
  chk(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  chk(hipDeviceSynchronize());
  if (e != hipSuccess) {
    release(b);
    delete b;
    return UPSAMPLE_ERR_HIP;
  }
  *out = b;
  return UPSAMPLE_OK;
}

int upsample_batch_step(upsample_batch b, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                        const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out, void* stream) {
  if (b == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (b->total_lr > 0 && (lr_x == nullptr || lr_v == nullptr))
    return bfail(b, UPSAMPLE_ERR_INVALID_ARG, "LR pointer is NULL");
  if (b->total_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr))
    return bfail(b, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != b->device)
    return bfail(b, UPSAMPLE_ERR_STATE, "the current HIP device is not the batch's device");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (b->counts_dirty) {
    e = hipMemsetAsync(b->g.counts, 0, sizeof(uint32_t) * (size_t)std::max<int64_t>(b->n_cells, 1), st);
    if (e != hipSuccess) return bhip(b, e, "batch_step");
    b->counts_dirty = false;
  }
  if (b->flags & UPSAMPLE_BATCH_EAGER) {
    e = enqueue(b, lr_x, lr_v, lr_rigid, hr_x, hr_v, hr_x_out, hr_v_out, st);
    if (e != hipSuccess) {
      b->counts_dirty = true;
      return bhip(b, e, "batch_step");
    }
    return UPSAMPLE_OK;
  }
  const void* key[7] = {lr_x, lr_v, lr_rigid, hr_x, hr_v, hr_x_out, hr_v_out};
  GraphEntry* g = nullptr;
  for (int k = 0; k < b->n_graphs; ++k)
    if (std::memcmp(b->graphs[k].key, key, sizeof(key)) == 0) g = &b->graphs[k];
  if (g == nullptr) {
    // capture the launches once for this set of buffers
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "graph capture");
    hipError_t le = enqueue(b, lr_x, lr_v, lr_rigid, hr_x, hr_v, hr_x_out, hr_v_out, b->cap);
    e = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      return bhip(b, le != hipSuccess ? le : e, "graph capture");
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return bhip(b, e, "graph instantiate");
    }
    if (b->n_graphs == kGraphCache) {  // evict the least recently used
      int old = 0;
      for (int k = 1; k < b->n_graphs; ++k)
        if (b->graphs[k].used < b->graphs[old].used) old = k;
      // the evicted graph may still run on some stream: wait for the device
      (void)hipDeviceSynchronize();
      (void)hipGraphExecDestroy(b->graphs[old].exec);
      (void)hipGraphDestroy(b->graphs[old].graph);
      b->graphs[old] = b->graphs[b->n_graphs - 1];
      --b->n_graphs;
    }
    g = &b->graphs[b->n_graphs++];
    std::memcpy(g->key, key, sizeof(key));
    g->graph = graph;
    g->exec = exec;
    ++b->captured;
  }
  g->used = ++b->clock;
  e = hipGraphLaunch(g->exec, st);
  if (e != hipSuccess) {
    b->counts_dirty = true;
    return bhip(b, e, "graph launch");
  }
  return UPSAMPLE_OK;
}

namespace {

// First call of upsample_batch_sort_hr: the sort scratch, and when the scenes
// own consecutive column ranges in scene order and all take Hilbert keys, the
// per-scene Hilbert rank tables of the one-pass sort.
hipError_t prepare_sort(upsample_batch b, hipStream_t st) {
  const int32_t S = b->n_scenes;
  bool one = true;
  int64_t pos = 0, rank_bins = 0, max_cube = 1, max_n = 0, max_bins = 1;
  std::vector<int64_t> start((size_t)S + 1, 0);
  std::vector<HrRankScene> rs((size_t)S);
  for (int32_t s = 0; s < S; ++s) {
    const BatchScene& d = b->host_scenes[(size_t)s];
    max_n = std::max<int64_t>(max_n, d.n_hr);
    if (d.n_hr > 0)
      max_bins = std::max(max_bins, sort_bins(d.gc.dims, b->sort_sub[(size_t)s], b->sort_mode[(size_t)s]));
    one = one && d.hr_off == pos && b->sort_mode[(size_t)s] == 2;
    pos += d.n_hr;
    start[(size_t)s + 1] = pos;
    HrRankScene& r = rs[(size_t)s];
    r.gc = d.gc;
    r.sub = b->sort_sub[(size_t)s];
    int bits = 0;
    for (int a = 0; a < 3; ++a) {
      r.fdims[a] = d.gc.dims[a] * r.sub;
      bits = std::max(bits, sort_bits(r.fdims[a]));
    }
    r.base = (uint32_t)rank_bins;
    rank_bins += (int64_t)r.fdims[0] * r.fdims[1] * r.fdims[2];
    max_cube = std::max<int64_t>(max_cube, (int64_t)1 << (3 * bits));
    if (rank_bins >= ((int64_t)1 << 31)) one = false;
  }
  one = one && pos == b->total_hr;
  b->sort_one_pass = one;
  const int64_t n_sort = one ? b->total_hr : max_n;
  const int64_t bins = one ? std::max(rank_bins, max_cube) : max_bins;
  HRSortScratch& h = b->hsort;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  chk(dalloc(&h.keys, n_sort));
  chk(dalloc(&h.slot, n_sort));
  chk(dalloc(&h.src, n_sort));
  chk(dalloc(&h.x, 3 * n_sort));
  chk(dalloc(&h.v, 3 * n_sort));
  chk(dalloc(&h.perm, n_sort));
  chk(dalloc(&h.counts, bins));
  chk(dalloc(&h.local, bins));
  chk(dalloc(&h.chunk_sum, bins / kScanChunk + 2));
  if (one) {
    chk(dalloc(&b->d_sort_start, (int64_t)S + 1));
    chk(dalloc(&b->d_rank_scenes, S));
    chk(dalloc(&b->d_rank, rank_bins));
  }
  if (e != hipSuccess) return e;
  h.n_bins = bins;
  h.max_sub = 2;
  b->rank_bins = rank_bins;
  // the sort leaves its counts at zero behind it; they start at zero here
  chk(hipMemset(h.counts, 0, sizeof(uint32_t) * (size_t)bins));
  if (one) {
    chk(hipMemcpy(b->d_sort_start, start.data(), sizeof(int64_t) * start.size(), hipMemcpyHostToDevice));
    chk(hipMemcpy(b->d_rank_scenes, rs.data(), sizeof(HrRankScene) * rs.size(), hipMemcpyHostToDevice));
    for (int32_t s = 0; s < S && e == hipSuccess; ++s)
      chk(launch_hilbert_ranks(rs[(size_t)s].fdims, b->d_rank + rs[(size_t)s].base, h.counts, h.local, h.chunk_sum,
                               st));
    chk(hipStreamSynchronize(st));
  }
  return e;
}

}  // namespace

int upsample_batch_sort_hr(upsample_batch b, float* hr_x, float* hr_v, int32_t* perm, void* stream) {
  if (b == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (b->total_hr == 0) return UPSAMPLE_OK;
  if (hr_x == nullptr || hr_v == nullptr) return bfail(b, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  if (b->total_hr >= ((int64_t)1 << 31)) return bfail(b, UPSAMPLE_ERR_INVALID_ARG, "total_hr >= 2^31");
  for (int32_t s = 0; s < b->n_scenes; ++s)
    if (b->host_scenes[(size_t)s].n_hr > 0 && b->sort_sub[(size_t)s] == 0)
      return bfail(b, UPSAMPLE_ERR_GRID_TOO_LARGE, "scene " + std::to_string(s) + ": grid too fine to reorder");
  hipStream_t st = (hipStream_t)stream;
  if (!b->hsort_ready) {
    const hipError_t e = prepare_sort(b, st);
    if (e != hipSuccess)
      return e == hipErrorOutOfMemory ? bfail(b, UPSAMPLE_ERR_OOM, "batch_sort_hr: out of device memory")
                                      : bhip(b, e, "batch_sort_hr set-up");
    b->hsort_ready = true;
  }
  if (b->sort_one_pass) {
    const hipError_t e = launch_sort_hr_batched(hr_x, hr_v, b->total_hr, b->d_sort_start, b->n_scenes,
                                                b->d_rank_scenes, b->d_rank, b->rank_bins, b->hsort, perm, st);
    if (e != hipSuccess) return bhip(b, e, "batch_sort_hr");
    return UPSAMPLE_OK;
  }
  for (int32_t s = 0; s < b->n_scenes; ++s) {
    const BatchScene& d = b->host_scenes[(size_t)s];
    if (d.n_hr == 0) continue;
    const int64_t off = d.hr_off;
    hipError_t e = launch_sort_hr(d.gc, hr_x + off, hr_v + off, hr_x + off, hr_v + off, d.n_hr,
                                  b->sort_sub[(size_t)s], b->sort_mode[(size_t)s], b->hsort,
                                  perm != nullptr ? perm + off : nullptr, st, b->total_hr, (int32_t)off);
    if (e != hipSuccess) return bhip(b, e, "batch_sort_hr");
  }
  return UPSAMPLE_OK;
}

int upsample_batch_destroy(upsample_batch b) {
  if (b == nullptr) return UPSAMPLE_OK;
  (void)hipDeviceSynchronize();
  release(b);
  delete b;
  return UPSAMPLE_OK;
}

const char* upsample_batch_last_error(upsample_batch b) {
  if (b == nullptr) return "null batch";
  return b->last_error.c_str();
}

int upsample_batch_info(upsample_batch b, int64_t* out) {
  if (b == nullptr || out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  out[0] = b->total_lr;
  out[1] = b->total_hr;
  out[2] = b->n_tiles;
  out[3] = b->grid_blocks;
  out[4] = b->captured;
  return UPSAMPLE_OK;
}

}  // extern "C"
