// Host runtime of the upsampling library: parameter validation, the grid
// definition, the handle and its scratch, and the extern "C" entry points
// declared in include/upsample.h.  No C++ exception crosses the ABI.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace ups;

static constexpr int kTimingRing = 256;
static constexpr int kRunBatch = 4;  // frames per grid-build batch of upsample_run
static constexpr int64_t kWallMaskMaxCells = (int64_t)1 << 22;  // larger grids test every wall

struct upsample_handle_s {
  upsample_params p;
  float walls[UPSAMPLE_MAX_WALLS * UPSAMPLE_WALL_FLOATS];
  upsample_grid_info gi;
  int device;
  int64_t n_cells;
  int n_chunks;
  GridScratch g;
  HRSortScratch hs;
  // upsample_run: the further grid buffers (with g, two sets of kRunBatch),
  // their build stream and events, the permutation scratch (allocated at the
  // first call)
  GridScratch run_g[2 * kRunBatch - 1];
  bool run_ready;
  bool run_dirty;
  hipStream_t side;
  hipEvent_t built[2], consumed[2], entry;
  int32_t* run_perm;
  uint32_t* finite_flag;
  float* g_sorted;      // [6][max_lr] adjoint LR gradients by sorted index, zero between calls
  GridScratch hr_g;     // DETERMINISTIC_BWD: HR particles sorted by cell (max_hr)
  float* det_coef;      // DETERMINISTIC_BWD: [7][max_hr] adjoint coefficients per HR particle
  bool hr_g_dirty;      // a failed deterministic backward may have left hr_g.counts non-zero
  uint32_t* wall_mask;  // [n_cells] walls near each cell's neighbourhood, or null
  bool grid_valid;
  bool counts_dirty;     // an interrupted build may have left counts non-zero
  bool hr_counts_dirty;  // same for the HR sort bins
  uint32_t* hr_rank;     // Hilbert ranks of the fine cells at hr_rank_sub (reorder mode 2), built at first use
  int64_t hr_rank_cap;
  int hr_rank_sub;       // 0: not built
  bool g_sorted_dirty;   // a failed backward may have left g_sorted non-zero
  int64_t grid_n_lr;
  bool has_rigid;
  upsample_tuning tune;
  bool timing;
  hipEvent_t ev[2 * kTimingRing];  // start/stop pairs, reused round-robin
  int64_t timed_issued;            // pairs recorded since the last read
  int64_t timed_folded;            // pairs already summed into timed_ms
  int32_t timed_n[kTimingRing];    // kernel launches between each pair's events
  int64_t timed_launches;          // launches in the pairs already folded
  int32_t seg_slot, seg_n;         // open pair: its slot and launches so far (seg_n < 0: none)
  double timed_ms;
  std::string last_error;
};

namespace {

int fail(upsample_handle h, int code, const std::string& msg) {
  if (h != nullptr) h->last_error = msg;
  return code;
}

int hip_fail(upsample_handle h, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(h, UPSAMPLE_ERR_HIP, m);
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// The Hilbert ranks of the grid's fine cells at the tuned sub-cell count, for
// a reorder in mode 2: built on the stream at the first such reorder and
// again after the tuning changes the count (the HR bins serve as the
// marking cube and are left zero).  Other modes need none.
hipError_t ensure_hr_ranks(upsample_handle h, hipStream_t st) {
  if (h->tune.sort_mode != 2 || h->hr_rank_sub == h->tune.sort_sub) return hipSuccess;
  const int sub = h->tune.sort_sub;
  const int fd[3] = {h->gi.dims[0] * sub, h->gi.dims[1] * sub, h->gi.dims[2] * sub};
  const int64_t F = (int64_t)fd[0] * fd[1] * fd[2];
  hipError_t e = hipSuccess;
  if (F > h->hr_rank_cap) {
    if (h->hr_rank != nullptr) e = hipFree(h->hr_rank);
    h->hr_rank = nullptr;
    h->hr_rank_cap = 0;
    if (e == hipSuccess) e = hipMalloc((void**)&h->hr_rank, sizeof(uint32_t) * (size_t)F);
    if (e != hipSuccess) return e;
    h->hr_rank_cap = F;
  }
  h->hr_rank_sub = 0;
  e = launch_hilbert_ranks(fd, h->hr_rank, h->hs.counts, h->hs.local, h->hs.chunk_sum, st);
  if (e != hipSuccess) {
    h->hr_counts_dirty = true;
    return e;
  }
  h->hr_rank_sub = sub;
  return hipSuccess;
}

// The grid definition (see upsample_grid_info in the header).
int compute_grid(const upsample_params* p, upsample_grid_info* gi, std::string* why) {
  const double r = (double)p->r_lr;
  const float kf = p->cell_factor > 0.0f ? p->cell_factor : UPSAMPLE_DEFAULT_CELL_FACTOR;
  const double kappa = (double)kf;
  const double h = 3.0 * r;
  const double cs = kappa * h;
  int64_t n = 1;
  int gmax = 1;
  for (int a = 0; a < 3; ++a) {
    const double ext = ((double)p->domain_hi[a] - (double)p->domain_lo[a]) / cs;
    if (!(ext < 1048576.0)) {
      *why = "grid axis exceeds 2^20 cells";
      return UPSAMPLE_ERR_GRID_TOO_LARGE;
    }
    int d = (int)std::ceil(ext);
    if (d < 1) d = 1;
    gi->dims[a] = d;
    gi->lo[a] = p->domain_lo[a];
    if (d > gmax) gmax = d;
    n *= d;
  }
  if (n >= (int64_t)1 << 31) {
    *why = "grid has 2^31 cells or more";
    return UPSAMPLE_ERR_GRID_TOO_LARGE;
  }
  const double reach = std::ceil(h / cs + 16.0 * gmax * std::ldexp(1.0, -24));
  if (reach > 64.0) {
    *why = "cell_factor too small: stencil reach above 64 cells";
    return UPSAMPLE_ERR_INVALID_ARG;
  }
  gi->reach = (int)reach;
  gi->n_cells = n;
  gi->cell_size = cs;
  gi->inv_cell_size = (float)(1.0 / cs);
  gi->h2 = (float)(9.0 * r * r);
  gi->inv_h2 = (float)(1.0 / (9.0 * r * r));
  return UPSAMPLE_OK;
}

int validate_params(const upsample_params* p, std::string* why) {
  if (p == nullptr) {
    *why = "params is NULL";
    return UPSAMPLE_ERR_INVALID_ARG;
  }
  if (!(std::isfinite(p->r_lr) && p->r_lr > 0.0f)) { *why = "r_lr must be finite and > 0"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!(std::isfinite(p->r_hr) && p->r_hr >= 0.0f)) { *why = "r_hr must be finite and >= 0"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!(std::isfinite(p->dt) && p->dt >= 0.0f)) { *why = "dt must be finite and >= 0"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!finite3(p->g)) { *why = "g must be finite"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!(std::isfinite(p->c1) && std::isfinite(p->c2))) { *why = "c1, c2 must be finite"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!finite3(p->domain_lo) || !finite3(p->domain_hi)) { *why = "domain must be finite"; return UPSAMPLE_ERR_INVALID_ARG; }
  for (int a = 0; a < 3; ++a)
    if (!(p->domain_hi[a] > p->domain_lo[a])) { *why = "domain_hi must exceed domain_lo"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (!(std::isfinite(p->cell_factor) && p->cell_factor >= 0.0f)) { *why = "cell_factor must be finite and >= 0"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (p->n_walls < 0 || p->n_walls > UPSAMPLE_MAX_WALLS) { *why = "n_walls must be in [0, 32]"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (p->n_walls > 0 && p->walls == nullptr) { *why = "walls is NULL"; return UPSAMPLE_ERR_INVALID_ARG; }
  for (int k = 0; k < p->n_walls; ++k) {
    const float* w = p->walls + k * UPSAMPLE_WALL_FLOATS;
    for (int c = 0; c < UPSAMPLE_WALL_FLOATS; ++c) {
      if (c == 7) continue;  // the clip offset may be a huge negative number
      if (!std::isfinite(w[c])) { *why = "wall table must be finite"; return UPSAMPLE_ERR_INVALID_ARG; }
    }
    if (std::isnan(w[7])) { *why = "wall clip offset is NaN"; return UPSAMPLE_ERR_INVALID_ARG; }
    if (w[11] < 0.0f) { *why = "wall hole radius must be >= 0"; return UPSAMPLE_ERR_INVALID_ARG; }
    const double nn = (double)w[0] * w[0] + (double)w[1] * w[1] + (double)w[2] * w[2];
    if (std::fabs(nn - 1.0) > 1e-4) { *why = "wall normal must be a unit vector"; return UPSAMPLE_ERR_INVALID_ARG; }
  }
  if (p->max_lr < 0 || p->max_hr < 0) { *why = "capacities must be >= 0"; return UPSAMPLE_ERR_INVALID_ARG; }
  if (p->max_lr >= ((int64_t)1 << 31) || p->max_hr >= ((int64_t)1 << 31)) {
    *why = "capacities must be below 2^31";
    return UPSAMPLE_ERR_INVALID_ARG;
  }
  if ((p->flags & ~(UPSAMPLE_FLAG_VALIDATE | UPSAMPLE_FLAG_DETERMINISTIC_BWD)) != 0u) {
    *why = "unknown flag bits";
    return UPSAMPLE_ERR_INVALID_ARG;
  }
  upsample_grid_info gi;
  return compute_grid(p, &gi, why);
}

template <typename T>
hipError_t dmalloc(T** p, int64_t count) {
  size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
  return hipMalloc((void**)p, bytes);
}

void free_scratch(upsample_handle h) {
  void* ptrs[] = {h->g.keys, h->g.slot, h->g.tmp, h->g.perm, h->g.counts, h->g.local, h->g.chunk_sum,
                  h->g.cell_start, h->g.lr_sorted, h->hs.keys, h->hs.slot, h->hs.src, h->hs.x,
                  h->hs.v, h->hs.perm, h->hs.counts, h->hs.local, h->hs.chunk_sum,
                  h->finite_flag, h->run_perm, h->wall_mask, h->g_sorted, h->det_coef, h->hr_rank};
  for (void* q : ptrs)
    if (q != nullptr) (void)hipFree(q);
  for (const GridScratch& g : h->run_g) {
    void* rq[] = {g.keys, g.slot, g.tmp, g.perm, g.counts, g.local, g.chunk_sum, g.cell_start, g.lr_sorted};
    for (void* q : rq)
      if (q != nullptr) (void)hipFree(q);
  }
  {
    const GridScratch& g = h->hr_g;
    void* rq[] = {g.keys, g.slot, g.tmp, g.perm, g.counts, g.local, g.chunk_sum, g.cell_start, g.lr_sorted};
    for (void* q : rq)
      if (q != nullptr) (void)hipFree(q);
  }
  if (h->run_ready) {
    (void)hipStreamDestroy(h->side);
    for (int k = 0; k < 2; ++k) {
      (void)hipEventDestroy(h->built[k]);
      (void)hipEventDestroy(h->consumed[k]);
    }
    (void)hipEventDestroy(h->entry);
  }
}

// Per grid cell, bit k set when wall k's plane can come within r_hr of the
// cell's neighbourhood, the box of cells c - reach - 1 .. c + reach + 1 on
// each axis (not clamped to the grid): the minimum of n . p - d over the box,
// in double, against r_hr plus a margin far above the float32 rounding of the
// kernel's wall test and of its region bounds.  A particle inside the box
// cannot meet a wall whose bit is clear.
std::vector<uint32_t> wall_masks(const upsample_handle h) {
  const upsample_grid_info& gi = h->gi;
  const double cs = gi.cell_size;
  const int M = gi.reach + 1;  // neighbourhood radius in cells
  double scale = 0.0;
  for (int a = 0; a < 3; ++a) {
    scale = std::fmax(scale, std::fabs((double)gi.lo[a]) + (double)(gi.dims[a] + M + 1) * cs);
  }
  double dmax = 0.0;
  for (int k = 0; k < h->p.n_walls; ++k) dmax = std::fmax(dmax, std::fabs((double)h->walls[k * UPSAMPLE_WALL_FLOATS + 3]));
  const double eps = 1e-5 * (1.0 + scale + dmax);
  const double half = (2 * M + 1) * cs * 0.5;  // half-width of a neighbourhood box
  std::vector<uint32_t> m((size_t)gi.n_cells, 0u);
  for (int k = 0; k < h->p.n_walls; ++k) {
    const float* w = h->walls + k * UPSAMPLE_WALL_FLOATS;
    const double n0 = w[0], n1 = w[1], n2 = w[2], d = w[3];
    const double spread = (std::fabs(n0) + std::fabs(n1) + std::fabs(n2)) * half;
    const double limit = (double)h->p.r_hr + eps;
    const uint32_t bit = 1u << k;
    size_t c = 0;
    for (int z = 0; z < gi.dims[2]; ++z) {
      const double pz = n2 * ((double)gi.lo[2] + (z + 0.5) * cs);
      for (int y = 0; y < gi.dims[1]; ++y) {
        const double pyz = pz + n1 * ((double)gi.lo[1] + (y + 0.5) * cs);
        for (int x = 0; x < gi.dims[0]; ++x, ++c) {
          const double centre = pyz + n0 * ((double)gi.lo[0] + (x + 0.5) * cs) - d;
          if (centre - spread < limit) m[c] |= bit;
        }
      }
    }
  }
  return m;
}

GridConst grid_const(const upsample_handle h) { return make_grid_const(h->gi); }

StepConst step_const(const upsample_handle h) { return make_step_const(h->p, h->has_rigid); }

WallTable wall_table(const upsample_handle h) { return make_wall_table(h->walls, h->p.n_walls); }

int check_device(upsample_handle h) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
    return fail(h, UPSAMPLE_ERR_STATE, "the current HIP device is not the handle's device");
  return UPSAMPLE_OK;
}

int validate_finite(upsample_handle h, hipStream_t st, const float* const* arrays, const int64_t* sizes,
                    int count) {
  if ((h->p.flags & UPSAMPLE_FLAG_VALIDATE) == 0u) return UPSAMPLE_OK;
  hipError_t e = hipMemsetAsync(h->finite_flag, 0, sizeof(uint32_t), st);
  if (e != hipSuccess) return hip_fail(h, e, "validate");
  for (int k = 0; k < count; ++k) {
    e = launch_check_finite(arrays[k], sizes[k], h->finite_flag, st);
    if (e != hipSuccess) return hip_fail(h, e, "validate");
  }
  uint32_t flag = 0;
  e = hipMemcpyAsync(&flag, h->finite_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "validate");
  if (flag != 0u) return fail(h, UPSAMPLE_ERR_NONFINITE, "non-finite value in the inputs");
  return UPSAMPLE_OK;
}

}  // namespace

namespace ups {

int check_scene_params(const upsample_params* p, upsample_grid_info* gi, std::string* why) {
  const int rc = validate_params(p, why);
  if (rc != UPSAMPLE_OK) return rc;
  return compute_grid(p, gi, why);
}

GridConst make_grid_const(const upsample_grid_info& gi) {
  GridConst gc;
  for (int a = 0; a < 3; ++a) {
    gc.lo[a] = gi.lo[a];
    gc.dims[a] = gi.dims[a];
  }
  gc.inv_cs = gi.inv_cell_size;
  gc.cs = (float)gi.cell_size;
  gc.reach = gi.reach;
  gc.h2 = gi.h2;
  gc.inv_h2 = gi.inv_h2;
  return gc;
}

StepConst make_step_const(const upsample_params& p, bool has_rigid) {
  StepConst sc;
  sc.c1 = p.c1;
  sc.c2 = p.c2;
  sc.dt = p.dt;
  sc.r_hr = p.r_hr;
  for (int a = 0; a < 3; ++a) sc.g[a] = p.g[a];
  sc.n_walls = p.n_walls;
  sc.has_rigid = has_rigid ? 1 : 0;
  return sc;
}

WallTable make_wall_table(const float* walls, int n_walls) {
  WallTable wt;
  std::memset(&wt, 0, sizeof(wt));
  if (n_walls > 0) std::memcpy(wt.w, walls, sizeof(float) * UPSAMPLE_WALL_FLOATS * n_walls);
  return wt;
}

}  // namespace ups

extern "C" {

int upsample_default_params(upsample_params* p) {
  if (p == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->r_lr = 0.02f;
  p->r_hr = 0.005f;
  p->dt = 1.0f / 60.0f;
  p->g[1] = -9.81f;
  p->c1 = 512.0f / 729.0f;
  p->c2 = 0.6f;
  for (int a = 0; a < 3; ++a) {
    p->domain_lo[a] = 0.0f;
    p->domain_hi[a] = 1.0f;
  }
  p->cell_factor = 0.0f;
  return UPSAMPLE_OK;
}

const char* upsample_strerror(int code) {
  switch (code) {
    case UPSAMPLE_OK: return "ok";
    case UPSAMPLE_ERR_INVALID_ARG: return "invalid argument";
    case UPSAMPLE_ERR_CAPACITY: return "particle count exceeds the handle's capacity";
    case UPSAMPLE_ERR_GRID_TOO_LARGE: return "neighbour grid too large";
    case UPSAMPLE_ERR_NO_DEVICE: return "no HIP device";
    case UPSAMPLE_ERR_OOM: return "device allocation failed";
    case UPSAMPLE_ERR_HIP: return "HIP runtime error";
    case UPSAMPLE_ERR_NONFINITE: return "non-finite input";
    case UPSAMPLE_ERR_STATE: return "call out of order";
    default: return "unknown error code";
  }
}

const char* upsample_last_error(upsample_handle h) {
  if (h == nullptr) return "null handle";
  return h->last_error.c_str();
}

int upsample_grid_info_for(const upsample_params* p, upsample_grid_info* out) {
  if (out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  std::string why;
  int rc = validate_params(p, &why);
  if (rc != UPSAMPLE_OK) return rc;
  return compute_grid(p, out, &why);
}

int upsample_init(const upsample_params* p, upsample_handle* out) {
  if (out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  std::string why;
  int rc = validate_params(p, &why);
  if (rc != UPSAMPLE_OK) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return UPSAMPLE_ERR_NO_DEVICE;
  upsample_handle h = new (std::nothrow) upsample_handle_s();
  if (h == nullptr) return UPSAMPLE_ERR_OOM;
  h->seg_n = -1;
  h->p = *p;
  std::memset(h->walls, 0, sizeof(h->walls));
  if (p->n_walls > 0) std::memcpy(h->walls, p->walls, sizeof(float) * UPSAMPLE_WALL_FLOATS * p->n_walls);
  h->p.walls = nullptr;
  compute_grid(&h->p, &h->gi, &why);
  h->tune.gather_groups = 1;
  h->tune.adjoint_tiled = 1;
  h->tune.tile_max = 512;
  h->tune.adjoint_tile_max = 384;
  h->tune.wall_cull = 1;
  h->n_cells = h->gi.n_cells;
  h->n_chunks = (int)((h->n_cells + kScanChunk - 1) / kScanChunk);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return UPSAMPLE_ERR_NO_DEVICE;
  }
  const int64_t nl = p->max_lr, nh = p->max_hr;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n) \
  if (e == hipSuccess) e = dmalloc(&(ptr), (n));
  ALLOC(h->g.keys, nl)
  ALLOC(h->g.slot, nl)
  ALLOC(h->g.tmp, nl)
  ALLOC(h->g.perm, nl)
  ALLOC(h->g.counts, h->n_cells)
  ALLOC(h->g.local, h->n_cells)
  ALLOC(h->g.chunk_sum, h->n_chunks + 1)
  ALLOC(h->g.cell_start, h->n_cells + 1)
  ALLOC(h->g.lr_sorted, nl)
  ALLOC(h->hs.keys, nh)
  ALLOC(h->hs.slot, nh)
  ALLOC(h->hs.src, nh)
  ALLOC(h->hs.x, 3 * nh)
  ALLOC(h->hs.v, 3 * nh)
  ALLOC(h->hs.perm, nh)
  // HR reorder bins: keys of fine cells, at most 2^24 bins
  h->hs.n_cells = h->n_cells;
  // both key modes must fit the bins allocated for max_sub
  auto bins_for = [&](int sub) {
    const int64_t b0 = sort_bins(h->gi.dims, sub, 0), b1 = sort_bins(h->gi.dims, sub, 1);
    return b0 > b1 ? b0 : b1;
  };
  h->hs.max_sub = 4;
  while (h->hs.max_sub > 1 && bins_for(h->hs.max_sub) > ((int64_t)1 << 24)) h->hs.max_sub /= 2;
  const bool can_sort = bins_for(h->hs.max_sub) <= ((int64_t)1 << 24);
  if (!can_sort) h->hs.max_sub = 0;  // grid too fine for the reorder: sort_hr reports GRID_TOO_LARGE
  int64_t n_bins = (nh > 0 && can_sort) ? bins_for(h->hs.max_sub) : 1;
  h->tune.sort_sub = h->hs.max_sub >= 2 ? 2 : 1;
  h->tune.sort_mode = 0;
  // Hilbert keys (mode 2) at the default sub-cell count are the default when
  // their bins fit: runs of particles in Hilbert order fill more compact wave
  // boxes than either Morton key
  const int64_t b2 = sort_bins(h->gi.dims, h->tune.sort_sub, 2);
  if (nh > 0 && can_sort && b2 <= ((int64_t)1 << 24)) {
    if (b2 > n_bins) n_bins = b2;
    h->tune.sort_mode = 2;
  }
  h->hs.n_bins = n_bins;
  ALLOC(h->hs.counts, n_bins)
  ALLOC(h->hs.local, n_bins)
  ALLOC(h->hs.chunk_sum, n_bins / kScanChunk + 2)
  ALLOC(h->finite_flag, 1)
  ALLOC(h->g_sorted, 6 * nl)
  const bool cull_walls = p->n_walls > 0 && h->n_cells <= kWallMaskMaxCells;
  if (cull_walls) ALLOC(h->wall_mask, h->n_cells)
  const bool det = (p->flags & UPSAMPLE_FLAG_DETERMINISTIC_BWD) != 0u;
  if (det) {
    ALLOC(h->hr_g.keys, nh)
    ALLOC(h->hr_g.slot, nh)
    ALLOC(h->hr_g.tmp, nh)
    ALLOC(h->hr_g.perm, nh)
    ALLOC(h->hr_g.counts, h->n_cells)
    ALLOC(h->hr_g.local, h->n_cells)
    ALLOC(h->hr_g.chunk_sum, h->n_chunks + 1)
    ALLOC(h->hr_g.cell_start, h->n_cells + 1)
    ALLOC(h->hr_g.lr_sorted, nh)
    ALLOC(h->det_coef, 7 * nh)
  }
#undef ALLOC
  if (e == hipSuccess && cull_walls) {
    const std::vector<uint32_t> m = wall_masks(h);
    e = hipMemcpy(h->wall_mask, m.data(), sizeof(uint32_t) * m.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(h->g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells);
  if (e == hipSuccess) e = hipMemset(h->hs.counts, 0, sizeof(uint32_t) * (size_t)n_bins);
  if (e == hipSuccess && nl > 0) e = hipMemset(h->g_sorted, 0, sizeof(float) * (size_t)(6 * nl));
  if (e == hipSuccess && det) e = hipMemset(h->hr_g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells);
  for (int k = 0; k < 2 * kTimingRing && e == hipSuccess; ++k) e = hipEventCreate(&h->ev[k]);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_scratch(h);
    delete h;
    return e == hipErrorOutOfMemory ? UPSAMPLE_ERR_OOM : UPSAMPLE_ERR_HIP;
  }
  *out = h;
  return UPSAMPLE_OK;
}

int upsample_destroy(upsample_handle h) {
  if (h == nullptr) return UPSAMPLE_OK;
  free_scratch(h);
  for (int k = 0; k < 2 * kTimingRing; ++k)
    if (h->ev[k] != nullptr) (void)hipEventDestroy(h->ev[k]);
  delete h;
  return UPSAMPLE_OK;
}

int upsample_get_grid_info(upsample_handle h, upsample_grid_info* out) {
  if (h == nullptr || out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  *out = h->gi;
  return UPSAMPLE_OK;
}

int upsample_build_grid(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                        int64_t n_lr, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_lr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_lr < 0");
  if (n_lr > h->p.max_lr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_lr exceeds max_lr");
  if (n_lr > 0 && (lr_x == nullptr || lr_v == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "lr_x / lr_v is NULL");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const float* arrs[2] = {lr_x, lr_v};
  const int64_t sizes[2] = {3 * n_lr, 3 * n_lr};
  rc = validate_finite(h, st, arrs, sizes, 2);
  if (rc != UPSAMPLE_OK) return rc;
  hipError_t e = hipSuccess;
  if (h->counts_dirty) {
    e = hipMemsetAsync(h->g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells, st);
    if (e != hipSuccess) return hip_fail(h, e, "build_grid");
    h->counts_dirty = false;
  }
  h->grid_valid = false;
  e = launch_build_grid(grid_const(h), lr_x, lr_v, lr_rigid, n_lr, h->n_cells, h->g, st);
  if (e != hipSuccess) {
    h->counts_dirty = true;
    return hip_fail(h, e, "build_grid");
  }
  h->grid_valid = true;
  h->grid_n_lr = n_lr;
  h->has_rigid = lr_rigid != nullptr;
  return UPSAMPLE_OK;
}

// Sum the elapsed time of recorded pairs up to (not including) index `upto`.
static hipError_t fold_timing(upsample_handle h, int64_t upto) {
  while (h->timed_folded < upto) {
    const int slot = (int)(h->timed_folded % kTimingRing);
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(h->ev[2 * slot + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev[2 * slot], h->ev[2 * slot + 1]);
    if (e != hipSuccess) return e;
    h->timed_ms += ms;
    h->timed_launches += h->timed_n[slot];
    h->timed_folded += 1;
  }
  return hipSuccess;
}

// Timing pairs bracket a run of consecutive step kernels on one stream (no
// other work between them): one launch for upsample_advance, up to a batch
// of frames in upsample_run.  A pair per launch would add its own event
// packets to every kernel's bracket.
static hipError_t timing_open(upsample_handle h, hipStream_t st) {
  if (h->timed_issued - h->timed_folded >= kTimingRing) {
    hipError_t e = fold_timing(h, h->timed_folded + 1);  // free the slot about to be reused
    if (e != hipSuccess) return e;
  }
  h->seg_slot = (int32_t)(h->timed_issued % kTimingRing);
  h->seg_n = 0;
  return hipEventRecord(h->ev[2 * h->seg_slot], st);
}

static hipError_t timing_close(upsample_handle h, hipStream_t st) {
  if (h->seg_n < 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (h->seg_n > 0) {
    e = hipEventRecord(h->ev[2 * h->seg_slot + 1], st);
    if (e == hipSuccess) {
      h->timed_n[h->seg_slot] = h->seg_n;
      h->timed_issued += 1;
    }
  }
  h->seg_n = -1;
  return e;
}

// debug: 0 the step, 1 the per-lane debug walk, 2 the step kernel's debug
// instance (count_w, wdis: its extra exports)
static int advance_impl(upsample_handle h, const float* hr_x, const float* hr_v, float* hr_x_out,
                        float* hr_v_out, int64_t n_hr, void* stream, int debug, uint32_t* count,
                        uint32_t* ids, int64_t max_k, uint8_t* branch, float* tape = nullptr,
                        const GridScratch* grid = nullptr, uint32_t* count_w = nullptr,
                        float* wdis = nullptr) {
  if (n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_hr < 0");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  if (max_k < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "max_k < 0");
  if (!h->grid_valid) return fail(h, UPSAMPLE_ERR_STATE, "no LR grid built on this handle");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const float* arrs[2] = {hr_x, hr_v};
  const int64_t sizes[2] = {3 * n_hr, 3 * n_hr};
  rc = validate_finite(h, st, arrs, sizes, 2);
  if (rc != UPSAMPLE_OK) return rc;
  AdvanceArgs a;
  a.gc = grid_const(h);
  a.sc = step_const(h);
  const GridScratch& gs = grid != nullptr ? *grid : h->g;
  a.lr = gs.lr_sorted;
  a.cell_start = gs.cell_start;
  a.hx = hr_x;
  a.hv = hr_v;
  a.hx_out = hr_x_out;
  a.hv_out = hr_v_out;
  a.n = n_hr;
  a.ld = n_hr;
  a.dbg_count = count;
  a.dbg_ids = ids;
  a.dbg_max_k = max_k;
  a.dbg_branch = branch;
  a.dbg_count_w = count_w;
  a.dbg_wdis = wdis;
  a.wall_mask = h->tune.wall_cull != 0 ? h->wall_mask : nullptr;
  a.groups = h->tune.gather_groups;
  a.tile_max = h->tune.tile_max;
  a.tape = tape;
  // timed on its own unless the caller (upsample_run) has a pair open
  const bool timed = h->timing && debug == 0 && n_hr > 0;
  const bool own = timed && h->seg_n < 0;
  hipError_t e = own ? timing_open(h, st) : hipSuccess;
  if (e == hipSuccess) e = launch_advance(a, wall_table(h), debug, st);
  if (e == hipSuccess && timed) h->seg_n += 1;
  if (e == hipSuccess && own) e = timing_close(h, st);
  if (e != hipSuccess) return hip_fail(h, e, "advance");
  return UPSAMPLE_OK;
}

int upsample_advance(upsample_handle h, const float* hr_x, const float* hr_v, float* hr_x_out,
                     float* hr_v_out, int64_t n_hr, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  return advance_impl(h, hr_x, hr_v, hr_x_out, hr_v_out, n_hr, stream, 0, nullptr, nullptr, 0,
                      nullptr);
}

int upsample_step(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                  int64_t n_lr, const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                  int64_t n_hr, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_hr < 0");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  int rc = upsample_build_grid(h, lr_x, lr_v, lr_rigid, n_lr, stream);
  if (rc != UPSAMPLE_OK) return rc;
  return upsample_advance(h, hr_x, hr_v, hr_x_out, hr_v_out, n_hr, stream);
}

int upsample_step_taped(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                        int64_t n_lr, const float* hr_x, const float* hr_v, float* hr_x_out, float* hr_v_out,
                        int64_t n_hr, float* tape, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_hr < 0");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr ||
                   tape == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR or tape pointer is NULL");
  int rc = upsample_build_grid(h, lr_x, lr_v, lr_rigid, n_lr, stream);
  if (rc != UPSAMPLE_OK) return rc;
  return advance_impl(h, hr_x, hr_v, hr_x_out, hr_v_out, n_hr, stream, 0, nullptr, nullptr, 0, nullptr,
                      tape);
}

// A saved grid: the LR copy in sorted order (max_lr entries of 32 B), then
// the cell ranges (n_cells + 1 words), each part 256-byte aligned.
static int64_t snapshot_lr_bytes(const upsample_handle h) {
  return (h->p.max_lr * (int64_t)sizeof(LRPoint) + 255) / 256 * 256;
}
static int64_t snapshot_bytes(const upsample_handle h) {
  return snapshot_lr_bytes(h) + ((h->n_cells + 1) * (int64_t)sizeof(uint32_t) + 255) / 256 * 256;
}

// grid: null rebuilds the grid from lr_x / lr_v / lr_rigid; otherwise a saved
// grid of the same frame (upsample_grid_snapshot), and only n_lr and whether
// lr_rigid is null are read of the LR arguments.
static int backward_impl(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                         int64_t n_lr, const float* hr_x, const float* hr_v, int64_t n_hr, const float* tape,
                         const float* gx_out, const float* gv_out, float* gx_in, float* gv_in, float* g_lr_x,
                         float* g_lr_v, void* stream, const void* grid = nullptr) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_hr < 0");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || gx_out == nullptr || gv_out == nullptr ||
                   gx_in == nullptr || gv_in == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  if (n_lr > 0 && n_hr > 0 && (g_lr_x == nullptr || g_lr_v == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "LR gradient pointer is NULL");
  const LRPoint* lr_sorted = h->g.lr_sorted;
  const uint32_t* cell_start = h->g.cell_start;
  bool has_rigid = h->has_rigid;
  int rc;
  if (grid == nullptr) {
    rc = upsample_build_grid(h, lr_x, lr_v, lr_rigid, n_lr, stream);
    if (rc != UPSAMPLE_OK) return rc;
    has_rigid = h->has_rigid;
  } else {
    if (n_lr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_lr < 0");
    if (n_lr > h->p.max_lr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_lr exceeds max_lr");
    if ((reinterpret_cast<uintptr_t>(grid) & 255u) != 0u)
      return fail(h, UPSAMPLE_ERR_INVALID_ARG, "grid snapshot is not 256-byte aligned");
    rc = check_device(h);
    if (rc != UPSAMPLE_OK) return rc;
    lr_sorted = static_cast<const LRPoint*>(grid);
    cell_start = reinterpret_cast<const uint32_t*>(static_cast<const char*>(grid) + snapshot_lr_bytes(h));
    has_rigid = lr_rigid != nullptr;
  }
  hipStream_t st = (hipStream_t)stream;
  const float* arrs[2] = {gx_out, gv_out};
  const int64_t sizes[2] = {3 * n_hr, 3 * n_hr};
  rc = validate_finite(h, st, arrs, sizes, 2);
  if (rc != UPSAMPLE_OK) return rc;
  AdjointArgs a;
  a.gc = grid_const(h);
  a.sc = make_step_const(h->p, has_rigid);
  a.lr = lr_sorted;
  a.cell_start = cell_start;
  a.hx = hr_x;
  a.hv = hr_v;
  a.gx_out = gx_out;
  a.gv_out = gv_out;
  a.gx_in = gx_in;
  a.gv_in = gv_in;
  a.g_lr_x = g_lr_x;
  a.g_lr_v = g_lr_v;
  a.g_sorted = h->g_sorted;
  a.n = n_hr;
  a.n_lr = n_lr;
  a.tiled = h->tune.adjoint_tiled;
  a.tile_max = h->tune.adjoint_tile_max;
  a.tape = tape;
  const bool det = (h->p.flags & UPSAMPLE_FLAG_DETERMINISTIC_BWD) != 0u;
  a.det_coef = det ? h->det_coef : nullptr;
  a.hr_cell_start = nullptr;
  a.hr_sorted = nullptr;
  hipError_t e = hipSuccess;
  if (h->g_sorted_dirty && n_lr > 0)
    e = hipMemsetAsync(h->g_sorted, 0, sizeof(float) * (size_t)(6 * h->p.max_lr), st);
  if (e == hipSuccess && det && h->hr_g_dirty)
    e = hipMemsetAsync(h->hr_g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells, st);
  if (e == hipSuccess) {
    h->g_sorted_dirty = true;
    h->hr_g_dirty = det;
    e = launch_adjoint(a, wall_table(h), st, det ? &h->hr_g : nullptr);
  }
  if (e != hipSuccess) return hip_fail(h, e, "step_backward");
  h->g_sorted_dirty = false;
  h->hr_g_dirty = false;
  return UPSAMPLE_OK;
}

int upsample_step_backward(upsample_handle h, const float* lr_x, const float* lr_v,
                           const uint8_t* lr_rigid, int64_t n_lr, const float* hr_x,
                           const float* hr_v, int64_t n_hr, const float* gx_out,
                           const float* gv_out, float* gx_in, float* gv_in, float* g_lr_x,
                           float* g_lr_v, void* stream) {
  return backward_impl(h, lr_x, lr_v, lr_rigid, n_lr, hr_x, hr_v, n_hr, nullptr, gx_out, gv_out, gx_in, gv_in,
                       g_lr_x, g_lr_v, stream);
}

int upsample_step_backward_taped(upsample_handle h, const float* lr_x, const float* lr_v,
                                 const uint8_t* lr_rigid, int64_t n_lr, const float* hr_x,
                                 const float* hr_v, int64_t n_hr, const float* tape, const float* gx_out,
                                 const float* gv_out, float* gx_in, float* gv_in, float* g_lr_x,
                                 float* g_lr_v, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr > 0 && tape == nullptr) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "tape is NULL");
  return backward_impl(h, lr_x, lr_v, lr_rigid, n_lr, hr_x, hr_v, n_hr, tape, gx_out, gv_out, gx_in, gv_in,
                       g_lr_x, g_lr_v, stream);
}

int upsample_grid_snapshot_bytes(upsample_handle h, int64_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "NULL argument");
  *bytes = snapshot_bytes(h);
  return UPSAMPLE_OK;
}

int upsample_grid_snapshot(upsample_handle h, void* grid, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (grid == nullptr) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "grid snapshot is NULL");
  if ((reinterpret_cast<uintptr_t>(grid) & 255u) != 0u)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "grid snapshot is not 256-byte aligned");
  if (!h->grid_valid) return fail(h, UPSAMPLE_ERR_STATE, "no grid has been built");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* dst = static_cast<char*>(grid);
  hipError_t e = hipSuccess;
  if (h->grid_n_lr > 0)
    e = hipMemcpyAsync(dst, h->g.lr_sorted, sizeof(LRPoint) * (size_t)h->grid_n_lr, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst + snapshot_lr_bytes(h), h->g.cell_start, sizeof(uint32_t) * (size_t)(h->n_cells + 1),
                       hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "grid_snapshot");
  return UPSAMPLE_OK;
}

int upsample_step_backward_taped_grid(upsample_handle h, const void* grid, const uint8_t* lr_rigid, int64_t n_lr,
                                      const float* hr_x, const float* hr_v, int64_t n_hr, const float* tape,
                                      const float* gx_out, const float* gv_out, float* gx_in, float* gv_in,
                                      float* g_lr_x, float* g_lr_v, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (grid == nullptr) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "grid snapshot is NULL");
  if (n_hr > 0 && tape == nullptr) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "tape is NULL");
  return backward_impl(h, nullptr, nullptr, lr_rigid, n_lr, hr_x, hr_v, n_hr, tape, gx_out, gv_out, gx_in, gv_in,
                       g_lr_x, g_lr_v, stream, grid);
}

static int run_prepare(upsample_handle h, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!h->run_ready) {
    const int64_t nl = h->p.max_lr, nh = h->p.max_hr;
#define ALLOC(ptr, n) \
  if (e == hipSuccess) e = dmalloc(&(ptr), (n));
    for (GridScratch& g : h->run_g) {
      ALLOC(g.keys, nl)
      ALLOC(g.slot, nl)
      ALLOC(g.tmp, nl)
      ALLOC(g.perm, nl)
      ALLOC(g.counts, h->n_cells)
      ALLOC(g.local, h->n_cells)
      ALLOC(g.chunk_sum, h->n_chunks + 1)
      ALLOC(g.cell_start, h->n_cells + 1)
      ALLOC(g.lr_sorted, nl)
    }
    ALLOC(h->run_perm, nh)
#undef ALLOC
    hipEvent_t* evs[5] = {&h->built[0], &h->built[1], &h->consumed[0], &h->consumed[1], &h->entry};
    for (hipEvent_t* ev : evs) *ev = nullptr;
    h->side = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    for (hipEvent_t* ev : evs)
      if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      // the handle stays usable without upsample_run; buffers are freed with it
      for (hipEvent_t* ev : evs)
        if (*ev != nullptr) (void)hipEventDestroy(*ev);
      if (h->side != nullptr) (void)hipStreamDestroy(h->side);
      return hip_fail(h, e, "run: allocation");
    }
    h->run_ready = true;
    h->run_dirty = true;
  }
  if (h->run_dirty) {
    for (const GridScratch& g : h->run_g)
      if (e == hipSuccess) e = hipMemsetAsync(g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells, st);
    if (e != hipSuccess) return hip_fail(h, e, "run");
    h->run_dirty = false;
  }
  if (h->counts_dirty) {
    e = hipMemsetAsync(h->g.counts, 0, sizeof(uint32_t) * (size_t)h->n_cells, st);
    if (e != hipSuccess) return hip_fail(h, e, "run");
    h->counts_dirty = false;
  }
  return UPSAMPLE_OK;
}

// The LR state one step of a run uses: frame x0, v0, or with x1, v1 the
// interpolation x0 + theta (x1 - x0) between two frames.
struct RunFrame {
  const float* x0;
  const float* v0;
  const float* x1;
  const float* v1;
  float theta;
};

static int run_impl(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                    int64_t n_lr, int32_t n_frames, const std::vector<RunFrame>& steps, float* hr_x, float* hr_v,
                    int64_t n_hr, int32_t sort_every, int32_t* perm_io, void* stream);

int upsample_run(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid, int64_t n_lr,
                 int32_t n_frames, float* hr_x, float* hr_v, int64_t n_hr, int32_t sort_every, int32_t* perm_io,
                 void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_frames < 1) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_frames < 1");
  if (n_lr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "negative count");
  std::vector<RunFrame> steps((size_t)n_frames);
  const size_t frame = 3 * (size_t)n_lr;
  for (int32_t f = 0; f < n_frames; ++f)
    steps[(size_t)f] = RunFrame{lr_x + frame * (size_t)f, lr_v + frame * (size_t)f, nullptr, nullptr, 0.0f};
  return run_impl(h, lr_x, lr_v, lr_rigid, n_lr, n_frames, steps, hr_x, hr_v, n_hr, sort_every, perm_io, stream);
}

int upsample_run_multirate(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                           int64_t n_lr, int32_t n_frames, double t_lr0, double dt_lr, double t_hr0,
                           int32_t n_steps, float* hr_x, float* hr_v, int64_t n_hr, int32_t sort_every,
                           int32_t* perm_io, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_frames < 2) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_frames < 2");
  if (n_steps < 1) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_steps < 1");
  if (n_lr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "negative count");
  if (!(std::isfinite(t_lr0) && std::isfinite(t_hr0) && std::isfinite(dt_lr) && dt_lr > 0.0))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "t_lr0, t_hr0 must be finite and dt_lr > 0");
  // the schedule, in double: step n ends at t_hr0 + (n + 1) dt and uses the
  // LR state there, between frames k and k + 1
  std::vector<RunFrame> steps((size_t)n_steps);
  const size_t frame = 3 * (size_t)n_lr;
  for (int32_t n = 0; n < n_steps; ++n) {
    const double t = t_hr0 + (double)(n + 1) * (double)h->p.dt;
    const double sf = (t - t_lr0) / dt_lr;
    double k = std::floor(sf);
    double th = sf - k;
    if (k == (double)(n_frames - 1) && th == 0.0) {
      k = (double)(n_frames - 2);
      th = 1.0;
    }
    if (!(k >= 0.0 && k <= (double)(n_frames - 2)))
      return fail(h, UPSAMPLE_ERR_INVALID_ARG, "an HR step ends outside the LR frames");
    const size_t kk = (size_t)k;
    steps[(size_t)n] = RunFrame{lr_x + frame * kk, lr_v + frame * kk, lr_x + frame * (kk + 1),
                                lr_v + frame * (kk + 1), (float)th};
  }
  return run_impl(h, lr_x, lr_v, lr_rigid, n_lr, n_frames, steps, hr_x, hr_v, n_hr, sort_every, perm_io, stream);
}

static int run_impl(upsample_handle h, const float* lr_x, const float* lr_v, const uint8_t* lr_rigid,
                    int64_t n_lr, int32_t n_frames, const std::vector<RunFrame>& steps, float* hr_x, float* hr_v,
                    int64_t n_hr, int32_t sort_every, int32_t* perm_io, void* stream) {
  if (sort_every < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "sort_every < 0");
  if (n_lr < 0 || n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "negative count");
  if (n_lr > h->p.max_lr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_lr exceeds max_lr");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_lr > 0 && (lr_x == nullptr || lr_v == nullptr)) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "LR pointer is NULL");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr)) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  if (sort_every > 0 && n_hr > 0 && h->hs.max_sub == 0)
    return fail(h, UPSAMPLE_ERR_GRID_TOO_LARGE, "grid too fine for the HR reorder (more than 2^24 key bins)");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const float* arrs[4] = {lr_x, lr_v, hr_x, hr_v};
  const int64_t sizes[4] = {3 * n_lr * (int64_t)n_frames, 3 * n_lr * (int64_t)n_frames, 3 * n_hr, 3 * n_hr};
  rc = validate_finite(h, st, arrs, sizes, 4);
  if (rc != UPSAMPLE_OK) return rc;
  rc = run_prepare(h, st);
  if (rc != UPSAMPLE_OK) return rc;
  if (h->hr_counts_dirty && sort_every > 0) {
    hipError_t e = hipMemsetAsync(h->hs.counts, 0, sizeof(uint32_t) * (size_t)h->hs.n_bins, st);
    if (e != hipSuccess) return hip_fail(h, e, "run");
    h->hr_counts_dirty = false;
  }
  h->has_rigid = lr_rigid != nullptr;
  const GridConst gc = grid_const(h);
  // Frames go in batches of kRunBatch: batch t uses buffer set t mod 2 (set
  // 0 starts with the handle's own grid).  The side stream builds batch t + 1
  // while the gathers of batch t run, once the gathers of batch t - 1 are done
  // with that set; the main stream waits once per batch.  Per frame, only the
  // gather (and a reorder when due) is queued on the caller's stream.
  GridScratch* buf[2 * kRunBatch];
  buf[0] = &h->g;
  for (int k = 1; k < 2 * kRunBatch; ++k) buf[k] = &h->run_g[k - 1];
  const int n_steps = (int)steps.size();
  const int n_batches = (n_steps + kRunBatch - 1) / kRunBatch;
  // the side stream starts after the caller's earlier work on the stream
  hipError_t e = hipEventRecord(h->entry, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->entry, 0);
  auto build_batch = [&](int t) -> hipError_t {
    const int set = t & 1;
    hipError_t r = hipStreamWaitEvent(h->side, h->consumed[set], 0);  // batch t - 2 is done with the set
    for (int j = 0; j < kRunBatch && r == hipSuccess; ++j) {
      const int f = t * kRunBatch + j;
      if (f >= n_steps) break;
      const RunFrame& fr = steps[(size_t)f];
      r = launch_build_grid_lerp(gc, fr.x0, fr.v0, fr.x1, fr.v1, fr.theta, lr_rigid, n_lr, h->n_cells,
                                 *buf[set * kRunBatch + j], h->side);
    }
    if (r == hipSuccess) r = hipEventRecord(h->built[set], h->side);
    return r;
  };
  if (e == hipSuccess) e = build_batch(0);
  int last = 0;  // buffer of the last frame gathered
  for (int t = 0; t < n_batches && e == hipSuccess; ++t) {
    const int set = t & 1;
    if (t + 1 < n_batches) e = build_batch(t + 1);  // overlaps with the gathers of batch t
    if (e == hipSuccess) e = hipStreamWaitEvent(st, h->built[set], 0);
    if (e != hipSuccess) break;
    h->grid_valid = true;
    h->grid_n_lr = n_lr;
    for (int j = 0; j < kRunBatch && e == hipSuccess; ++j) {
      const int f = t * kRunBatch + j;
      if (f >= n_steps) break;
      const float* in_x = hr_x;
      const float* in_v = hr_v;
      if (sort_every > 0 && f % sort_every == 0 && n_hr > 0) {
        // reorder into scratch; the step writes the state back into hr_x / hr_v
        e = timing_close(h, st);  // the reorder stays outside the timed stretch
        if (e != hipSuccess) break;
        int32_t* p = perm_io != nullptr ? h->run_perm : nullptr;
        e = ensure_hr_ranks(h, st);
        if (e == hipSuccess)
          e = launch_sort_hr(gc, hr_x, hr_v, h->hs.x, h->hs.v, n_hr, h->tune.sort_sub, h->tune.sort_mode, h->hs,
                             p, st, -1, 0, h->hr_rank);
        if (e == hipSuccess && p != nullptr) e = launch_compose_perm(perm_io, p, n_hr, h->hs.slot, st);
        if (e != hipSuccess) {
          h->hr_counts_dirty = true;
          break;
        }
        in_x = h->hs.x;
        in_v = h->hs.v;
      }
      last = set * kRunBatch + j;
      if (h->timing && n_hr > 0 && h->seg_n < 0) {
        e = timing_open(h, st);
        if (e != hipSuccess) break;
      }
      rc = advance_impl(h, in_x, in_v, hr_x, hr_v, n_hr, stream, 0, nullptr, nullptr, 0, nullptr, nullptr,
                        buf[last]);
      if (rc != UPSAMPLE_OK) {
        h->counts_dirty = h->run_dirty = true;
        (void)timing_close(h, st);
        (void)hipStreamSynchronize(h->side);
        return rc;
      }
    }
    if (e == hipSuccess) e = timing_close(h, st);
    if (e == hipSuccess) e = hipEventRecord(h->consumed[set], st);
  }
  if (e != hipSuccess) {
    h->counts_dirty = h->run_dirty = true;
    (void)timing_close(h, st);
    (void)hipStreamSynchronize(h->side);
    return hip_fail(h, e, "run");
  }
  // the handle's grid is the last frame's
  if (last != 0) {
    const GridScratch t = h->g;
    h->g = *buf[last];
    *buf[last] = t;
  }
  return UPSAMPLE_OK;
}

int upsample_sort_hr(upsample_handle h, const float* hr_x, const float* hr_v, float* hr_x_out,
                     float* hr_v_out, int64_t n_hr, int32_t* perm_out, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_hr < 0");
  if (n_hr > h->p.max_hr) return fail(h, UPSAMPLE_ERR_CAPACITY, "n_hr exceeds max_hr");
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "HR pointer is NULL");
  if (n_hr > 0 && ((hr_x_out == hr_x) != (hr_v_out == hr_v)))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "outputs must both alias their inputs or neither");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (h->hs.max_sub == 0)
    return fail(h, UPSAMPLE_ERR_GRID_TOO_LARGE, "grid too fine for the HR reorder (more than 2^24 key bins)");
  if (h->hr_counts_dirty) {
    hipError_t e = hipMemsetAsync(h->hs.counts, 0, sizeof(uint32_t) * (size_t)h->hs.n_bins, st);
    if (e != hipSuccess) return hip_fail(h, e, "sort_hr");
    h->hr_counts_dirty = false;
  }
  hipError_t e = ensure_hr_ranks(h, st);
  if (e == hipSuccess)
    e = launch_sort_hr(grid_const(h), hr_x, hr_v, hr_x_out, hr_v_out, n_hr, h->tune.sort_sub, h->tune.sort_mode,
                       h->hs, perm_out, st, -1, 0, h->hr_rank);
  if (e != hipSuccess) {
    h->hr_counts_dirty = true;
    return hip_fail(h, e, "sort_hr");
  }
  return UPSAMPLE_OK;
}

int upsample_permute(upsample_handle h, const float* a, const float* b, float* a_out, float* b_out,
                     int64_t n, const int32_t* perm, int mode, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n < 0) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "n < 0");
  if (mode != UPSAMPLE_PERMUTE_GATHER && mode != UPSAMPLE_PERMUTE_SCATTER)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "mode must be UPSAMPLE_PERMUTE_GATHER or UPSAMPLE_PERMUTE_SCATTER");
  if (n > 0 && (a == nullptr || a_out == nullptr || perm == nullptr))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "a, a_out or perm is NULL");
  if ((b == nullptr) != (b_out == nullptr)) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "b and b_out: both or neither");
  if (n > 0 && (a_out == a || (b != nullptr && (b_out == b || b_out == a || a_out == b))))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "outputs must not alias inputs");
  int rc = check_device(h);
  if (rc != UPSAMPLE_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const bool validate = (h->p.flags & UPSAMPLE_FLAG_VALIDATE) != 0u;
  hipError_t e = hipSuccess;
  if (validate) e = hipMemsetAsync(h->finite_flag, 0, sizeof(uint32_t), st);
  if (e == hipSuccess)
    e = launch_permute(a, b, a_out, b_out, n, perm, mode == UPSAMPLE_PERMUTE_SCATTER ? 1 : 0, h->finite_flag, st);
  if (e != hipSuccess) return hip_fail(h, e, "permute");
  if (validate) {
    uint32_t bad = 0;
    e = hipMemcpyAsync(&bad, h->finite_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(h, e, "permute");
    if (bad != 0u) return fail(h, UPSAMPLE_ERR_INVALID_ARG, "perm holds an index outside [0, n)");
  }
  return UPSAMPLE_OK;
}

int upsample_debug_grid(upsample_handle h, uint32_t* keys, uint32_t* perm, uint32_t* cell_start,
                        void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (!h->grid_valid) return fail(h, UPSAMPLE_ERR_STATE, "no LR grid built on this handle");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const size_t nl = (size_t)h->grid_n_lr * sizeof(uint32_t);
  if (keys != nullptr && nl) e = hipMemcpyAsync(keys, h->g.keys, nl, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && perm != nullptr && nl)
    e = hipMemcpyAsync(perm, h->g.perm, nl, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && cell_start != nullptr)
    e = hipMemcpyAsync(cell_start, h->g.cell_start, sizeof(uint32_t) * (size_t)(h->n_cells + 1),
                       hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "debug_grid");
  return UPSAMPLE_OK;
}

int upsample_debug_lr_sorted(upsample_handle h, float* x_sorted, float* v_sorted, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (!h->grid_valid) return fail(h, UPSAMPLE_ERR_STATE, "no LR grid built on this handle");
  hipError_t e = launch_unpack_sorted(h->g.lr_sorted, h->grid_n_lr, x_sorted, v_sorted, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(h, e, "debug_lr_sorted");
  return UPSAMPLE_OK;
}

int upsample_debug_neighbors(upsample_handle h, const float* hr_x, const float* hr_v, int64_t n_hr,
                             uint32_t* count, uint32_t* ids, int64_t max_k, uint8_t* branch,
                             void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr > 0 && ids != nullptr && max_k <= 0)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "ids needs max_k > 0");
  // The debug walk writes the stepped state to the handle's HR sort scratch.
  return advance_impl(h, hr_x, hr_v, h->hs.x, h->hs.v, n_hr, stream, 1, count, ids, max_k, branch);
}

int upsample_debug_step_members(upsample_handle h, const float* hr_x, const float* hr_v, float* hr_x_out,
                                float* hr_v_out, int64_t n_hr, uint32_t* count, uint32_t* ids, int64_t max_k,
                                uint32_t* count_w, float* w_disagree, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr > 0 && ids != nullptr && max_k <= 0)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "ids needs max_k > 0");
  return advance_impl(h, hr_x, hr_v, hr_x_out, hr_v_out, n_hr, stream, 2, count, ids, max_k, nullptr, nullptr,
                      nullptr, count_w, w_disagree);
}

int upsample_set_tuning(upsample_handle h, const upsample_tuning* t) {
  if (h == nullptr || t == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (t->gather_groups != 1 && t->gather_groups != 2 && t->gather_groups != 4)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "gather_groups must be 1, 2 or 4");
  if (t->sort_sub != 1 && t->sort_sub != 2 && t->sort_sub != 4)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "sort_sub must be 1, 2 or 4");
  if (t->sort_mode != 0 && t->sort_mode != 1 && t->sort_mode != 2)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "sort_mode must be 0, 1 or 2");
  if (t->tile_max < 0 || t->adjoint_tile_max < 0)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "tile_max must be >= 0");
  if (t->adjoint_tiled != 0 && t->adjoint_tiled != 1)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "adjoint_tiled must be 0 or 1");
  if (t->wall_cull != 0 && t->wall_cull != 1)
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "wall_cull must be 0 or 1");
  if (t->sort_sub > h->hs.max_sub ||
      (h->p.max_hr > 0 && h->hs.max_sub > 0 && sort_bins(h->gi.dims, t->sort_sub, t->sort_mode) > h->hs.n_bins))
    return fail(h, UPSAMPLE_ERR_INVALID_ARG, "sort_sub / sort_mode exceed the bins allocated for this grid");
  h->tune = *t;
  return UPSAMPLE_OK;
}

int upsample_get_tuning(upsample_handle h, upsample_tuning* t) {
  if (h == nullptr || t == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  *t = h->tune;
  return UPSAMPLE_OK;
}

int upsample_timing_enable(upsample_handle h, int enable) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  hipError_t e = fold_timing(h, h->timed_issued);
  if (e != hipSuccess) return hip_fail(h, e, "timing");
  h->timing = enable != 0;
  h->seg_n = -1;
  h->timed_ms = 0.0;
  h->timed_issued = h->timed_folded = h->timed_launches = 0;
  return UPSAMPLE_OK;
}

int upsample_timing_read(upsample_handle h, double* advance_ms, int64_t* launches) {
  if (h == nullptr || advance_ms == nullptr || launches == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  hipError_t e = fold_timing(h, h->timed_issued);
  if (e != hipSuccess) return hip_fail(h, e, "timing");
  *advance_ms = h->timed_ms;
  *launches = h->timed_launches;
  h->timed_ms = 0.0;
  h->timed_issued = h->timed_folded = h->timed_launches = 0;
  return UPSAMPLE_OK;
}

}  // extern "C"
