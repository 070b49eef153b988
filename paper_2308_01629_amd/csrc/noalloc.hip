// upsample_step_noalloc: one upsampling step (Section 4) for callers that
// cannot allocate device memory -- code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc.  It needs no handle: the LR grid's
// scratch lives in one file-scope device array of fixed size, and the call
// enqueues the same grid build and the same step kernel as upsample_step on a
// handle with the default tuning, so the results are bit-identical to it.
//
// The array exists once per device the library runs on and is held until the
// process ends.  In host code its name stands for a host-side shadow, not for
// device memory: its device address is taken once per device with
// hipGetSymbolAddress (the current device at the first call) and only that
// address is handed to kernels.  Every call on a device uses the same array,
// so calls that overlap on one device race on it.
#include <mutex>
#include <string>

#include "kernels.hpp"

namespace ups {
namespace {

constexpr int64_t kNoAllocMaxLR = UPSAMPLE_NOALLOC_MAX_LR;        // LR particles per call
constexpr int64_t kNoAllocMaxCells = UPSAMPLE_NOALLOC_MAX_CELLS;  // grid cells per call
constexpr int kMaxDevices = 64;

constexpr size_t seg(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
constexpr int64_t kMaxChunks = (kNoAllocMaxCells + kScanChunk - 1) / kScanChunk;
// Segments of the scratch array, each 256-byte aligned.
constexpr size_t kOffKeys = 0;
constexpr size_t kOffSlot = kOffKeys + seg(4 * kNoAllocMaxLR);
constexpr size_t kOffTmp = kOffSlot + seg(4 * kNoAllocMaxLR);
constexpr size_t kOffPerm = kOffTmp + seg(4 * kNoAllocMaxLR);
constexpr size_t kOffCounts = kOffPerm + seg(4 * kNoAllocMaxLR);
constexpr size_t kOffLocal = kOffCounts + seg(4 * kNoAllocMaxCells);
constexpr size_t kOffChunk = kOffLocal + seg(4 * kNoAllocMaxCells);
constexpr size_t kOffStart = kOffChunk + seg(4 * (kMaxChunks + 1));
constexpr size_t kOffSorted = kOffStart + seg(4 * (kNoAllocMaxCells + 1));
constexpr size_t kScratchBytes = kOffSorted + seg(sizeof(LRPoint) * kNoAllocMaxLR);  // about 6.3 MB

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of scratch on each device, once taken

// Zero the per-cell counts: the build's scan leaves them zero for the next
// build, but a call that failed part-way may not have.  A kernel, not a
// memset, so that a captured step holds no memset node.
__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace
}  // namespace ups

using namespace ups;

extern "C" int upsample_step_noalloc(const upsample_params* p, const float* lr_x, const float* lr_v,
                                     const uint8_t* lr_rigid, int64_t n_lr, const float* hr_x,
                                     const float* hr_v, float* hr_x_out, float* hr_v_out, int64_t n_hr,
                                     void* stream) {
  upsample_grid_info gi;
  std::string why;
  int rc = check_scene_params(p, &gi, &why);
  if (rc != UPSAMPLE_OK) return rc;
  if ((p->flags & UPSAMPLE_FLAG_VALIDATE) != 0u) return UPSAMPLE_ERR_INVALID_ARG;  // it synchronises
  if (n_lr < 0 || n_hr < 0) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_lr > kNoAllocMaxLR || gi.n_cells > kNoAllocMaxCells) return UPSAMPLE_ERR_CAPACITY;
  if (n_lr > 0 && (lr_x == nullptr || lr_v == nullptr)) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_hr > 0 && (hr_x == nullptr || hr_v == nullptr || hr_x_out == nullptr || hr_v_out == nullptr))
    return UPSAMPLE_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return UPSAMPLE_ERR_NO_DEVICE;
  if (dev >= kMaxDevices) return UPSAMPLE_ERR_NO_DEVICE;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev] == nullptr) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
        return UPSAMPLE_ERR_HIP;
      g_ptr[dev] = ptr;
    }
    base = static_cast<unsigned char*>(g_ptr[dev]);
  }
  GridScratch s;
  s.keys = reinterpret_cast<uint32_t*>(base + kOffKeys);
  s.slot = reinterpret_cast<uint32_t*>(base + kOffSlot);
  s.tmp = reinterpret_cast<uint32_t*>(base + kOffTmp);
  s.perm = reinterpret_cast<uint32_t*>(base + kOffPerm);
  s.counts = reinterpret_cast<uint32_t*>(base + kOffCounts);
  s.local = reinterpret_cast<uint32_t*>(base + kOffLocal);
  s.chunk_sum = reinterpret_cast<uint32_t*>(base + kOffChunk);
  s.cell_start = reinterpret_cast<uint32_t*>(base + kOffStart);
  s.lr_sorted = reinterpret_cast<LRPoint*>(base + kOffSorted);

  hipStream_t st = (hipStream_t)stream;
  const GridConst gc = make_grid_const(gi);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((gi.n_cells + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     s.counts, gi.n_cells);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_build_grid(gc, lr_x, lr_v, lr_rigid, n_lr, gi.n_cells, s, st);
  if (e == hipSuccess && n_hr > 0) {
    AdvanceArgs a;
    a.gc = gc;
    a.sc = make_step_const(*p, lr_rigid != nullptr);
    a.lr = s.lr_sorted;
    a.cell_start = s.cell_start;
    a.hx = hr_x;
    a.hv = hr_v;
    a.hx_out = hr_x_out;
    a.hv_out = hr_v_out;
    a.n = n_hr;
    a.ld = n_hr;
    a.dbg_count = nullptr;
    a.dbg_ids = nullptr;
    a.dbg_max_k = 0;
    a.dbg_branch = nullptr;
    a.dbg_count_w = nullptr;
    a.dbg_wdis = nullptr;
    a.wall_mask = nullptr;  // every wave tests every wall (same results as the per-cell cull)
    a.groups = 1;
    a.tile_max = 512;
    a.tape = nullptr;
    e = launch_advance(a, make_wall_table(p->walls, p->n_walls), 0, st);
  }
  return e == hipSuccess ? UPSAMPLE_OK : UPSAMPLE_ERR_HIP;
}
