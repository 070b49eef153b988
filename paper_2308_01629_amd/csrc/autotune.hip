// Autotuner: measures the step kernel on the caller's particles for candidate
// cell factors (kappa, cs = kappa * h) and launch knobs, and returns the
// fastest setting; results are cached in a JSON-lines file keyed by the
// device and the problem's signature.  Built on the public entry points: a
// temporary handle per kappa, a reordered copy of the HR state, HIP events
// around upsample_advance.  Off the timed path of any step.
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace {

constexpr float kKappas[] = {0.51f, 0.6f, 0.75f, UPSAMPLE_DEFAULT_CELL_FACTOR, 1.25f};
// HR reorder keys tried: (sub-cells per axis, key mode)
constexpr int kSorts[][2] = {{1, 2}, {2, 2}, {2, 0}};
constexpr int kGroups[] = {1, 2};
constexpr int kTileMax[] = {384, 512, 768};
constexpr int kReps = 2;

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t k = 0; k < n; ++k) {
    h ^= c[k];
    h *= 1099511628211ull;
  }
  return h;
}

// Signature: device architecture, counts, and every parameter that shapes the
// grid or the work (the wall table included).
std::string make_key(const upsample_params* p, int64_t n_lr, int64_t n_frames, int64_t n_hr, bool rigid,
                     int device) {
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  (void)hipGetDeviceProperties(&prop, device);
  uint64_t h = 1469598103934665603ull;
  const float f[] = {p->r_lr, p->r_hr, p->dt, p->g[0], p->g[1], p->g[2], p->c1, p->c2,
                     p->domain_lo[0], p->domain_lo[1], p->domain_lo[2],
                     p->domain_hi[0], p->domain_hi[1], p->domain_hi[2]};
  h = fnv1a(h, f, sizeof(f));
  h = fnv1a(h, &n_lr, sizeof(n_lr));
  h = fnv1a(h, &n_frames, sizeof(n_frames));
  h = fnv1a(h, &n_hr, sizeof(n_hr));
  const int32_t nw = p->n_walls, rg = rigid ? 1 : 0;
  h = fnv1a(h, &nw, sizeof(nw));
  h = fnv1a(h, &rg, sizeof(rg));
  if (p->n_walls > 0) h = fnv1a(h, p->walls, sizeof(float) * UPSAMPLE_WALL_FLOATS * (size_t)p->n_walls);
  char buf[128];
  std::snprintf(buf, sizeof(buf), "%s:%016" PRIx64, prop.gcnArchName[0] ? prop.gcnArchName : "hip", h);
  for (char* c = buf; *c; ++c)  // the key is a JSON string
    if (*c == '"' || *c == '\\') *c = '_';
  return std::string(buf);
}

bool field(const std::string& line, const char* name, double* out) {
  const std::string pat = std::string("\"") + name + "\": ";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  return std::sscanf(line.c_str() + at + pat.size(), "%lf", out) == 1;
}

bool cache_lookup(const char* path, const std::string& key, upsample_autotune_result* r) {
  if (path == nullptr) return false;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return false;
  const std::string kpat = "\"key\": \"" + key + "\"";
  char buf[1024];
  bool found = false;
  while (std::fgets(buf, sizeof(buf), f) != nullptr) {
    const std::string line(buf);
    if (line.find(kpat) == std::string::npos) continue;
    double kf, gg, ss, sm, tm, am, ms;
    if (field(line, "cell_factor", &kf) && field(line, "gather_groups", &gg) && field(line, "sort_sub", &ss) &&
        field(line, "sort_mode", &sm) && field(line, "tile_max", &tm) && field(line, "adjoint_tile_max", &am) &&
        field(line, "advance_ms", &ms)) {
      r->cell_factor = (float)kf;
      r->tuning.gather_groups = (int32_t)gg;
      r->tuning.sort_sub = (int32_t)ss;
      r->tuning.sort_mode = (int32_t)sm;
      r->tuning.tile_max = (int32_t)tm;
      r->tuning.adjoint_tile_max = (int32_t)am;
      r->tuning.adjoint_tiled = 1;
      r->tuning.wall_cull = 1;
      r->advance_ms = (float)ms;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_append(const char* path, const std::string& key, const upsample_autotune_result& r) {
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "a");
  if (f == nullptr) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"cell_factor\": %.9g, \"gather_groups\": %d, \"sort_sub\": %d, "
               "\"sort_mode\": %d, \"tile_max\": %d, \"adjoint_tile_max\": %d, \"advance_ms\": %.6g}\n",
               key.c_str(), (double)r.cell_factor, r.tuning.gather_groups, r.tuning.sort_sub, r.tuning.sort_mode,
               r.tuning.tile_max, r.tuning.adjoint_tile_max, (double)r.advance_ms);
  std::fclose(f);
}

struct Buffers {
  float* x = nullptr;   // reordered copy of the HR state
  float* v = nullptr;
  float* ox = nullptr;  // step outputs
  float* ov = nullptr;
  ~Buffers() {
    for (float* p : {x, v, ox, ov})
      if (p != nullptr) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int upsample_autotune(const upsample_params* p, const float* lr_x, const float* lr_v,
                                 const uint8_t* lr_rigid, int64_t n_lr, int32_t n_frames, const float* hr_x,
                                 const float* hr_v, int64_t n_hr, const char* cache_path, void* stream,
                                 upsample_autotune_result* out) {
  if (p == nullptr || out == nullptr || n_lr < 0 || n_hr < 1 || n_frames < 1 || n_frames > 1024)
    return UPSAMPLE_ERR_INVALID_ARG;
  if ((n_lr > 0 && (lr_x == nullptr || lr_v == nullptr)) || hr_x == nullptr || hr_v == nullptr)
    return UPSAMPLE_ERR_INVALID_ARG;
  upsample_grid_info gi;
  std::string why;
  int rc = ups::check_scene_params(p, &gi, &why);
  if (rc != UPSAMPLE_OK) return rc;
  int ndev = 0, device = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || hipGetDevice(&device) != hipSuccess)
    return UPSAMPLE_ERR_NO_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const std::string key = make_key(p, n_lr, n_frames, n_hr, lr_rigid != nullptr, device);
  std::memset(out, 0, sizeof(*out));
  if (cache_lookup(cache_path, key, out)) {
    out->from_cache = 1;
    return UPSAMPLE_OK;
  }

  Buffers buf;
  const size_t bytes = sizeof(float) * 3 * (size_t)n_hr;
  if (hipMalloc((void**)&buf.x, bytes) != hipSuccess || hipMalloc((void**)&buf.v, bytes) != hipSuccess ||
      hipMalloc((void**)&buf.ox, bytes) != hipSuccess || hipMalloc((void**)&buf.ov, bytes) != hipSuccess)
    return UPSAMPLE_ERR_OOM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return UPSAMPLE_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return UPSAMPLE_ERR_HIP;
  }

  bool have = false;
  upsample_autotune_result best;
  std::memset(&best, 0, sizeof(best));
  int status = UPSAMPLE_OK;
  for (float kappa : kKappas) {
    upsample_params q = *p;
    q.cell_factor = kappa;
    q.max_lr = n_lr;
    q.max_hr = n_hr;
    q.flags = 0;
    upsample_handle h = nullptr;
    rc = upsample_init(&q, &h);
    if (rc == UPSAMPLE_ERR_GRID_TOO_LARGE || rc == UPSAMPLE_ERR_INVALID_ARG) continue;  // kappa not usable here
    if (rc != UPSAMPLE_OK) {
      status = rc;
      break;
    }
    upsample_tuning t;
    upsample_get_tuning(h, &t);
    const upsample_tuning t0 = t;
    for (const auto& sort : kSorts) {
      if (rc != UPSAMPLE_OK) break;
      t = t0;
      t.sort_sub = sort[0];
      t.sort_mode = sort[1];
      if (upsample_set_tuning(h, &t) != UPSAMPLE_OK) continue;  // more bins than this grid allows
      // (groups, tile_max) combos; times summed over the frames
      constexpr int kCombos = sizeof(kGroups) / sizeof(int) * (sizeof(kTileMax) / sizeof(int));
      float total[kCombos];
      for (int c = 0; c < kCombos; ++c) total[c] = 0.0f;
      for (int32_t f = 0; f < n_frames && rc == UPSAMPLE_OK; ++f) {
        const size_t off = (size_t)f * 3 * (size_t)n_lr;
        rc = upsample_build_grid(h, lr_x + off, lr_v + off, lr_rigid, n_lr, stream);
        if (rc == UPSAMPLE_OK && f == 0) {
          // the reorder a run performs at the start of the interval
          rc = upsample_sort_hr(h, hr_x, hr_v, buf.x, buf.v, n_hr, nullptr, stream);
          if (rc == UPSAMPLE_ERR_GRID_TOO_LARGE) {
            rc = UPSAMPLE_OK;  // no reorder possible: time the caller's order
            if (hipMemcpyAsync(buf.x, hr_x, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(buf.v, hr_v, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
              rc = UPSAMPLE_ERR_HIP;
          }
        }
        int c = 0;
        for (int g : kGroups) {
          for (int tm : kTileMax) {
            if (rc != UPSAMPLE_OK) break;
            t.gather_groups = g;
            t.tile_max = tm;
            rc = upsample_set_tuning(h, &t);
            if (rc == UPSAMPLE_OK) rc = upsample_advance(h, buf.x, buf.v, buf.ox, buf.ov, n_hr, stream);  // warm-up
            float ms_best = 1e30f;
            for (int k = 0; k < kReps && rc == UPSAMPLE_OK; ++k) {
              float ms = 0.0f;
              if (hipEventRecord(e0, st) != hipSuccess) rc = UPSAMPLE_ERR_HIP;
              if (rc == UPSAMPLE_OK) rc = upsample_advance(h, buf.x, buf.v, buf.ox, buf.ov, n_hr, stream);
              if (rc == UPSAMPLE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = UPSAMPLE_ERR_HIP;
              if (rc == UPSAMPLE_OK && ms < ms_best) ms_best = ms;
            }
            total[c++] += ms_best;
          }
        }
        // carry the state along the trajectory (results do not depend on the knobs)
        if (rc == UPSAMPLE_OK && f + 1 < n_frames) rc = upsample_advance(h, buf.x, buf.v, buf.x, buf.v, n_hr, stream);
      }
      int c = 0;
      for (int g : kGroups) {
        for (int tm : kTileMax) {
          const float ms = total[c++] / (float)n_frames;
          if (rc == UPSAMPLE_OK && (!have || ms < best.advance_ms)) {
            have = true;
            best.cell_factor = kappa;
            best.tuning = t;
            best.tuning.gather_groups = g;
            best.tuning.tile_max = tm;
            best.advance_ms = ms;
          }
        }
      }
    }
    upsample_destroy(h);
    if (rc != UPSAMPLE_OK) {
      status = rc;
      break;
    }
  }
  (void)hipStreamSynchronize(st);  // the work on the scratch buffers has ended before they are freed
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != UPSAMPLE_OK) return status;
  if (!have) return UPSAMPLE_ERR_GRID_TOO_LARGE;  // no candidate grid fits
  *out = best;
  out->from_cache = 0;
  cache_append(cache_path, key, best);
  return UPSAMPLE_OK;
}
