// The upsampling step proper (Section 4): per HR particle, a walk over the
// (2R+1)^3 cell stencil of the LR grid accumulating the kernel-weighted sums,
// then the blend parameter, the gravity blend, symplectic Euler and the walls,
// all in one kernel so each HR particle is read once and written once.
//
// HR state is structure-of-arrays float32 [3][n]: lanes of a wave read and
// write consecutive floats (six fully coalesced 256-byte accesses per wave
// each way).  Along x the cells of one (y, z) row of the stencil are adjacent
// keys, so each row is one contiguous range of the sorted LR copy.
#include "kernels.hpp"

namespace ups {
namespace {

struct Sums {
  float S, Ux, Uy, Uz, M;
  bool gran;
  uint32_t count;
};

// Walk the stencil of HR position (x, y, z); accumulate members (float32
// predicate s < h2).  DEBUG also records member ids.
template <bool DEBUG>
__device__ __forceinline__ Sums gather(const GridConst& gc, const LRPoint* __restrict__ lr,
                                       const uint32_t* __restrict__ cell_start, float x, float y,
                                       float z, uint32_t* ids, int64_t max_k) {
  Sums r{0.f, 0.f, 0.f, 0.f, 0.f, false, 0u};
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
        const float s = sq_dist(P.x, P.y, P.z, x, y, z);
        if (s < gc.h2) {
          const float4 V = lr[j].v;
          const float t = fmaxf(fmaf(-s, gc.inv_h2, 1.0f), 0.0f);
          const float w = t * t * t;
          r.S += w;
          r.Ux = fmaf(w, V.x, r.Ux);
          r.Uy = fmaf(w, V.y, r.Uy);
          r.Uz = fmaf(w, V.z, r.Uz);
          r.M = fmaxf(r.M, w);
          r.gran |= (P.w == 0.0f);
          if (DEBUG) {
            if (ids != nullptr && (int64_t)r.count < max_k) ids[r.count] = __float_as_uint(V.w);
          }
          r.count += 1u;
        }
      }
    }
  }
  // Rigid LR particles count only next to a granular one (Section 4).
  if (!r.gran) {
    r.S = 0.f;
    r.Ux = r.Uy = r.Uz = 0.f;
    r.M = 0.f;
  }
  return r;
}

__device__ __forceinline__ void apply_walls(const WallTable& wt, int n_walls, float r_hr, float ox,
                                            float oy, float oz, float& x, float& y, float& z,
                                            float& vx, float& vy, float& vz) {
  for (int k = 0; k < n_walls; ++k) {
    const float* w = &wt.w[k * UPSAMPLE_WALL_FLOATS];
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
      }
    }
  }
}

// Shepard average, blend, symplectic Euler and walls for one HR particle.
__device__ __forceinline__ void finish(const AdvanceArgs& a, const WallTable& wt, int64_t i, float x,
                                      float y, float z, float vx, float vy, float vz, float S,
                                      float Ux, float Uy, float Uz, float M, bool* A_out) {
  // Shepard average and blend parameter (Section 4); empty support -> v~ = 0, alpha = 1.
  float tx = 0.f, ty = 0.f, tz = 0.f;
  bool A = true;
  if (S > 0.0f) {
    tx = Ux / S;
    ty = Uy / S;
    tz = Uz / S;
    A = (M <= a.sc.c1) || (M / S >= a.sc.c2);
  }
  const float alpha = A ? 1.0f - M : 0.0f;
  const float dt = a.sc.dt;
  const float fx = fmaf(dt, a.sc.g[0], vx), fy = fmaf(dt, a.sc.g[1], vy), fz = fmaf(dt, a.sc.g[2], vz);
  float nvx = fmaf(alpha, fx - tx, tx), nvy = fmaf(alpha, fy - ty, ty), nvz = fmaf(alpha, fz - tz, tz);
  float nx = fmaf(dt, nvx, x), ny = fmaf(dt, nvy, y), nz = fmaf(dt, nvz, z);
  apply_walls(wt, a.sc.n_walls, a.sc.r_hr, x, y, z, nx, ny, nz, nvx, nvy, nvz);
  const int64_t n = a.n;
  a.hx_out[i] = nx;
  a.hx_out[n + i] = ny;
  a.hx_out[2 * n + i] = nz;
  a.hv_out[i] = nvx;
  a.hv_out[n + i] = nvy;
  a.hv_out[2 * n + i] = nvz;
  *A_out = A;
}

// Per-lane walk (exact predicate): debug exports and waves whose particles are
// too spread out for a shared candidate list.
template <bool DEBUG>
__global__ __launch_bounds__(kBlock) void k_advance(AdvanceArgs a, WallTable wt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  uint32_t* ids = (DEBUG && a.dbg_ids != nullptr) ? a.dbg_ids + i * a.dbg_max_k : nullptr;
  const Sums s = gather<DEBUG>(a.gc, a.lr, a.cell_start, x, y, z, ids, a.dbg_max_k);
  bool A;
  finish(a, wt, i, x, y, z, vx, vy, vz, s.S, s.Ux, s.Uy, s.Uz, s.M, &A);
  if (DEBUG) {
    if (a.dbg_count != nullptr) a.dbg_count[i] = s.count;
    if (a.dbg_branch != nullptr)
      a.dbg_branch[i] = (uint8_t)((A ? 1 : 0) | (s.gran ? 2 : 0) | (s.S > 0.0f ? 4 : 0));
  }
}

// ---------------------------------------------------------------------------
// Wave-tiled gather.  A wave holds 64 consecutive HR particles, kept spatially
// compact by the HR reorder, as G groups of 64/G lanes (G = 1, 2 or 4; a group
// is one or more 16-lane DPP rows).
// The LR particles of the cells in the union of the lanes' stencils are
// streamed through the wave once; each is kept in a group's LDS list when its
// distance to that group's bounding box is below the support.  Every lane
// then walks its group's list with (four-address) broadcast LDS reads:
//     d = X_j - x_i,  t = 1 - |d|^2 / h^2,  w = max(t, 0)^3.
// Lists are padded to a common length with far-away dummies (w = 0).
// ---------------------------------------------------------------------------

constexpr int kWaves = kBlock / 64;
constexpr int kListBytes = 8192;  // LDS per wave for the candidate lists (32 B per entry)

// Order-preserving map float -> int (non-NaN), an involution.
__device__ __forceinline__ int ord(float f) {
  const int i = __float_as_int(f);
  return i ^ ((i >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float unord(int i) { return __int_as_float(i ^ ((i >> 31) & 0x7fffffff)); }

// Min / max over each 16-lane row; lane 15 of the row holds the result.
__device__ __forceinline__ int row_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x111, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x112, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x114, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x118, 0xf, 0xf, false));
  return v;
}
__device__ __forceinline__ int row_max(int v) {
  const int lo = (int)0x80000000;
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x118, 0xf, 0xf, false));
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Box {
  float lo[3], hi[3];
};

// Squared distance from point p to box b (0 inside).
__device__ __forceinline__ float box_dist2(const Box& b, float px, float py, float pz) {
  const float dx = fmaxf(fmaxf(b.lo[0] - px, px - b.hi[0]), 0.0f);
  const float dy = fmaxf(fmaxf(b.lo[1] - py, py - b.hi[1]), 0.0f);
  const float dz = fmaxf(fmaxf(b.lo[2] - pz, pz - b.hi[2]), 0.0f);
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

template <bool RIGID, int G>
__global__ __launch_bounds__(kBlock) void k_advance_tiled(AdvanceArgs a, WallTable wt) {
  constexpr int kGroups = G;
  constexpr int kListCap = kListBytes / 32 / G;      // entries per group list
  constexpr int kRowsPerGroup = 4 / G;               // 16-lane rows per group
  __shared__ float4 s_p[kWaves][kGroups][kListCap];  // (X_j, sorted index | rigid << 31)
  __shared__ float4 s_v[kWaves][kGroups][kListCap];  // (V_j, unused)
  __shared__ uint32_t s_rb[kWaves][64];              // first sorted index of each stencil row
  __shared__ uint32_t s_rp[kWaves][65];              // exclusive prefix of row lengths

  const int lane = threadIdx.x & 63;
  const int grp = lane / (64 / G);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n = a.n;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool live = i0 < n;
  const int64_t i = live ? i0 : n - 1;  // idle lanes shadow the last particle
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  const GridConst& gc = a.gc;

  // group boxes (per 16-lane row), then the wave box
  const int e0 = row_min(ord(x)), e1 = row_min(ord(y)), e2 = row_min(ord(z));
  const int f0 = row_max(ord(x)), f1 = row_max(ord(y)), f2 = row_max(ord(z));
  Box gb[kGroups];
  int w0x = 0x7fffffff, w0y = 0x7fffffff, w0z = 0x7fffffff;
  int w1x = (int)0x80000000, w1y = (int)0x80000000, w1z = (int)0x80000000;
#pragma unroll
  for (int g = 0; g < kGroups; ++g) {
    int a0 = 0x7fffffff, a1 = 0x7fffffff, a2 = 0x7fffffff;
    int b0 = (int)0x80000000, b1 = (int)0x80000000, b2 = (int)0x80000000;
#pragma unroll
    for (int r = 0; r < kRowsPerGroup; ++r) {
      const int l = 16 * (g * kRowsPerGroup + r) + 15;
      a0 = min(a0, __builtin_amdgcn_readlane(e0, l));
      a1 = min(a1, __builtin_amdgcn_readlane(e1, l));
      a2 = min(a2, __builtin_amdgcn_readlane(e2, l));
      b0 = max(b0, __builtin_amdgcn_readlane(f0, l));
      b1 = max(b1, __builtin_amdgcn_readlane(f1, l));
      b2 = max(b2, __builtin_amdgcn_readlane(f2, l));
    }
    gb[g].lo[0] = unord(a0); gb[g].lo[1] = unord(a1); gb[g].lo[2] = unord(a2);
    gb[g].hi[0] = unord(b0); gb[g].hi[1] = unord(b1); gb[g].hi[2] = unord(b2);
    w0x = min(w0x, a0); w0y = min(w0y, a1); w0z = min(w0z, a2);
    w1x = max(w1x, b0); w1y = max(w1y, b1); w1z = max(w1z, b2);
  }
  // cell coordinates are monotone in position: the cells of the wave box
  // corners bound every lane's cell
  const int R = gc.reach;
  const int X0 = max(cell_coord(unord(w0x), gc.lo[0], gc.inv_cs, gc.dims[0]) - R, 0);
  const int X1 = min(cell_coord(unord(w1x), gc.lo[0], gc.inv_cs, gc.dims[0]) + R, gc.dims[0] - 1);
  const int Y0 = max(cell_coord(unord(w0y), gc.lo[1], gc.inv_cs, gc.dims[1]) - R, 0);
  const int Y1 = min(cell_coord(unord(w1y), gc.lo[1], gc.inv_cs, gc.dims[1]) + R, gc.dims[1] - 1);
  const int Z0 = max(cell_coord(unord(w0z), gc.lo[2], gc.inv_cs, gc.dims[2]) - R, 0);
  const int Z1 = min(cell_coord(unord(w1z), gc.lo[2], gc.inv_cs, gc.dims[2]) + R, gc.dims[2] - 1);
  const int ny = Y1 - Y0 + 1;
  const int nrows = ny * (Z1 - Z0 + 1);

  float S = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, M = 0.f;
  bool gran = !RIGID;
  if (nrows > 64) {
    // spread-out wave: every lane walks its own stencil
    const Sums s = gather<false>(gc, a.lr, a.cell_start, x, y, z, nullptr, 0);
    S = s.S; Ux = s.Ux; Uy = s.Uy; Uz = s.Uz; M = s.M;
    gran = true;  // gather() already applied the rigid rule
  } else {
    // one stencil row per lane: sorted range [rb, rb + rl)
    uint32_t rb = 0, rl = 0;
    if (lane < nrows) {
      const int yy = Y0 + lane % ny, zz = Z0 + lane / ny;
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      rb = a.cell_start[row + (uint32_t)X0];
      rl = a.cell_start[row + (uint32_t)X1 + 1u] - rb;
    }
    const uint32_t incl = wave_incl_scan(rl, lane);
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    s_rb[wid][lane] = rb;
    s_rp[wid][lane + 1] = incl;
    if (lane == 0) s_rp[wid][0] = 0u;
    wave_lds_sync();

    const float inv_h2 = gc.inv_h2;
    const float cull2 = gc.h2 * 1.001f;
    const float4 far_p = make_float4(3.0e38f, 3.0e38f, 3.0e38f, 0.0f);
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);

    uint32_t cnt[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) cnt[g] = 0u;
    for (uint32_t k0 = 0; k0 < total; k0 += 64u) {
      // -- stage: one candidate per lane, kept per group
      const uint32_t k = k0 + (uint32_t)lane;
      bool keep[kGroups];
#pragma unroll
      for (int g = 0; g < kGroups; ++g) keep[g] = false;
      float4 P = zero4, V = zero4;
      uint32_t j = 0;
      if (k < total) {
        int lo = 0, hi = nrows;  // largest row r with s_rp[r] <= k
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_rp[wid][mid] <= k) lo = mid; else hi = mid;
        }
        j = s_rb[wid][lo] + (k - s_rp[wid][lo]);
        P = a.lr[j].p;
        V = a.lr[j].v;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) keep[g] = box_dist2(gb[g], P.x, P.y, P.z) <= cull2;
      }
      const float4 pj = make_float4(P.x, P.y, P.z, __uint_as_float(j | (P.w != 0.0f ? 0x80000000u : 0u)));
      uint32_t nmax = 0;
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        const uint64_t m = __ballot(keep[g]);
        if (keep[g]) {
          const uint32_t pos = cnt[g] + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          s_p[wid][g][pos] = pj;
          s_v[wid][g][pos] = V;
        }
        cnt[g] += (uint32_t)__popcll(m);
        nmax = max(nmax, cnt[g]);
      }
      if (nmax + 64u <= (uint32_t)kListCap && k0 + 64u < total) continue;  // room for another pass
      // pad the shorter lists with far-away dummies
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        for (uint32_t q = cnt[g] + (uint32_t)lane; q < nmax; q += 64u) {
          s_p[wid][g][q] = far_p;
          s_v[wid][g][q] = zero4;
        }
      }
      wave_lds_sync();
      // -- accumulate: each lane walks its group's list
      const uint32_t nc = __builtin_amdgcn_readfirstlane(nmax);
      const float4* lp = &s_p[wid][grp][0];
      const float4* lv = &s_v[wid][grp][0];
      for (uint32_t c = 0; c < nc; ++c) {
        const float4 Q = lp[c];
        const float4 W = lv[c];
        const float dx = Q.x - x, dy = Q.y - y, dz = Q.z - z;
        const float sq = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float u = fmaxf(fmaf(-sq, inv_h2, 1.0f), 0.0f);
        const float w = u * u * u;
        S += w;
        Ux = fmaf(w, W.x, Ux);
        Uy = fmaf(w, W.y, Uy);
        Uz = fmaf(w, W.z, Uz);
        M = fmaxf(M, w);
        if (RIGID) {
          const uint32_t bits = __float_as_uint(Q.w);
          // exact membership of a granular LR particle decides the rigid rule
          if ((bits & 0x80000000u) == 0u && Q.x < 1.0e38f) gran |= sq_dist(Q.x, Q.y, Q.z, x, y, z) < gc.h2;
        }
      }
#pragma unroll
      for (int g = 0; g < kGroups; ++g) cnt[g] = 0u;
      wave_lds_sync();
    }
    if (RIGID && !gran) {
      S = Ux = Uy = Uz = M = 0.f;
    }
  }
  if (live) {
    bool A;
    finish(a, wt, i, x, y, z, vx, vy, vz, S, Ux, Uy, Uz, M, &A);
  }
}

}  // namespace

hipError_t launch_advance(const AdvanceArgs& a, const WallTable& walls, bool debug, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n + kBlock - 1) / kBlock);
  if (debug)
    hipLaunchKernelGGL(k_advance<true>, dim3(blocks), dim3(kBlock), 0, st, a, walls);
  else if (a.sc.has_rigid)
    hipLaunchKernelGGL((k_advance_tiled<true, 1>), dim3(blocks), dim3(kBlock), 0, st, a, walls);
  else if (a.groups == 4)
    hipLaunchKernelGGL((k_advance_tiled<false, 4>), dim3(blocks), dim3(kBlock), 0, st, a, walls);
  else if (a.groups == 2)
    hipLaunchKernelGGL((k_advance_tiled<false, 2>), dim3(blocks), dim3(kBlock), 0, st, a, walls);
  else
    hipLaunchKernelGGL((k_advance_tiled<false, 1>), dim3(blocks), dim3(kBlock), 0, st, a, walls);
  return hipGetLastError();
}

}  // namespace ups
