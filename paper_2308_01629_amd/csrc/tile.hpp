// Wave tiling shared by the step kernel and its adjoint.
//
// A wave holds 64 consecutive HR particles, kept spatially compact by the HR
// reorder, as G groups of 64/G lanes (G = 1, 2 or 4; a group is one or more
// 16-lane DPP rows).  tile_setup() reduces the lanes' positions to per-group
// bounding boxes and lists the (y, z) rows of the union of the lanes' cell
// stencils; tile_visit() streams the LR particles of those rows through the
// wave (one candidate per lane; each round of 64 finds its candidates' rows by
// a prefix maximum over row-start marks) and keeps a candidate in a group's
// LDS list when its distance to the group's box
// is below the support (a conservative test: every LR particle within the
// support of some lane of the group is kept).  Lists are handed to the caller's
// visitor in chunks, padded to a common length with far-away dummies whose
// weight is exactly 0, so every lane of the wave walks the same number of
// entries with broadcast LDS reads.
#pragma once

#include "common.hpp"

namespace ups {

constexpr int kWaves = kBlock / 64;

// Order-preserving map float -> int (non-NaN); an involution.
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

// Min / max over each group of 64 / G lanes (G = 1, 2, 4): the row reduction,
// then the row broadcasts of lanes 15 and 31; the group's last lane holds it.
template <int G>
__device__ __forceinline__ int group_min(int v) {
  v = row_min(v);
  if (G <= 2) v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x142, 0xa, 0xf, false));
  if (G == 1) v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x143, 0xc, 0xf, false));
  return v;
}
template <int G>
__device__ __forceinline__ int group_max(int v) {
  const int lo = (int)0x80000000;
  v = row_max(v);
  if (G <= 2) v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x142, 0xa, 0xf, false));
  if (G == 1) v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x143, 0xc, 0xf, false));
  return v;
}

// Candidates of the longest per-lane walk of the wave: each lane counts its
// own stencil rows (the rows a per-lane walk visits), and the wave takes the
// maximum.  Wave-uniform.
__device__ __forceinline__ uint32_t lane_walk_max(const GridConst& gc, const uint32_t* __restrict__ cell_start,
                                                  float x, float y, float z) {
  const int R = gc.reach;
  const int cx = cell_coord(x, gc.lo[0], gc.inv_cs, gc.dims[0]);
  const int cy = cell_coord(y, gc.lo[1], gc.inv_cs, gc.dims[1]);
  const int cz = cell_coord(z, gc.lo[2], gc.inv_cs, gc.dims[2]);
  const int x0 = max(cx - R, 0), x1 = min(cx + R, gc.dims[0] - 1);
  const int y0 = max(cy - R, 0), y1 = min(cy + R, gc.dims[1] - 1);
  const int z0 = max(cz - R, 0), z1 = min(cz + R, gc.dims[2] - 1);
  uint32_t s = 0u;
  for (int zz = z0; zz <= z1; ++zz)
    for (int yy = y0; yy <= y1; ++yy) {
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      s += cell_start[row + (uint32_t)x1 + 1u] - cell_start[row + (uint32_t)x0];
    }
  return (uint32_t)__builtin_amdgcn_readlane(group_max<1>((int)s), 63);
}

// Inclusive prefix maximum over the wave (DPP row shifts, then the row
// broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_prefix_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return v;
}

// Inclusive prefix sum over the wave, in the same DPP pattern (lanes whose
// source lies outside the row, and rows outside the mask, add 0).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
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

// LDS of the wave tiles of one block of Waves waves: Cap list entries per
// group (32 B each) and up to Rows stencil rows per wave (a multiple of 64; a
// wave with more rows takes the per-lane walk).
template <int G, int Cap, int Rows, int Waves = kWaves>
struct TileLDS {
  static constexpr int kCap = Cap;
  static constexpr int kRows = Rows;
  static_assert(Rows % 64 == 0 && Rows <= 256, "rows are scanned 64 at a time");
  // one streaming pass appends up to 64 candidates to every group list
  static_assert(Cap >= 64, "a group list must hold one full pass");
  float4 p[Waves][G][kCap];  // (X_j, sorted index | rigid << 31)
  float4 v[Waves][G][kCap];  // (V_j, original index as bits)
  uint32_t rb[Waves][kRows];      // first sorted index of each stencil row
  uint32_t rp[Waves][kRows + 1];  // exclusive prefix of row lengths
  uint32_t mark[Waves][64];       // streaming: row starting at each position of a round
};

template <int G>
struct TileSetup {
  Box gb[G];
  int nrows;       // > the LDS row capacity: the wave is too spread out for a shared list
  uint32_t total;  // candidates streamed (sum of row lengths)
  int X0, Y0, Z0, ny;  // first cell of the rows; rows run y-fastest
  int bx0, bx1, by0, by1, bz0, bz1;  // cells of the wave box's corners
  uint32_t my_start, my_len;  // row `lane` (rows <= 64): first streamed index and length
};

// Group boxes, stencil rows and their prefix sums (rows only when nrows fits the LDS).
template <int G, class L>
__device__ __forceinline__ TileSetup<G> tile_setup(const GridConst& gc,
                                                   const uint32_t* __restrict__ cell_start, float x,
                                                   float y, float z, int lane, int wid, L& lds) {
  static_assert(G == 1 || G == 2 || G == 4, "groups are 64, 32 or 16 lanes");
  TileSetup<G> ts;
  const int e0 = group_min<G>(ord(x)), e1 = group_min<G>(ord(y)), e2 = group_min<G>(ord(z));
  const int f0 = group_max<G>(ord(x)), f1 = group_max<G>(ord(y)), f2 = group_max<G>(ord(z));
  int w0x = 0x7fffffff, w0y = 0x7fffffff, w0z = 0x7fffffff;
  int w1x = (int)0x80000000, w1y = (int)0x80000000, w1z = (int)0x80000000;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int l = (64 / G) * (g + 1) - 1;
    const int a0 = __builtin_amdgcn_readlane(e0, l);
    const int a1 = __builtin_amdgcn_readlane(e1, l);
    const int a2 = __builtin_amdgcn_readlane(e2, l);
    const int b0 = __builtin_amdgcn_readlane(f0, l);
    const int b1 = __builtin_amdgcn_readlane(f1, l);
    const int b2 = __builtin_amdgcn_readlane(f2, l);
    ts.gb[g].lo[0] = unord(a0); ts.gb[g].lo[1] = unord(a1); ts.gb[g].lo[2] = unord(a2);
    ts.gb[g].hi[0] = unord(b0); ts.gb[g].hi[1] = unord(b1); ts.gb[g].hi[2] = unord(b2);
    w0x = min(w0x, a0); w0y = min(w0y, a1); w0z = min(w0z, a2);
    w1x = max(w1x, b0); w1y = max(w1y, b1); w1z = max(w1z, b2);
  }
  // Cell coordinates are monotone in position: the cells of the wave box
  // corners bound every lane's cell, so these rows hold every lane's stencil.
  const int R = gc.reach;
  ts.bx0 = cell_coord(unord(w0x), gc.lo[0], gc.inv_cs, gc.dims[0]);
  ts.bx1 = cell_coord(unord(w1x), gc.lo[0], gc.inv_cs, gc.dims[0]);
  ts.by0 = cell_coord(unord(w0y), gc.lo[1], gc.inv_cs, gc.dims[1]);
  ts.by1 = cell_coord(unord(w1y), gc.lo[1], gc.inv_cs, gc.dims[1]);
  ts.bz0 = cell_coord(unord(w0z), gc.lo[2], gc.inv_cs, gc.dims[2]);
  ts.bz1 = cell_coord(unord(w1z), gc.lo[2], gc.inv_cs, gc.dims[2]);
  const int X0 = max(ts.bx0 - R, 0), X1 = min(ts.bx1 + R, gc.dims[0] - 1);
  const int Y0 = max(ts.by0 - R, 0), Y1 = min(ts.by1 + R, gc.dims[1] - 1);
  const int Z0 = max(ts.bz0 - R, 0), Z1 = min(ts.bz1 + R, gc.dims[2] - 1);
  const int ny = Y1 - Y0 + 1;
  ts.nrows = ny * (Z1 - Z0 + 1);
  ts.total = 0u;
  ts.X0 = X0;
  ts.Y0 = Y0;
  ts.Z0 = Z0;
  ts.ny = ny;
  ts.my_start = 0u;
  ts.my_len = 0u;
  if (ts.nrows > L::kRows) return ts;
  // rows r = lane + 64 q: one wave scan per 64 rows, in row order.  r / ny by
  // a float reciprocal: with r < 256 and ny <= 256, (r + 1/2) / ny lies at
  // least 1/512 from an integer, far beyond the reciprocal's error.
  const float rny = __builtin_amdgcn_rcpf((float)ny);
  uint32_t carry = 0;
#pragma unroll
  for (int q = 0; q < L::kRows / 64; ++q) {
    if (64 * q >= ts.nrows) break;
    const int r = lane + 64 * q;
    uint32_t rb = 0, rl = 0;
    if (r < ts.nrows) {
      const int rz = (int)fmaf((float)r, rny, 0.5f * rny);
      const int yy = Y0 + __mul24(-rz, ny) + r, zz = Z0 + rz;
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      rb = cell_start[row + (uint32_t)X0];
      rl = cell_start[row + (uint32_t)X1 + 1u] - rb;
    }
    const uint32_t incl = wave_incl_scan(rl) + carry;
    lds.rb[wid][r] = rb;
    lds.rp[wid][r + 1] = incl;
    if (q == 0) {
      ts.my_start = incl - rl;
      ts.my_len = rl;
    }
    carry = __builtin_amdgcn_readlane(incl, 63);
  }
  ts.total = carry;
  if (lane == 0) lds.rp[wid][0] = 0u;
  wave_lds_sync();
  return ts;
}

// Default tag stored with a candidate: sorted index | rigid << 31.
struct SortedTag {
  __device__ __forceinline__ uint32_t operator()(int /*row*/, uint32_t /*k*/, uint32_t j, float flag) const {
    return j | (flag != 0.0f ? 0x80000000u : 0u);
  }
};

// Default staging: the candidate's position with its tag; padding entries sit
// far away (weight exactly 0 for every lane).  vel(V) gives the 16 bytes
// stored in the velocity list (by default the LR copy's (V_j, index bits)).
struct PlainStage {
  static constexpr bool kCentred = false;
  __device__ __forceinline__ float4 operator()(float4 P, uint32_t bits) const {
    return make_float4(P.x, P.y, P.z, __uint_as_float(bits));
  }
  __device__ __forceinline__ float4 pad() const { return make_float4(3.0e38f, 3.0e38f, 3.0e38f, 0.0f); }
  __device__ __forceinline__ float4 vel(float4 V, uint32_t /*bits*/) const { return V; }
  __device__ __forceinline__ float4 pad_vel() const { return make_float4(0.f, 0.f, 0.f, 0.f); }
};

// Stream the candidates and hand the LDS lists to visit(nc, p_list, v_list)
// in chunks; p_list / v_list point at this lane's group list.  tag(row, k, j,
// flag) gives the 32 bits stored in the .w of the position entry.
// stage(P, tag) gives the 16 bytes stored for a kept candidate (culling
// always uses its absolute position), stage.vel(V, tag) its velocity entry,
// stage.pad() the padding entry and stage.pad_vel() the padding's velocity
// entry (zero for the step kernels).
// Round > 1 pads every chunk to a multiple of Round entries, so that the
// visitor can unroll by Round with immediate LDS offsets.
// A stage with kCentred carries the wave box's centre (cx, cy, cz) and
// half-extents (hx, hy, hz); with one group the cull then works on
// q = X - c, |q| - half per axis, and stage.centred(P, tag) forms the entry.
template <int G, int Round = 1, class L, class Visit, class Tag = SortedTag, class Stage = PlainStage>
__device__ __forceinline__ void tile_visit(const TileSetup<G>& ts, const GridConst& gc,
                                           const LRPoint* __restrict__ lr, int lane, int wid,
                                           L& lds, Visit&& visit, Tag tag = Tag(), Stage stage = Stage()) {
  constexpr int kCap = L::kCap;
  static_assert(Round >= 1 && kCap % Round == 0, "padded chunks must fit the list");
  static_assert(L::kRows == 64, "the streaming gives each lane one stencil row");
  const int grp = lane / (64 / G);
  const float cull2 = gc.h2 * 1.001f;
  const float4 far_p = stage.pad();
  uint32_t carried = 0u;  // the row holding the round's first candidate
  const float4 pad_v = stage.pad_vel();
  uint32_t cnt[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cnt[g] = 0u;
  for (uint32_t k0 = 0; k0 < ts.total; k0 += 64u) {
    const uint32_t k = k0 + (uint32_t)lane;
    // The row of candidate k is the last non-empty row starting at or before
    // it: each such row marks its start inside this round (non-empty rows
    // start at distinct positions), and a prefix maximum over the lanes
    // spreads the marks.
    lds.mark[wid][lane] = lane == 0 ? carried : 0u;
    wave_lds_sync();
    if (lane < ts.nrows && ts.my_len > 0u && ts.my_start >= k0 && ts.my_start - k0 < 64u)
      lds.mark[wid][ts.my_start - k0] = (uint32_t)lane;
    wave_lds_sync();
    const int lo = (int)wave_prefix_max(lds.mark[wid][lane]);
    carried = __builtin_amdgcn_readlane(lo, 63);
    // Lanes past the last candidate load the last one (its row is the one
    // the prefix maximum gives them) and keep nothing: no branch around the
    // loads.
    const bool valid = k < ts.total;
    const uint32_t kk = valid ? k : ts.total - 1u;
    const uint32_t j = lds.rb[wid][lo] + (kk - lds.rp[wid][lo]);
    const float4 P = lr[j].p;
    const float4 V = lr[j].v;
    // V is stored only by lanes that keep their candidate; taking it here
    // stops the compiler from sinking its load behind the cull, so both
    // loads of the round share one round trip
    asm volatile("" ::"v"(V.x), "v"(V.y), "v"(V.z), "v"(V.w));
    const uint32_t bits = tag(lo, kk, j, P.w);
    bool keep[G];
    float4 pj;
    if constexpr (Stage::kCentred && G == 1) {
      const float qx = P.x - stage.cx, qy = P.y - stage.cy, qz = P.z - stage.cz;
      // max(|q| - half, 0) by the [0, 1] output clamp of the subtraction:
      // capping a distance at 1 only keeps more candidates, and culls the
      // same ones when the support is below 1
      const float dx = __builtin_amdgcn_fmed3f(fabsf(qx) - stage.hx, 0.0f, 1.0f);
      const float dy = __builtin_amdgcn_fmed3f(fabsf(qy) - stage.hy, 0.0f, 1.0f);
      const float dz = __builtin_amdgcn_fmed3f(fabsf(qz) - stage.hz, 0.0f, 1.0f);
      keep[0] = valid & (fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= cull2);  // no branch
      pj = stage.centred(P, bits);
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) keep[g] = valid && box_dist2(ts.gb[g], P.x, P.y, P.z) <= cull2;
      pj = stage(P, bits);
    }
    uint32_t nmax = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint64_t m = __builtin_amdgcn_ballot_w64(keep[g]);
      if (keep[g]) {
        const uint32_t pos = cnt[g] + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        lds.p[wid][g][pos] = pj;
        lds.v[wid][g][pos] = stage.vel(V, bits);
      }
      cnt[g] += (uint32_t)__popcll(m);
      nmax = max(nmax, cnt[g]);
    }
    if (nmax + 64u <= (uint32_t)kCap && k0 + 64u < ts.total) continue;  // room for another pass
    const uint32_t npad = (nmax + (uint32_t)(Round - 1)) / (uint32_t)Round * (uint32_t)Round;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      for (uint32_t q = cnt[g] + (uint32_t)lane; q < npad; q += 64u) {
        lds.p[wid][g][q] = far_p;
        lds.v[wid][g][q] = pad_v;
      }
    }
    wave_lds_sync();
    visit(__builtin_amdgcn_readfirstlane(npad), &lds.p[wid][grp][0], &lds.v[wid][grp][0]);
#pragma unroll
    for (int g = 0; g < G; ++g) cnt[g] = 0u;
    wave_lds_sync();
  }
}

}  // namespace ups
