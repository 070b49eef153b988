// Adjoint of the upsampling step (an extension: the paper does not
// differentiate it).  Per HR particle: a first pass over the LR neighbours
// recomputes the weighted sums, the argmax of the weights and the alpha
// branch; the forward blend, integration and walls are replayed to record
// which walls acted; the upstream gradient is pulled back through the walls,
// the integration and the blend; a second pass distributes the weight
// gradients to the LR particles and to the HR position.
//
// Held fixed (piecewise differentiation): alpha branch, neighbour membership,
// argmax of w (ties: smallest original LR index), wall activations.
//
// Two kernels share that arithmetic:
//   k_adjoint_tiled  waves of spatially compact HR particles (tile.hpp): each
//                    LR candidate's six gradient components are summed over
//                    the wave with a permlane-swap transpose reduction and added
//                    to global memory by six lanes (two atomic instructions);
//   k_adjoint        one particle per lane, its own stencil walk, atomics per
//                    pair: spread-out waves and scenes with rigid LR particles.
// Deterministic LR gradients take a third route: k_adjoint_det_tiled (the
// tiled HR pass) or k_adjoint_det (per lane) writes each HR particle's
// adjoint coefficients, k_det_sort_coef puts them in the HR grid's sorted
// order, and k_adjoint_det_lr gives every LR
// particle one wave that walks its HR neighbours (HR sorted by cell, stable)
// in a fixed order and reduces over the lanes in a fixed pattern; each LR
// gradient then has one writer and no float atomic is involved.
#include "kernels.hpp"
#include "tile.hpp"

namespace ups {
namespace {

// Per-particle adjoint state between the two passes.
struct Back {
  float gUx, gUy, gUz, gS, gM;  // dL/dU, dL/dS, dL/dM
  float gx, gy, gz;             // dL/dx (direct part; the pair terms are added in pass 2)
  float gvx, gvy, gvz;          // dL/dv
};

// Forward replay of blend, integration and walls, then the pull-back of the
// upstream gradient (gx_out, gv_out) to the sums S, U, M and to x, v.
__device__ __forceinline__ Back backprop(const StepConst& sc, const WallTable& wt, float x, float y,
                                         float z, float vx, float vy, float vz, float S, float Ux,
                                         float Uy, float Uz, float M, float gxo, float gyo, float gzo,
                                         float hxo, float hyo, float hzo) {
  float tx = 0.f, ty = 0.f, tz = 0.f, rS = 0.f;
  bool A = true;
  if (S > 0.0f) {
    rS = __builtin_amdgcn_rcpf(S);  // as in the forward step
    tx = Ux * rS;
    ty = Uy * rS;
    tz = Uz * rS;
    A = (M <= sc.c1) || (M * rS >= sc.c2);
  }
  const float alpha = A ? 1.0f - M : 0.0f;
  const float dt = sc.dt;
  const float fx = fmaf(dt, sc.g[0], vx), fy = fmaf(dt, sc.g[1], vy), fz = fmaf(dt, sc.g[2], vz);
  float nvx = fmaf(alpha, fx - tx, tx), nvy = fmaf(alpha, fy - ty, ty), nvz = fmaf(alpha, fz - tz, tz);
  float nx = fmaf(dt, nvx, x), ny = fmaf(dt, nvy, y), nz = fmaf(dt, nvz, z);
  uint32_t pushed = 0u, clipped = 0u;
  for (int k = 0; k < sc.n_walls; ++k) {
    const float* w = &wt.w[k * UPSAMPLE_WALL_FLOATS];
    const float wnx = w[0], wny = w[1], wnz = w[2], d = w[3];
    const float pen = fmaf(wnz, nz, fmaf(wny, ny, wnx * nx)) - d;
    if (pen < sc.r_hr) {
      bool act = fmaf(w[6], nz, fmaf(w[5], ny, w[4] * nx)) >= w[7];
      if (w[11] > 0.0f) {
        const float rx = nx - w[8], ry = ny - w[9], rz = nz - w[10];
        const float rn = fmaf(wnz, rz, fmaf(wny, ry, wnx * rx));
        const float ix = fmaf(-rn, wnx, rx), iy = fmaf(-rn, wny, ry), iz = fmaf(-rn, wnz, rz);
        act = act && (fmaf(iz, iz, fmaf(iy, iy, ix * ix)) >= w[11] * w[11]);
      }
      act = act && (fmaf(wnz, z, fmaf(wny, y, wnx * x)) - d >= 0.0f);
      if (act) {
        pushed |= 1u << k;
        const float push = sc.r_hr - pen;
        nx = fmaf(push, wnx, nx);
        ny = fmaf(push, wny, ny);
        nz = fmaf(push, wnz, nz);
        const float vn = fmaf(wnz, nvz, fmaf(wny, nvy, wnx * nvx));
        if (vn < 0.0f) {
          clipped |= 1u << k;
          nvx = fmaf(-vn, wnx, nvx);
          nvy = fmaf(-vn, wny, nvy);
          nvz = fmaf(-vn, wnz, nvz);
        }
      }
    }
  }
  // walls, last first: a push or a clip has Jacobian I - n n^T
  float gx = gxo, gy = gyo, gz = gzo, hx = hxo, hy = hyo, hz = hzo;
  for (int k = sc.n_walls - 1; k >= 0; --k) {
    const float* w = &wt.w[k * UPSAMPLE_WALL_FLOATS];
    if (pushed & (1u << k)) {
      const float gn = fmaf(w[2], gz, fmaf(w[1], gy, w[0] * gx));
      gx = fmaf(-gn, w[0], gx);
      gy = fmaf(-gn, w[1], gy);
      gz = fmaf(-gn, w[2], gz);
    }
    if (clipped & (1u << k)) {
      const float hn = fmaf(w[2], hz, fmaf(w[1], hy, w[0] * hx));
      hx = fmaf(-hn, w[0], hx);
      hy = fmaf(-hn, w[1], hy);
      hz = fmaf(-hn, w[2], hz);
    }
  }
  // x' = x + dt v'  ->  dL/dv' += dt dL/dx'
  const float qx = fmaf(dt, gx, hx), qy = fmaf(dt, gy, hy), qz = fmaf(dt, gz, hz);
  // v' = (1 - alpha) v~ + alpha (v + dt g)
  const float g_alpha = qx * (fx - tx) + qy * (fy - ty) + qz * (fz - tz);
  Back b;
  b.gM = A ? -g_alpha : 0.0f;
  b.gUx = b.gUy = b.gUz = b.gS = 0.f;
  if (S > 0.0f) {
    const float om = (1.0f - alpha) * rS;
    b.gUx = om * qx;
    b.gUy = om * qy;
    b.gUz = om * qz;
    b.gS = -(b.gUx * tx + b.gUy * ty + b.gUz * tz);
  }
  b.gx = gx;
  b.gy = gy;
  b.gz = gz;
  b.gvx = alpha * qx;
  b.gvy = alpha * qy;
  b.gvz = alpha * qz;
  return b;
}

__device__ __forceinline__ void stencil_bounds(const GridConst& gc, float x, float y, float z,
                                               int lo[3], int hi[3]) {
  const int c[3] = {cell_coord(x, gc.lo[0], gc.inv_cs, gc.dims[0]),
                    cell_coord(y, gc.lo[1], gc.inv_cs, gc.dims[1]),
                    cell_coord(z, gc.lo[2], gc.inv_cs, gc.dims[2])};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = max(c[a] - gc.reach, 0);
    hi[a] = min(c[a] + gc.reach, gc.dims[a] - 1);
  }
}

// One particle, its own stencil walk, float atomics per member pair.  DET:
// no LR gradient is added; the particle's coefficients (dL/dU, dL/dS, dL/dM,
// argmax bits; zeros when the rigid rule drops its support) go to
// a.det_coef for the LR pass, and only the HR position terms are summed here.
template <bool DET = false>
__device__ __forceinline__ void adjoint_lane(const AdjointArgs& a, const WallTable& wt, int64_t i) {
  const int64_t n = a.n;
  const GridConst& gc = a.gc;
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  int lo[3], hi[3];
  stencil_bounds(gc, x, y, z, lo, hi);

  float S = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, M = 0.f;
  uint32_t arg = 0xffffffffu;
  bool gran = false;
  if (a.tape != nullptr) {
    // the forward's record; a rigid-only support was recorded as zero sums
    S = a.tape[i];
    Ux = a.tape[n + i];
    Uy = a.tape[2 * n + i];
    Uz = a.tape[3 * n + i];
    M = a.tape[4 * n + i];
    arg = __float_as_uint(a.tape[5 * n + i]);
    gran = S > 0.0f;
  } else {
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
      for (int yy = lo[1]; yy <= hi[1]; ++yy) {
        const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
        const uint32_t b = a.cell_start[row + (uint32_t)lo[0]], e = a.cell_start[row + (uint32_t)hi[0] + 1u];
        for (uint32_t j = b; j < e; ++j) {
          const float4 P = a.lr[j].p;
          const float s = sq_dist(P.x, P.y, P.z, x, y, z);
          if (s < gc.h2) {
            const float4 V = a.lr[j].v;
            const float t = fmaxf(fmaf(-s, gc.inv_h2, 1.0f), 0.0f);
            const float w = t * t * t;
            const uint32_t id = __float_as_uint(V.w);
            S += w;
            Ux = fmaf(w, V.x, Ux);
            Uy = fmaf(w, V.y, Uy);
            Uz = fmaf(w, V.z, Uz);
            if (w > M || (w == M && id < arg)) {
              M = w;
              arg = id;
            }
            gran |= (P.w == 0.0f);
          }
        }
      }
    if (!gran) S = Ux = Uy = Uz = M = 0.f;  // rigid LR count only next to a granular one
  }
  Back bk = backprop(a.sc, wt, x, y, z, vx, vy, vz, S, Ux, Uy, Uz, M, a.gx_out[i], a.gx_out[n + i],
                     a.gx_out[2 * n + i], a.gv_out[i], a.gv_out[n + i], a.gv_out[2 * n + i]);
  if (DET) {
    a.det_coef[i] = gran ? bk.gUx : 0.0f;
    a.det_coef[n + i] = gran ? bk.gUy : 0.0f;
    a.det_coef[2 * n + i] = gran ? bk.gUz : 0.0f;
    a.det_coef[3 * n + i] = gran ? bk.gS : 0.0f;
    a.det_coef[4 * n + i] = gran ? bk.gM : 0.0f;
    a.det_coef[5 * n + i] = __uint_as_float(gran ? arg : 0xffffffffu);
  }
  if (gran) {
    const float k2 = -6.0f * gc.inv_h2;  // dw/ds = -3 t^2 / h2, times 2 for ds/dX
    const int64_t nl = a.n_lr;
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
      for (int yy = lo[1]; yy <= hi[1]; ++yy) {
        const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
        const uint32_t b = a.cell_start[row + (uint32_t)lo[0]], e = a.cell_start[row + (uint32_t)hi[0] + 1u];
        for (uint32_t j = b; j < e; ++j) {
          const float4 P = a.lr[j].p;
          const float s = sq_dist(P.x, P.y, P.z, x, y, z);
          if (s < gc.h2) {
            const float4 V = a.lr[j].v;
            const uint32_t id = __float_as_uint(V.w);
            const float t = fmaxf(fmaf(-s, gc.inv_h2, 1.0f), 0.0f);
            const float w = t * t * t;
            float gw = fmaf(bk.gUz, V.z, fmaf(bk.gUy, V.y, bk.gUx * V.x)) + bk.gS;
            if (id == arg) gw += bk.gM;
            const float c = gw * k2 * t * t;
            const float dx = P.x - x, dy = P.y - y, dz = P.z - z;
            if (!DET) {
              unsafeAtomicAdd(&a.g_lr_v[id], w * bk.gUx);
              unsafeAtomicAdd(&a.g_lr_v[nl + id], w * bk.gUy);
              unsafeAtomicAdd(&a.g_lr_v[2 * nl + id], w * bk.gUz);
              unsafeAtomicAdd(&a.g_lr_x[id], c * dx);
              unsafeAtomicAdd(&a.g_lr_x[nl + id], c * dy);
              unsafeAtomicAdd(&a.g_lr_x[2 * nl + id], c * dz);
            }
            bk.gx = fmaf(-c, dx, bk.gx);
            bk.gy = fmaf(-c, dy, bk.gy);
            bk.gz = fmaf(-c, dz, bk.gz);
          }
        }
      }
  }
  a.gx_in[i] = bk.gx;
  a.gx_in[n + i] = bk.gy;
  a.gx_in[2 * n + i] = bk.gz;
  a.gv_in[i] = bk.gvx;
  a.gv_in[n + i] = bk.gvy;
  a.gv_in[2 * n + i] = bk.gvz;
}

__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a, WallTable wt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  adjoint_lane(a, wt, i);
}

__global__ __launch_bounds__(kBlock) void k_adjoint_det(AdjointArgs a, WallTable wt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  adjoint_lane<true>(a, wt, i);
}

// The HR coefficients in the HR grid's sorted order, so that the LR pass
// reads them with the sorted positions instead of by original index: slot q
// of the sorted copy gets (dL/dU, dL/dS) in v and the argmax bits in p.w
// (its velocity and flag are not used by that pass), and dL/dM goes to row 6
// of the coefficient array.
__global__ __launch_bounds__(kBlock) void k_det_sort_coef(const uint32_t* __restrict__ perm,
                                                           float* __restrict__ coef, int64_t n,
                                                           LRPoint* __restrict__ hs) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const uint32_t i = perm[q];
  if (i >= (uint64_t)n) return;  // defensive: perm is a permutation of [0, n)
  hs[q].v = make_float4(coef[i], coef[n + i], coef[2 * n + i], coef[3 * n + i]);
  hs[q].p.w = coef[5 * n + i];
  coef[6 * n + q] = coef[4 * n + i];
}

// Sum over the wave by a fixed butterfly: the same inputs give the same bits.
__device__ __forceinline__ float wave_sum_fixed(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One wave per LR particle (sorted index js = 4 blockIdx.x + wave): its HR
// neighbours come from the HR grid (stable cell order) over the stencil of
// its own cell, each lane taking every 64th candidate of the walk; the terms
// of a member pair are those of adjoint_lane, from the pair's HR coefficients
// (sorted with the HR particles by k_det_sort_coef) and the same separately
// rounded squared distance.  Lane 0 adds the wave's
// sums into the caller's gradients (one writer per LR particle).
__global__ __launch_bounds__(kBlock) void k_adjoint_det_lr(AdjointArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t js = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (js >= a.n_lr) return;
  const GridConst& gc = a.gc;
  const LRPoint L = a.lr[js];
  const uint32_t id = __float_as_uint(L.v.w);
  const uint32_t* hcs = a.hr_cell_start;
  const LRPoint* hs = a.hr_sorted;
  const float* gm = a.det_coef + 6 * a.n;  // dL/dM by sorted slot
  const float k2 = -6.0f * gc.inv_h2;
  int lo[3], hi[3];
  stencil_bounds(gc, L.p.x, L.p.y, L.p.z, lo, hi);
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int zz = lo[2]; zz <= hi[2]; ++zz)
    for (int yy = lo[1]; yy <= hi[1]; ++yy) {
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      const uint32_t b = hcs[row + (uint32_t)lo[0]], e = hcs[row + (uint32_t)hi[0] + 1u];
      // candidate q: H = (x, y, z, argmax bits), C = (dL/dU, dL/dS)
      auto term = [&](const float4 H, const float4 C, uint32_t q) {
        const float s = sq_dist(L.p.x, L.p.y, L.p.z, H.x, H.y, H.z);
        if (s < gc.h2) {
          const float gUx = C.x, gUy = C.y, gUz = C.z, gS = C.w;
          const uint32_t arg = __float_as_uint(H.w);
          const float t = fmaxf(fmaf(-s, gc.inv_h2, 1.0f), 0.0f);
          const float w = t * t * t;
          float gw = fmaf(gUz, L.v.z, fmaf(gUy, L.v.y, gUx * L.v.x)) + gS;
          if (id == arg) gw += gm[q];
          const float c = gw * k2 * t * t;
          acc[0] += w * gUx;
          acc[1] += w * gUy;
          acc[2] += w * gUz;
          acc[3] += c * (L.p.x - H.x);
          acc[4] += c * (L.p.y - H.y);
          acc[5] += c * (L.p.z - H.z);
        }
      };
      // the lane's candidates q, q + 64, ... in order; eight (then four) at a
      // time, so that their loads are in flight together
      uint32_t q = b + (uint32_t)lane;
      for (; q + 448u < e; q += 512u) {
        LRPoint P[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) P[k] = hs[q + 64u * (uint32_t)k];
#pragma unroll
        for (int k = 0; k < 8; ++k) term(P[k].p, P[k].v, q + 64u * (uint32_t)k);
      }
      for (; q + 192u < e; q += 256u) {
        const LRPoint P0 = hs[q], P1 = hs[q + 64u], P2 = hs[q + 128u], P3 = hs[q + 192u];
        term(P0.p, P0.v, q);
        term(P1.p, P1.v, q + 64u);
        term(P2.p, P2.v, q + 128u);
        term(P3.p, P3.v, q + 192u);
      }
      for (; q < e; q += 64u) {
        const LRPoint P = hs[q];
        term(P.p, P.v, q);
      }
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = wave_sum_fixed(acc[c]);
  if (lane == 0) {
    const int64_t nl = a.n_lr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.g_lr_v[c * nl + id] += acc[c];
      a.g_lr_x[c * nl + id] += acc[3 + c];
    }
  }
}

// Sum over 16 lanes of a row; lane 15 of the row receives it.
__device__ __forceinline__ float row_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));
  return v;
}

__device__ __forceinline__ float swap_sum32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wave sums of twelve per-lane values (two candidates a, b; six components
// each).  After the 32- and 16-lane swap levels the three registers hold,
// row by row (rows of 16 lanes),
//   r0: a0 a1 a3 a4     r1: a2 b0 a5 b3     r2: b1 b2 b4 b5
// and a DPP row sum leaves each total on lane 15 of its row.
struct Six {
  float v[6];
};

__device__ __forceinline__ void reduce12(const Six& av, const Six& bv, float* r0, float* r1, float* r2) {
  const float p0 = swap_sum32(av.v[0], av.v[3]);
  const float p1 = swap_sum32(av.v[1], av.v[4]);
  const float p2 = swap_sum32(av.v[2], av.v[5]);
  const float p3 = swap_sum32(bv.v[0], bv.v[3]);
  const float p4 = swap_sum32(bv.v[1], bv.v[4]);
  const float p5 = swap_sum32(bv.v[2], bv.v[5]);
  const auto t0 = __builtin_amdgcn_permlane16_swap(__float_as_uint(p0), __float_as_uint(p1), false, false);
  const auto t1 = __builtin_amdgcn_permlane16_swap(__float_as_uint(p2), __float_as_uint(p3), false, false);
  const auto t2 = __builtin_amdgcn_permlane16_swap(__float_as_uint(p4), __float_as_uint(p5), false, false);
  *r0 = row_sum(__uint_as_float(t0[0]) + __uint_as_float(t0[1]));
  *r1 = row_sum(__uint_as_float(t1[0]) + __uint_as_float(t1[1]));
  *r2 = row_sum(__uint_as_float(t2[0]) + __uint_as_float(t2[1]));
}

// Gradient contributions of one (HR particle, LR candidate) pair: the six LR
// components (dL/dV, dL/dX) are returned, the HR position term is subtracted
// from bk.g{x,y,z}.
struct PairGeom {
  float dx, dy, dz, t;  // X_j - x and max(1 - |X_j - x|^2 / h^2, 0)
};
__device__ __forceinline__ PairGeom pair_geom(float4 Q, float x, float y, float z, float inv_h2) {
  PairGeom g;
  g.dx = Q.x - x;
  g.dy = Q.y - y;
  g.dz = Q.z - z;
  const float sq = fmaf(g.dz, g.dz, fmaf(g.dy, g.dy, g.dx * g.dx));
  // 1 - sq / h^2 <= 1, so the [0, 1] clamp (folded into the fma) is max(., 0)
  g.t = __builtin_amdgcn_fmed3f(fmaf(-sq, inv_h2, 1.0f), 0.0f, 1.0f);
  return g;
}

__device__ __forceinline__ Six pair_contrib(const PairGeom& pg, float4 W, float k2, uint32_t arg, Back& bk) {
  const uint32_t id = __float_as_uint(W.w);
  const float dx = pg.dx, dy = pg.dy, dz = pg.dz, t = pg.t;
  const float t2 = t * t;
  const float w = t2 * t;
  const float gw = fmaf(bk.gUz, W.z, fmaf(bk.gUy, W.y, bk.gUx * W.x)) + bk.gS + (id == arg ? bk.gM : 0.0f);
  const float cf = gw * k2 * t2;
  Six o;
  o.v[0] = w * bk.gUx;
  o.v[1] = w * bk.gUy;
  o.v[2] = w * bk.gUz;
  o.v[3] = cf * dx;
  o.v[4] = cf * dy;
  o.v[5] = cf * dz;
  bk.gx -= o.v[3];
  bk.gy -= o.v[4];
  bk.gz -= o.v[5];
  return o;
}

// Block accumulation of LR gradients: the four waves of a block cover one
// compact region, so their candidates share LR particles.  The block lists
// the (y, z) rows of the union of its waves' stencils; slot s of the
// flattened rows is one LR particle (sorted order).  Waves add their
// wave-summed contributions to an LDS accumulator acc[component][slot] and the
// block adds the non-zero slots to global memory once at the end.
constexpr int kAccCap = 352;        // accumulator slots per block (22.4 KB of LDS in all: 7 blocks per CU)
constexpr int kBlockRows = 256;     // at most one row per thread
constexpr int kAdjListCap = 64;     // LDS candidate entries per wave and flush
constexpr int kAdjRows = 64;        // stencil rows of one wave

// A wave of the adjoint tiles its candidates unless its rows overflow the
// LDS, or it would stream more than tile_max candidates while its lanes' own
// stencils hold fewer than 1 / kAdjLaneWalkShare of them (spread-out waves
// walk per lane; compact waves in dense LR keep the shared list).  tile_max 0
// sends every wave with candidates to the per-lane walk.  Wave-uniform; the
// tiled and the deterministic kernels decide alike.
constexpr uint32_t kAdjLaneWalkShare = 8;
__device__ __forceinline__ bool adjoint_wave_tiled(const TileSetup<1>& ts, const AdjointArgs& a, float x,
                                                   float y, float z) {
  if (ts.nrows > kAdjRows) return false;
  if (ts.total <= (uint32_t)a.tile_max) return true;
  return a.tile_max != 0 && kAdjLaneWalkShare * lane_walk_max(a.gc, a.cell_start, x, y, z) >= ts.total;
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t s = wsum[w];
    off += (w < wid) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_adjoint_tiled(AdjointArgs a, WallTable wt) {
  __shared__ TileLDS<1, kAdjListCap, kAdjRows> lds;
  __shared__ float acc[6][kAccCap];
  __shared__ uint32_t brb[kBlockRows];       // first sorted index of each block row
  __shared__ uint32_t brp[kBlockRows + 1];   // exclusive prefix of block row lengths
  __shared__ uint32_t sbase[kWaves][kAdjRows];  // block slot of each wave row's first entry
  __shared__ int wbox[kWaves][6];
  __shared__ int bmeta[8];
  __shared__ uint32_t wsum[kWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = a.n;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + tid;
  const bool live = i0 < n;
  const int64_t i = live ? i0 : n - 1;  // idle lanes shadow the last particle
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const GridConst& gc = a.gc;
  const int64_t nl = a.n_lr;

  const TileSetup<1> ts = tile_setup<1>(gc, a.cell_start, x, y, z, lane, wid, lds);
  const bool wave_tiled = adjoint_wave_tiled(ts, a, x, y, z);

  // ---- block box and block rows
  if (lane == 0) {
    wbox[wid][0] = ord(ts.gb[0].lo[0]); wbox[wid][1] = ord(ts.gb[0].lo[1]); wbox[wid][2] = ord(ts.gb[0].lo[2]);
    wbox[wid][3] = ord(ts.gb[0].hi[0]); wbox[wid][4] = ord(ts.gb[0].hi[1]); wbox[wid][5] = ord(ts.gb[0].hi[2]);
  }
  __syncthreads();
  if (tid == 0) {
    int lo[3] = {wbox[0][0], wbox[0][1], wbox[0][2]}, hi[3] = {wbox[0][3], wbox[0][4], wbox[0][5]};
    for (int w = 1; w < kWaves; ++w)
      for (int c = 0; c < 3; ++c) {
        lo[c] = min(lo[c], wbox[w][c]);
        hi[c] = max(hi[c], wbox[w][3 + c]);
      }
    int c0[3], c1[3];
    for (int c = 0; c < 3; ++c) {
      c0[c] = max(cell_coord(unord(lo[c]), gc.lo[c], gc.inv_cs, gc.dims[c]) - gc.reach, 0);
      c1[c] = min(cell_coord(unord(hi[c]), gc.lo[c], gc.inv_cs, gc.dims[c]) + gc.reach, gc.dims[c] - 1);
    }
    bmeta[0] = c0[0]; bmeta[1] = c1[0]; bmeta[2] = c0[1]; bmeta[3] = c1[1]; bmeta[4] = c0[2];
    bmeta[5] = (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
  }
  __syncthreads();
  const int bX0 = bmeta[0], bX1 = bmeta[1], bY0 = bmeta[2], bY1 = bmeta[3], bZ0 = bmeta[4];
  const int bny = bY1 - bY0 + 1;
  const int bnrows = bmeta[5];
  bool block_acc = bnrows <= kBlockRows;
  uint32_t btotal = 0;
  if (block_acc) {
    uint32_t rb = 0, rl = 0;
    if (tid < bnrows) {
      const int yy = bY0 + tid % bny, zz = bZ0 + tid / bny;
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      rb = a.cell_start[row + (uint32_t)bX0];
      rl = a.cell_start[row + (uint32_t)bX1 + 1u] - rb;
    }
    const uint32_t ex = block_exclusive_scan(rl, &btotal, wsum);
    if (tid < bnrows) {
      brb[tid] = rb;
      brp[tid] = ex;
    }
    if (tid == 0) brp[bnrows] = btotal;
    block_acc = btotal <= (uint32_t)kAccCap;
  }
  if (block_acc) {
    for (uint32_t t = tid; t < btotal; t += kBlock)
      for (int c = 0; c < 6; ++c) acc[c][t] = 0.0f;
  }
  __syncthreads();
  if (block_acc && wave_tiled) {
    for (int r = lane; r < ts.nrows; r += 64) {
      const int yy = ts.Y0 + r % ts.ny, zz = ts.Z0 + r / ts.ny;
      const int br = (yy - bY0) + bny * (zz - bZ0);
      sbase[wid][r] = brp[br] + (lds.rb[wid][r] - brb[br]);
    }
  }
  wave_lds_sync();

  if (!wave_tiled) {
    if (live) adjoint_lane(a, wt, i);
  } else {
    const float inv_h2 = gc.inv_h2;
    // ---- pass 1: sums and argmax (ties: smallest original index)
    float S = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, M = 0.f;
    uint32_t arg = 0xffffffffu;
    if (a.tape != nullptr) {
      S = a.tape[i];
      Ux = a.tape[n + i];
      Uy = a.tape[2 * n + i];
      Uz = a.tape[3 * n + i];
      M = a.tape[4 * n + i];
      arg = __float_as_uint(a.tape[5 * n + i]);
    } else {
      uint64_t key = 0ull;  // (weight bits << 32 | ~index): unsigned maximum = argmax
      tile_visit<1>(ts, gc, a.lr, lane, wid, lds, [&](uint32_t nc, const float4* lp, const float4* lv) {
        for (uint32_t c = 0; c < nc; ++c) {
          const float4 Q = lp[c];
          const float4 W = lv[c];
          const float dx = Q.x - x, dy = Q.y - y, dz = Q.z - z;
          const float sq = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          const float u = __builtin_amdgcn_fmed3f(fmaf(-sq, inv_h2, 1.0f), 0.0f, 1.0f);
          const float w = u * u * u;
          const uint32_t id = __float_as_uint(W.w);
          S += w;
          Ux = fmaf(w, W.x, Ux);
          Uy = fmaf(w, W.y, Uy);
          Uz = fmaf(w, W.z, Uz);
          const uint64_t kk = ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(~id);
          key = kk > key ? kk : key;
        }
      });
      M = __uint_as_float((uint32_t)(key >> 32));
      arg = ~(uint32_t)key;  // largest weight, ties to the smallest index; meaningful when M > 0
    }
    // ---- replay and pull-back; idle lanes carry a zero upstream gradient
    const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
    const float z0 = 0.0f;
    Back bk = backprop(a.sc, wt, x, y, z, vx, vy, vz, S, Ux, Uy, Uz, M,
                       live ? a.gx_out[i] : z0, live ? a.gx_out[n + i] : z0, live ? a.gx_out[2 * n + i] : z0,
                       live ? a.gv_out[i] : z0, live ? a.gv_out[n + i] : z0, live ? a.gv_out[2 * n + i] : z0);
    // ---- pass 2: pair gradients; LR parts summed over the wave, then over the block
    const float k2 = -6.0f * inv_h2;  // dw/ds = -3 t^2 / h2, times 2 for ds/dX
    const int row = lane >> 4;
    const bool row_tail = (lane & 15) == 15;
    // components of the twelve reduced values (reduce12 layout), per row
    const int ca0 = row < 2 ? row : row + 1;               // r0: a0 a1 a3 a4
    const int ca1 = (row == 0) ? 2 : (row == 1) ? 0 : (row == 2) ? 5 : 3;  // r1: a2 b0 a5 b3
    const bool cb1 = (row == 1) || (row == 3);             //     (b entries in rows 1, 3)
    const int ca2 = (row == 0) ? 1 : (row == 1) ? 2 : (row == 2) ? 4 : 5;  // r2: b1 b2 b4 b5
    // destinations of this lane's three reduced values (per row, fixed for the loop)
    auto lr_grad = [&](int comp) {
      return comp < 3 ? a.g_lr_v + (int64_t)comp * nl : a.g_lr_x + (int64_t)(comp - 3) * nl;
    };
    float* const dst0 = lr_grad(ca0);
    float* const dst1 = lr_grad(ca1);
    float* const dst2 = lr_grad(ca2);
    // Wave-summed LR parts of two candidates, added by the row-tail lanes
    // (slots / ids of candidates a and b; a lone candidate passes zeros as b
    // and its own slot, so the adds stay branch-free).
    auto flush = [&](const Six& va, const Six& vb, uint32_t sa, uint32_t sbb, uint32_t ia, uint32_t ib) {
      float r0, r1, r2;
      reduce12(va, vb, &r0, &r1, &r2);
      if (row_tail) {
        if (block_acc) {
          atomicAdd(&acc[ca0][sa], r0);
          atomicAdd(&acc[ca1][cb1 ? sbb : sa], r1);
          atomicAdd(&acc[ca2][sbb], r2);
        } else {
          unsafeAtomicAdd(dst0 + ia, r0);
          unsafeAtomicAdd(dst1 + (cb1 ? ib : ia), r1);
          unsafeAtomicAdd(dst2 + ib, r2);
        }
      }
    };
    // About a quarter of a list's entries lie beyond the support of every
    // lane (the wave's particles do not fill its box): their terms are zero
    // for all lanes, so a ballot skips them.  The others are reduced two at a
    // time, the first of a pair held until the second arrives.
    auto pair_pass = [&](uint32_t nc, const float4* lp, const float4* lv) {
      Six held;
      uint32_t hs = 0u, hi = 0u;
      bool holding = false;  // uniform
      for (uint32_t c = 0; c < nc; ++c) {
        const float4 Q = lp[c];
        const PairGeom pg = pair_geom(Q, x, y, z, inv_h2);
        if (__builtin_amdgcn_ballot_w64(pg.t > 0.0f) == 0ull) continue;
        const float4 W = lv[c];
        const Six v = pair_contrib(pg, W, k2, arg, bk);
        if (!holding) {
          held = v;
          hs = __float_as_uint(Q.w);
          hi = __float_as_uint(W.w);
          holding = true;
        } else {
          flush(held, v, hs, __float_as_uint(Q.w), hi, __float_as_uint(W.w));
          holding = false;
        }
      }
      if (holding) {
        Six zero;
#pragma unroll
        for (int q = 0; q < 6; ++q) zero.v[q] = 0.0f;
        flush(held, zero, hs, hs, hi, hi);
      }
    };
    if (block_acc) {
      const uint32_t* sb = &sbase[wid][0];
      const uint32_t* rp = &lds.rp[wid][0];
      tile_visit<1>(ts, gc, a.lr, lane, wid, lds, pair_pass,
                    [=](int r, uint32_t k, uint32_t, float) { return sb[r] + (k - rp[r]); });
    } else {
      tile_visit<1>(ts, gc, a.lr, lane, wid, lds, pair_pass);
    }
    if (live) {
      a.gx_in[i] = bk.gx;
      a.gx_in[n + i] = bk.gy;
      a.gx_in[2 * n + i] = bk.gz;
      a.gv_in[i] = bk.gvx;
      a.gv_in[n + i] = bk.gvy;
      a.gv_in[2 * n + i] = bk.gvz;
    }
  }
  __syncthreads();
  // ---- flush the block accumulator: one atomic per non-zero (slot, component)
  if (block_acc) {
    for (uint32_t t = tid; t < btotal; t += kBlock) {
      int lo = 0, hi = bnrows;  // largest block row r with brp[r] <= t
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (brp[mid] <= t) lo = mid; else hi = mid;
      }
      const uint32_t j = brb[lo] + (t - brp[lo]);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const float v = acc[c][t];
        if (v != 0.0f) unsafeAtomicAdd(a.g_sorted + (int64_t)c * nl + j, v);
      }
    }
  }
}

// The block flushes' sums, by sorted index, added into the caller's LR
// gradients by original index (the sorted copy is a permutation of the LR
// particles, so each destination has one writer), zeroing them behind.
__global__ __launch_bounds__(kBlock) void k_lr_grad_unsort(const LRPoint* __restrict__ lr, float* g_sorted,
                                                          int64_t nl, float* g_lr_x, float* g_lr_v) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nl) return;
  const uint32_t id = __float_as_uint(lr[j].v.w);
  // all twelve loads first (one round trip), then the stores
  float v[6], old[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) v[c] = g_sorted[(int64_t)c * nl + j];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float* dst = c < 3 ? g_lr_v + (int64_t)c * nl : g_lr_x + (int64_t)(c - 3) * nl;
    old[c] = dst[id];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    if (v[c] != 0.0f) {
      float* dst = c < 3 ? g_lr_v + (int64_t)c * nl : g_lr_x + (int64_t)(c - 3) * nl;
      dst[id] = old[c] + v[c];
      g_sorted[(int64_t)c * nl + j] = 0.0f;
    }
  }
}

// Deterministic LR gradients, scenes without rigid LR particles: the HR
// pass of k_adjoint_tiled (the same sums, replay and pull-back, and the HR
// position terms in the same list order and arithmetic, so the HR gradients
// are that kernel's bits) without its LR accumulation; each particle's
// coefficients go to a.det_coef for the LR pass.  Spread waves walk per lane.
__global__ __launch_bounds__(kBlock) void k_adjoint_det_tiled(AdjointArgs a, WallTable wt) {
  __shared__ TileLDS<1, kAdjListCap, kAdjRows> lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = a.n;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + tid;
  const bool live = i0 < n;
  const int64_t i = live ? i0 : n - 1;  // idle lanes shadow the last particle
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const GridConst& gc = a.gc;

  const TileSetup<1> ts = tile_setup<1>(gc, a.cell_start, x, y, z, lane, wid, lds);
  if (!adjoint_wave_tiled(ts, a, x, y, z)) {
    if (live) adjoint_lane<true>(a, wt, i);
    return;  // wave-uniform: no block barrier follows
  }
  const float inv_h2 = gc.inv_h2;
  float S = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, M = 0.f;
  uint32_t arg = 0xffffffffu;
  if (a.tape != nullptr) {
    S = a.tape[i];
    Ux = a.tape[n + i];
    Uy = a.tape[2 * n + i];
    Uz = a.tape[3 * n + i];
    M = a.tape[4 * n + i];
    arg = __float_as_uint(a.tape[5 * n + i]);
  } else {
    uint64_t key = 0ull;  // (weight bits << 32 | ~index): unsigned maximum = argmax
    tile_visit<1>(ts, gc, a.lr, lane, wid, lds, [&](uint32_t nc, const float4* lp, const float4* lv) {
      for (uint32_t c = 0; c < nc; ++c) {
        const float4 Q = lp[c];
        const float4 W = lv[c];
        const float dx = Q.x - x, dy = Q.y - y, dz = Q.z - z;
        const float sq = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float u = __builtin_amdgcn_fmed3f(fmaf(-sq, inv_h2, 1.0f), 0.0f, 1.0f);
        const float w = u * u * u;
        const uint32_t id = __float_as_uint(W.w);
        S += w;
        Ux = fmaf(w, W.x, Ux);
        Uy = fmaf(w, W.y, Uy);
        Uz = fmaf(w, W.z, Uz);
        const uint64_t kk = ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(~id);
        key = kk > key ? kk : key;
      }
    });
    M = __uint_as_float((uint32_t)(key >> 32));
    arg = ~(uint32_t)key;
  }
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  const float z0 = 0.0f;
  Back bk = backprop(a.sc, wt, x, y, z, vx, vy, vz, S, Ux, Uy, Uz, M,
                     live ? a.gx_out[i] : z0, live ? a.gx_out[n + i] : z0, live ? a.gx_out[2 * n + i] : z0,
                     live ? a.gv_out[i] : z0, live ? a.gv_out[n + i] : z0, live ? a.gv_out[2 * n + i] : z0);
  if (live) {
    a.det_coef[i] = bk.gUx;
    a.det_coef[n + i] = bk.gUy;
    a.det_coef[2 * n + i] = bk.gUz;
    a.det_coef[3 * n + i] = bk.gS;
    a.det_coef[4 * n + i] = bk.gM;
    a.det_coef[5 * n + i] = __uint_as_float(arg);
  }
  const float k2 = -6.0f * inv_h2;  // dw/ds = -3 t^2 / h2, times 2 for ds/dX
  tile_visit<1>(ts, gc, a.lr, lane, wid, lds, [&](uint32_t nc, const float4* lp, const float4* lv) {
    for (uint32_t c = 0; c < nc; ++c) {
      const PairGeom pg = pair_geom(lp[c], x, y, z, inv_h2);
      if (__builtin_amdgcn_ballot_w64(pg.t > 0.0f) == 0ull) continue;
      (void)pair_contrib(pg, lv[c], k2, arg, bk);  // the HR position terms
    }
  });
  if (live) {
    a.gx_in[i] = bk.gx;
    a.gx_in[n + i] = bk.gy;
    a.gx_in[2 * n + i] = bk.gz;
    a.gv_in[i] = bk.gvx;
    a.gv_in[n + i] = bk.gvy;
    a.gv_in[2 * n + i] = bk.gvz;
  }
}

}  // namespace

hipError_t launch_adjoint(const AdjointArgs& a, const WallTable& walls, hipStream_t st,
                          const GridScratch* hr_grid) {
  if (a.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n + kBlock - 1) / kBlock);
  if (a.det_coef != nullptr) {
    if (hr_grid == nullptr) return hipErrorInvalidValue;
    if (a.sc.has_rigid || !a.tiled)
      hipLaunchKernelGGL(k_adjoint_det, dim3(blocks), dim3(kBlock), 0, st, a, walls);
    else
      hipLaunchKernelGGL(k_adjoint_det_tiled, dim3(blocks), dim3(kBlock), 0, st, a, walls);
    if (a.n_lr > 0) {
      const int64_t n_cells = (int64_t)a.gc.dims[0] * a.gc.dims[1] * a.gc.dims[2];
      hipError_t e = launch_build_grid(a.gc, a.hx, a.hv, nullptr, a.n, n_cells, *hr_grid, st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_det_sort_coef, dim3(blocks), dim3(kBlock), 0, st, hr_grid->perm, a.det_coef, a.n,
                         hr_grid->lr_sorted);
      AdjointArgs b = a;
      b.hr_cell_start = hr_grid->cell_start;
      b.hr_sorted = hr_grid->lr_sorted;
      hipLaunchKernelGGL(k_adjoint_det_lr, dim3((unsigned)((a.n_lr + kWaves - 1) / kWaves)), dim3(kBlock), 0, st, b);
    }
  } else if (a.sc.has_rigid || !a.tiled) {
    hipLaunchKernelGGL(k_adjoint, dim3(blocks), dim3(kBlock), 0, st, a, walls);
  } else {
    hipLaunchKernelGGL(k_adjoint_tiled, dim3(blocks), dim3(kBlock), 0, st, a, walls);
    if (a.n_lr > 0)
      hipLaunchKernelGGL(k_lr_grad_unsort, dim3((unsigned)((a.n_lr + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                         st, a.lr, a.g_sorted, a.n_lr, a.g_lr_x, a.g_lr_v);
  }
  return hipGetLastError();
}

}  // namespace ups
