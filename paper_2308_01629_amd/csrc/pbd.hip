// The LR simulation step (Section 3, Algorithm 1) on the GPU: position-based
// dynamics with contact and friction constraints solved by constraint
// averaging (Jacobi: every constraint of an iteration is evaluated at the
// positions the iteration starts from, each particle's displacements are
// summed and divided by its number of active constraints), stabilization
// iterations, height-scaled masses, and shape-matching constraints that
// couple rigid bodies to the granular material.
//
// Each particle computes the displacements its own constraints give it, from
// its contact list: a pair's two sides are evaluated by the two particles
// with the same arithmetic, so no atomics are needed and the result does not
// depend on scheduling.  The contact lists come from the LR grid build (a
// uniform grid of cells at least 2r wide, counting sort).
//
// Per step: k_pbd_predict, grid + k_pbd_pairs on the start positions,
// stab_iters x k_pbd_stab, grid + k_pbd_pairs on the predicted positions
// (each grid build's keys and counts come from the kernel before it),
// solve_iters x (k_pbd_shape per rigid body, k_pbd_solve), and k_pbd_finish
// unless the last k_pbd_solve writes the velocities itself.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace ups {
namespace {

constexpr int kGranular = -1;
constexpr int kStatic = -2;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct PbdConst {
  float r2;      // 2 r: the contact distance
  float dt, inv_dt;
  float g[3];
  float mu_s2r;  // 2 r mu_s: static friction threshold
  float mu_k2r;  // 2 r mu_k: kinetic friction length
  float ground_y;
  int mass_scaling;
};

// 1. v += dt g (dynamic), x~ = x + dt v; scaled inverse mass w* = w exp(h).
// KEYS 1 / 2 also start the next grid build: the cell keys of x / of the new
// x~, counted into the build's bins (claim_slot), so the build begins at its
// scan.
enum { kKeysNone = 0, kKeysOfX = 1, kKeysOfXt = 2 };

template <int KEYS>
__global__ __launch_bounds__(kBlock) void k_pbd_predict(PbdConst pc, int64_t n, const float* __restrict__ x,
                                                        float* __restrict__ v, float* __restrict__ xt,
                                                        const int32_t* __restrict__ body,
                                                        const float* __restrict__ inv_m, float* __restrict__ w,
                                                        GridConst gc, uint32_t* __restrict__ keys,
                                                        uint32_t* __restrict__ slot, uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  float P[3] = {0.f, 0.f, 0.f}, T[3] = {0.f, 0.f, 0.f};
  if (valid) {
    const bool stat = body[i] == kStatic;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P[a] = x[a * n + i];
      const float va = stat ? 0.0f : fmaf(pc.dt, pc.g[a], v[a * n + i]);
      v[a * n + i] = va;
      T[a] = fmaf(pc.dt, va, P[a]);
      xt[a * n + i] = T[a];
    }
    float wi = stat ? 0.0f : inv_m[i];
    if (pc.mass_scaling) wi *= expf(P[1] - pc.ground_y);
    w[i] = wi;
  }
  if (KEYS != kKeysNone) {
    const float* K3 = KEYS == kKeysOfX ? P : T;
    const uint32_t k = valid ? cell_key(gc, K3[0], K3[1], K3[2]) : 0u;
    const uint32_t sl = claim_slot(k, valid, counts);
    if (valid) {
      keys[i] = k;
      slot[i] = sl;
    }
  }
}

// Lanes per particle: up to kIterLanes8Max particles the pair search gives
// each of the 9 stencil rows (dy, dz in {-1, 0, 1}) its own lane of 16, and
// the iterations split a particle's pair list over 8 lanes and sum them by a
// fixed butterfly.  Small LR systems (tens of thousands of particles) would
// otherwise leave the chip with about one wave per CU and every wave waiting
// on memory; with 8 lanes a system of kIterLanes8Max particles still fits
// about 8 waves per SIMD in one round.  Larger systems take 8 lanes in the
// pair search (the first lane scanning the ninth row too) and 4 in the
// iterations, which then fill the chip with fewer waves.
constexpr int64_t kIterLanes8Max = 65536;
inline int iter_lanes(int64_t n) { return n <= kIterLanes8Max ? 8 : 4; }
inline int pair_lanes(int64_t n) { return n <= kIterLanes8Max ? 16 : 8; }

// Contact list of each particle: the other particles closer than 2r
// (a static particle keeps none: with zero inverse mass every constraint
// moves it by exactly zero, and its partners list the pair themselves;
// squared distance rounded as in the upsampling's membership predicate,
// against fl32(4 r^2)), without static-static and same-body pairs, ordered by
// the lane that scans them and, inside a lane's rows, by particle index: with
// PL = 16 lanes that is by stencil row (dz, then dy); with 8 the first lane
// takes the first and the ninth row together.  The grid's order inside a cell
// varies from run to run; this order does not, so the iterations sum each
// particle's constraints in the same order every time.  Groups of PL lanes
// take the sorted slots in order (the sorted copy carries each particle's
// body id in p.w and its index in v.w).  Each lane reads its candidates four
// at a time and stages its first kRowStage
// matches in LDS; the group forms the exclusive prefix of the lanes' counts,
// and a lane with at most kRowStage matches sorts them in registers (a
// 19-comparator network) and copies them to the list.  A lane with more
// matches scans its row once more, writes all of them and sorts them in
// place.  (A rescan that picked the matches in order, one scan each, made
// the common path about 30% slower on a large grid though it never ran.)
// A list longer than K sets *overflow and keeps K of its entries, which
// ones then depending on the grid's order inside the cells.
constexpr int kRowStage = 8;

__device__ __forceinline__ void cmp_swap(uint32_t& a, uint32_t& b) {
  const uint32_t lo = min(a, b);
  b = max(a, b);
  a = lo;
}

// Sorts eight values (Batcher's odd-even merge sort network for 8 inputs).
__device__ __forceinline__ void sort8(uint32_t (&s)[8]) {
  cmp_swap(s[0], s[2]); cmp_swap(s[1], s[3]); cmp_swap(s[4], s[6]); cmp_swap(s[5], s[7]);
  cmp_swap(s[0], s[4]); cmp_swap(s[1], s[5]); cmp_swap(s[2], s[6]); cmp_swap(s[3], s[7]);
  cmp_swap(s[0], s[1]); cmp_swap(s[2], s[3]); cmp_swap(s[4], s[5]); cmp_swap(s[6], s[7]);
  cmp_swap(s[2], s[4]); cmp_swap(s[3], s[5]);
  cmp_swap(s[1], s[4]); cmp_swap(s[3], s[6]);
  cmp_swap(s[1], s[2]); cmp_swap(s[3], s[4]); cmp_swap(s[5], s[6]);
}

template <int PL>
__global__ __launch_bounds__(kBlock) void k_pbd_pairs(GridConst gc, const LRPoint* __restrict__ sorted,
                                                      const uint32_t* __restrict__ cell_start, int64_t n, int K,
                                                      uint32_t* __restrict__ cnt, uint32_t* __restrict__ ids,
                                                      uint32_t* overflow) {
  __shared__ uint32_t stage[kRowStage][kBlock];
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t t = g / PL;
  const int lane = (int)(g % PL);
  if (t >= n) return;  // the 16 lanes of a particle leave together
  const LRPoint me = sorted[t];
  const uint32_t i = __float_as_uint(me.v.w);
  const int bi = __float_as_int(me.p.w);
  if (bi == kStatic) {  // its own constraints move it by exactly zero: no list
    if (lane == 0) cnt[i] = 0u;
    return;  // all lanes of the particle leave together
  }
  const int cx = cell_coord(me.p.x, gc.lo[0], gc.inv_cs, gc.dims[0]);
  const int cy = cell_coord(me.p.y, gc.lo[1], gc.inv_cs, gc.dims[1]);
  const int cz = cell_coord(me.p.z, gc.lo[2], gc.inv_cs, gc.dims[2]);
  auto row_range = [&](int r, uint32_t& rb, uint32_t& re) {
    rb = re = 0u;
    const int yy = cy + r % 3 - 1, zz = cz + r / 3 - 1;
    if (r < 9 && yy >= 0 && yy < gc.dims[1] && zz >= 0 && zz < gc.dims[2]) {
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      rb = cell_start[row + (uint32_t)max(cx - 1, 0)];
      re = cell_start[row + (uint32_t)min(cx + 1, gc.dims[0] - 1) + 1u];
    }
  };
  uint32_t b, e, b2 = 0u, e2 = 0u;
  row_range(lane, b, e);
  if (PL < 9 && lane == 0) row_range(8, b2, e2);  // the ninth row goes to the first lane
  auto match = [&](const LRPoint& L) -> bool {
    const uint32_t j = __float_as_uint(L.v.w);
    const int bj = __float_as_int(L.p.w);
    if (j == i || (bi == kStatic && bj == kStatic) || (bi >= 0 && bi == bj)) return false;
    return sq_dist(L.p.x, L.p.y, L.p.z, me.p.x, me.p.y, me.p.z) < gc.h2;
  };
  uint32_t c = 0;
  auto scan = [&](uint32_t rb, uint32_t re) {
    for (uint32_t q0 = rb; q0 < re; q0 += 4) {
      LRPoint L[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + u < re) L[u] = sorted[q0 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + u < re && match(L[u])) {
          if (c < (uint32_t)kRowStage) stage[c][threadIdx.x] = __float_as_uint(L[u].v.w);
          ++c;
        }
    }
  };
  scan(b, e);
  if (PL < 9) scan(b2, e2);
  uint32_t incl = c;
#pragma unroll
  for (int d = 1; d < PL; d <<= 1) {
    const uint32_t u = __shfl_up(incl, d, PL);
    if (lane >= d) incl += u;
  }
  const uint32_t total = __shfl(incl, PL - 1, PL);
  const uint32_t o0 = incl - c;
  uint32_t* list = ids + (int64_t)i * K;
  if (c <= (uint32_t)kRowStage) {
    uint32_t sv[kRowStage];
#pragma unroll
    for (int k = 0; k < kRowStage; ++k) sv[k] = (uint32_t)k < c ? stage[k][threadIdx.x] : 0xffffffffu;
    sort8(sv);
#pragma unroll
    for (int k = 0; k < kRowStage; ++k)
      if ((uint32_t)k < c && o0 + (uint32_t)k < (uint32_t)K) list[o0 + (uint32_t)k] = sv[k];
  } else {  // rare: more matches than staged; all of them by one more scan, then sorted in place
    uint32_t o = o0;
    for (uint32_t q = b; q < e && o < (uint32_t)K; ++q) {
      const LRPoint L = sorted[q];
      if (match(L)) list[o++] = __float_as_uint(L.v.w);
    }
    for (uint32_t q = b2; q < e2 && o < (uint32_t)K; ++q) {
      const LRPoint L = sorted[q];
      if (match(L)) list[o++] = __float_as_uint(L.v.w);
    }
    for (uint32_t a1 = o0 + 1u; a1 < o; ++a1) {
      const uint32_t vv = list[a1];
      uint32_t p = a1;
      for (; p > o0 && list[p - 1u] > vv; --p) list[p] = list[p - 1u];
      list[p] = vv;
    }
  }
  if (lane == 0) {
    cnt[i] = min(total, (uint32_t)K);
    if (total > (uint32_t)K) atomicOr(overflow, 1u);
  }
}

// Sum of a float over the L lanes of a particle, in a fixed order.
template <int L>
__device__ __forceinline__ float group_sum(float a) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, L);
  return a;
}

// Contact displacement of particle i in pair (i, j) at positions Pi, Pj
// (Section 3): -w_i / (w_i + w_j) (2r - d) x_ij / d for d = |x_ij| < 2r.
// Returns false when the pair does not act.
struct PairGeo {
  float xij[3];
  float d2;
  float s;   // (2r - d) / d
};
__device__ __forceinline__ bool contact_geo(const float* Pi, const float* Pj, float wi, float wj, float r2,
                                            PairGeo& g) {
  g.xij[0] = Pj[0] - Pi[0];
  g.xij[1] = Pj[1] - Pi[1];
  g.xij[2] = Pj[2] - Pi[2];
  g.d2 = fmaf(g.xij[2], g.xij[2], fmaf(g.xij[1], g.xij[1], g.xij[0] * g.xij[0]));
  const float d = sqrtf(g.d2);
  if (!(d < r2) || !(d > 0.0f) || !(wi + wj > 0.0f)) return false;
  g.s = (r2 - d) / d;
  return true;
}

__device__ __forceinline__ void load3(const float* a, int64_t n, int64_t i, float* o) {
  o[0] = a[i];
  o[1] = a[n + i];
  o[2] = a[2 * n + i];
}

// 2. One stabilization iteration on the start positions: the averaged
// contact displacement goes to x (xs_out) and to x~ (in place, by the
// particle's first lane).  KEYS: the last iteration also starts the solver
// phase's grid build on the new x~ (as k_pbd_predict does).
template <bool KEYS, int L>
__global__ __launch_bounds__(kBlock) void k_pbd_stab(PbdConst pc, int64_t n, const float* __restrict__ xs_in,
                                                     float* __restrict__ xs_out, float* __restrict__ xt,
                                                     const float* __restrict__ w, int K,
                                                     const uint32_t* __restrict__ cnt,
                                                     const uint32_t* __restrict__ ids, GridConst gc,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ slot,
                                                     uint32_t* __restrict__ counts) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / L;
  const int l = (int)(g % L);
  if (!KEYS && i >= n) return;  // the lanes of a particle leave together
  const bool valid = i < n;     // with KEYS every lane of the wave reaches claim_slot
  float Pi[3] = {0.f, 0.f, 0.f};
  float acc[3] = {0.f, 0.f, 0.f};
  float na = 0.0f;
  if (valid) {
    load3(xs_in, n, i, Pi);
    const float wi = w[i];
    const uint32_t c = cnt[i];
    for (uint32_t k = (uint32_t)l; k < c; k += L) {
      const int64_t j = ids[i * K + k];
      float Pj[3];
      load3(xs_in, n, j, Pj);
      const float wj = w[j];
      PairGeo gg;
      if (!contact_geo(Pi, Pj, wi, wj, pc.r2, gg)) continue;
      const float mi = wi / (wi + wj);
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[a] -= mi * gg.s * gg.xij[a];
      na += 1.0f;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[a] = group_sum<L>(acc[a]);
  na = group_sum<L>(na);
  float T[3] = {0.f, 0.f, 0.f};
  if (valid && l == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float u = na > 0.0f ? acc[a] / na : 0.0f;
      xs_out[a * n + i] = Pi[a] + u;
      T[a] = xt[a * n + i] + u;
      xt[a * n + i] = T[a];
    }
  }
  if (KEYS) {
    const bool own = valid && l == 0;
    const uint32_t k = own ? cell_key(gc, T[0], T[1], T[2]) : 0u;
    const uint32_t sl = claim_slot(k, own, counts);
    if (own) {
      keys[i] = k;
      slot[i] = sl;
    }
  }
}

// Shape matching, per rigid body (one wave each): c = the mean of the body's
// x~ and C = sum (x~ - c) o^T, formed in double in one pass as
// sum x~ o^T - c (sum o)^T (sum o, a constant of the body, is 0 up to the
// rounding of the rest offsets), then the rotation R of the polar
// decomposition of C: the eigenvectors v_k of C^T C by cyclic Jacobi in
// double, u_k = C v_k / |C v_k| for the two largest eigenvalues,
// u_3 = u_1 x u_2 and v_3 signed so that det R = +1, R = sum_k u_k v_k^T.
// (When det C < 0 this takes the nearest rotation, like an SVD with the sign
// of its smallest singular direction flipped.)  A well-conditioned C with
// det C > 0, the usual case of a body near its rest shape, takes the scaled
// Newton iteration for the polar factor instead (Higham 1986,
// X <- (z X + X^-T / z) / 2, z = sqrt(|X^-1|_F / |X|_F)), which reaches the
// same rotation with far fewer square roots and divisions.  Writes (c, R
// row-major) as 12 floats per body.
constexpr int kShapeThreads = 256;

template <int P, int Q>
__device__ __forceinline__ void jacobi_rot(double (&A)[3][3], double (&V)[3][3]) {
  if (A[P][Q] == 0.0) return;
  const double theta = (A[Q][Q] - A[P][P]) / (2.0 * A[P][Q]);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // A <- A J
    const double akp = A[k][P], akq = A[k][Q];
    A[k][P] = c * akp - s * akq;
    A[k][Q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // A <- J^T A
    const double apk = A[P][k], aqk = A[Q][k];
    A[P][k] = c * apk - s * aqk;
    A[Q][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // V <- V J
    const double vkp = V[k][P], vkq = V[k][Q];
    V[k][P] = c * vkp - s * vkq;
    V[k][Q] = s * vkp + c * vkq;
  }
}

// Orders eigenpairs (diagonal of A, columns of V) by decreasing eigenvalue.
template <int P, int Q>
__device__ __forceinline__ void eig_order(double (&A)[3][3], double (&V)[3][3]) {
  if (A[Q][Q] > A[P][P]) {
    const double t = A[P][P];
    A[P][P] = A[Q][Q];
    A[Q][Q] = t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double u = V[k][P];
      V[k][P] = V[k][Q];
      V[k][Q] = u;
    }
  }
}

__device__ void polar_rotation(const double (&M)[3][3], double (&R)[3][3]) {
  double A[3][3], V[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A[a][c] = M[0][a] * M[0][c] + M[1][a] * M[1][c] + M[2][a] * M[2][c];
      V[a][c] = a == c ? 1.0 : 0.0;
    }
  const double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    if (!(off > 1e-30 * scale)) break;
    jacobi_rot<0, 1>(A, V);
    jacobi_rot<0, 2>(A, V);
    jacobi_rot<1, 2>(A, V);
  }
  eig_order<0, 1>(A, V);
  eig_order<0, 2>(A, V);
  eig_order<1, 2>(A, V);
  double u[3][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[k][a] = M[a][0] * V[0][k] + M[a][1] * V[1][k] + M[a][2] * V[2][k];
      nrm += u[k][a] * u[k][a];
    }
    nrm = sqrt(nrm);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[k][a] = nrm > 0.0 ? u[k][a] / nrm : (a == k ? 1.0 : 0.0);
  }
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  const double detv = V[0][0] * (V[1][1] * V[2][2] - V[2][1] * V[1][2]) -
                      V[0][1] * (V[1][0] * V[2][2] - V[2][0] * V[1][2]) +
                      V[0][2] * (V[1][0] * V[2][1] - V[2][0] * V[1][1]);
  const double sg = detv < 0.0 ? -1.0 : 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[a][c] = u[0][a] * V[c][0] + u[1][a] * V[c][1] + sg * u[2][a] * V[c][2];
}

// Polar rotation by the scaled Newton iteration; false if M is not proper and
// well conditioned (the caller then takes the eigenvector path).
__device__ bool polar_newton(const double (&M)[3][3], double (&R)[3][3]) {
  double fro = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) fro += M[a][c] * M[a][c];
  fro = sqrt(fro / 3.0);
  if (!(fro > 0.0)) return false;
  const double ifro = 1.0 / fro;
  double X[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) X[a][c] = M[a][c] * ifro;
  for (int it = 0; it < 40; ++it) {
    // cofactors: X^-T = cof(X) / det X
    double C[3][3];
    C[0][0] = X[1][1] * X[2][2] - X[1][2] * X[2][1];
    C[0][1] = X[1][2] * X[2][0] - X[1][0] * X[2][2];
    C[0][2] = X[1][0] * X[2][1] - X[1][1] * X[2][0];
    C[1][0] = X[0][2] * X[2][1] - X[0][1] * X[2][2];
    C[1][1] = X[0][0] * X[2][2] - X[0][2] * X[2][0];
    C[1][2] = X[0][1] * X[2][0] - X[0][0] * X[2][1];
    C[2][0] = X[0][1] * X[1][2] - X[0][2] * X[1][1];
    C[2][1] = X[0][2] * X[1][0] - X[0][0] * X[1][2];
    C[2][2] = X[0][0] * X[1][1] - X[0][1] * X[1][0];
    const double det = X[0][0] * C[0][0] + X[0][1] * C[0][1] + X[0][2] * C[0][2];
    if (it == 0 && !(det > 1e-6)) return false;  // improper or near-singular
    const double id = 1.0 / det;
    double nx = 0.0, ny = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C[a][c] *= id;
        nx += X[a][c] * X[a][c];
        ny += C[a][c] * C[a][c];
      }
    const double z = sqrt(sqrt(ny / nx));
    const double hz = 0.5 * z, hiz = 0.5 / z;
    double diff = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xn = hz * X[a][c] + hiz * C[a][c];
        diff += (xn - X[a][c]) * (xn - X[a][c]);
        X[a][c] = xn;
      }
    if (diff < 1e-26) break;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[a][c] = X[a][c];
  return true;
}

__global__ __launch_bounds__(kShapeThreads) void k_pbd_shape(int64_t n, const float* __restrict__ xt,
                                                             const uint32_t* __restrict__ members,
                                                             const uint32_t* __restrict__ body_ptr,
                                                             const float* __restrict__ rest,
                                                             const double* __restrict__ osum,
                                                             float* __restrict__ cr) {
  __shared__ double part[kShapeThreads / 64][12];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const uint32_t p0 = body_ptr[b], p1 = body_ptr[b + 1];
  double s[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = 0.0;
  for (uint32_t q = p0 + (uint32_t)tid; q < p1; q += kShapeThreads) {
    const int64_t i = members[q];
    double xa[3], o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xa[a] = (double)xt[a * n + i];
      o[a] = (double)rest[a * n + i];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s[a] += xa[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) s[3 + 3 * a + c] += xa[a] * o[c];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] += __shfl_xor(s[k], off, 64);
  if ((tid & 63) == 0)
#pragma unroll
    for (int k = 0; k < 12; ++k) part[tid >> 6][k] = s[k];
  __syncthreads();
  if (tid != 0) return;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double t = part[0][k];
#pragma unroll
    for (int w = 1; w < kShapeThreads / 64; ++w) t += part[w][k];
    s[k] = t;
  }
  const double im = 1.0 / (double)(p1 - p0);
  double cen[3], M[3][3], R[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) cen[a] = s[a] * im;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) M[a][c] = s[3 + 3 * a + c] - cen[a] * osum[3 * b + c];
  if (!polar_newton(M, R)) polar_rotation(M, R);
  float* o = cr + 12 * b;
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = (float)cen[a];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) o[3 + 3 * a + c] = (float)R[a][c];
}

// 3. One solver iteration: contact and friction of each pair (one constraint)
// plus the shape-matching displacement of rigid particles, averaged.  With
// FINISH (the last iteration, x0 not aliasing x) the particle's first lane
// also does step 4: v = (x~ - x0) / dt, x = x~ (static particles keep x0,
// v = 0), and copies the state into the frame buffers if given.
struct FinishArgs {
  float* x;
  float* v;
  float* fx;
  float* fv;
};

template <bool FINISH, int L>
__global__ __launch_bounds__(kBlock) void k_pbd_solve(PbdConst pc, int64_t n, const float* __restrict__ xt_in,
                                                      float* __restrict__ xt_out, const float* __restrict__ x0,
                                                      const float* __restrict__ w, int K,
                                                      const uint32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ ids,
                                                      const int32_t* __restrict__ body,
                                                      const float* __restrict__ rest, const float* __restrict__ cr,
                                                      FinishArgs fin) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / L;
  const int l = (int)(g % L);
  if (i >= n) return;  // the lanes of a particle leave together
  float Pi[3], X0i[3];
  load3(xt_in, n, i, Pi);
  load3(x0, n, i, X0i);
  const float wi = w[i];
  float acc[3] = {0.f, 0.f, 0.f};
  float na = 0.0f;
  const uint32_t c = cnt[i];
  for (uint32_t k = (uint32_t)l; k < c; k += L) {
    const int64_t j = ids[i * K + k];
    float Pj[3], X0j[3];
    load3(xt_in, n, j, Pj);
    const float wj = w[j];
    load3(x0, n, j, X0j);
    PairGeo gg;
    if (!contact_geo(Pi, Pj, wi, wj, pc.r2, gg)) continue;
    const float mi = wi / (wi + wj), mj = wj / (wi + wj);
    float Dx[3], ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ci[a] = -mi * gg.s * gg.xij[a];
      const float cj = mj * gg.s * gg.xij[a];
      Dx[a] = ((Pi[a] + ci[a]) - X0i[a]) - ((Pj[a] + cj) - X0j[a]);
    }
    // friction on the part of Dx perpendicular to x_ij
    const float dn = fmaf(Dx[2], gg.xij[2], fmaf(Dx[1], gg.xij[1], Dx[0] * gg.xij[0])) / gg.d2;
    float Dt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Dt[a] = Dx[a] - dn * gg.xij[a];
    const float lt = sqrtf(fmaf(Dt[2], Dt[2], fmaf(Dt[1], Dt[1], Dt[0] * Dt[0])));
    const float scale = lt < pc.mu_s2r ? 1.0f : fminf(pc.mu_k2r / lt, 1.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] += ci[a] - mi * (Dt[a] * scale);
    na += 1.0f;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[a] = group_sum<L>(acc[a]);
  na = group_sum<L>(na);
  if (l != 0) return;
  const int bi = body[i];
  if (bi >= 0) {
    const float* q = cr + 12 * bi;
    float o[3];
    load3(rest, n, i, o);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float ro = fmaf(q[3 + 3 * a + 2], o[2], fmaf(q[3 + 3 * a + 1], o[1], q[3 + 3 * a] * o[0]));
      acc[a] += (ro + q[a]) - Pi[a];
    }
    na += 1.0f;
  }
  const bool stat = bi == kStatic;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float xn = Pi[a] + (na > 0.0f ? acc[a] / na : 0.0f);
    xt_out[a * n + i] = xn;
    if (FINISH) {
      const float xf = stat ? X0i[a] : xn;
      const float vf = stat ? 0.0f : (xf - X0i[a]) * pc.inv_dt;
      fin.x[a * n + i] = xf;
      fin.v[a * n + i] = vf;
      if (fin.fx != nullptr) {
        fin.fx[a * n + i] = xf;
        fin.fv[a * n + i] = vf;
      }
    }
  }
}

// 4. (when not fused into the last solver iteration) v = (x~ - x0) / dt,
// x = x~ (static particles keep x0, v = 0), x0 the stabilized start
// positions; optionally the new state into a frame buffer.  x0 may alias x
// (not restrict-qualified): each thread reads its element before writing it.
__global__ __launch_bounds__(kBlock) void k_pbd_finish(PbdConst pc, int64_t n, const float* x0,
                                                       const float* __restrict__ xt,
                                                       const int32_t* __restrict__ body, float* x,
                                                       float* __restrict__ v, float* __restrict__ fx,
                                                       float* __restrict__ fv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const bool stat = body[i] == kStatic;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float xo = x0[a * n + i];
    const float xn = stat ? xo : xt[a * n + i];
    const float vn = stat ? 0.0f : (xn - xo) * pc.inv_dt;
    x[a * n + i] = xn;
    v[a * n + i] = vn;
    if (fx != nullptr) {
      fx[a * n + i] = xn;
      fv[a * n + i] = vn;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t* __restrict__ p, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) p[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_copy_f32(float* __restrict__ dst, const float* __restrict__ src,
                                                     int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) dst[i] = src[i];
}

}  // namespace
}  // namespace ups

using namespace ups;

struct upsample_pbd_s {
  upsample_pbd_params p;
  int64_t n;
  int n_bodies;
  int K;
  GridConst gc;
  int64_t n_cells;
  GridScratch g;
  int32_t* body;
  float* inv_m;
  float* rest;
  uint32_t* members;
  uint32_t* body_ptr;
  double* osum;  // [n_bodies][3] sum of each body's rest offsets
  float* cr;
  float *w, *xt, *xt2, *xs, *xs2;
  uint32_t *cnt, *ids, *overflow;
  bool counts_dirty;  // a step that failed part way may have left grid counts non-zero
  std::string last_error;
};

namespace {

int pbd_fail(upsample_pbd h, int code, const std::string& m) {
  if (h != nullptr) h->last_error = m;
  return code;
}

void pbd_free(upsample_pbd h) {
  void* ptrs[] = {h->g.keys, h->g.slot, h->g.tmp, h->g.perm, h->g.counts, h->g.local, h->g.chunk_sum,
                  h->g.cell_start, h->g.lr_sorted, h->body, h->inv_m, h->rest, h->members, h->body_ptr, h->osum,
                  h->cr, h->w, h->xt, h->xt2, h->xs, h->xs2, h->cnt, h->ids, h->overflow};
  for (void* q : ptrs)
    if (q != nullptr) (void)hipFree(q);
}

template <typename T>
hipError_t dalloc(T** p, int64_t n) {
  return hipMalloc((void**)p, (size_t)(n > 0 ? n : 1) * sizeof(T));
}

PbdConst pbd_const(const upsample_pbd_params& p) {
  PbdConst c;
  c.r2 = 2.0f * p.r;
  c.dt = p.dt;
  c.inv_dt = 1.0f / p.dt;
  for (int a = 0; a < 3; ++a) c.g[a] = p.g[a];
  c.mu_s2r = c.r2 * p.mu_s;
  c.mu_k2r = c.r2 * p.mu_k;
  c.ground_y = p.ground_y;
  c.mass_scaling = p.mass_scaling;
  return c;
}

}  // namespace

namespace {

// Where upsample_pbd_debug_step records the stages (float offsets).
struct PbdTrace {
  float* base;
  uint32_t* pair_cnt;
  uint32_t* pair_ids;
};

int64_t trace_floats(const upsample_pbd_s* h) {
  const int64_t n = h->n;
  return 7 * n + (int64_t)h->p.stab_iters * 6 * n + (int64_t)h->p.solve_iters * (12 * (int64_t)h->n_bodies + 3 * n) +
         6 * n;
}

hipError_t copy_async(float* dst, const float* src, int64_t m, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(m)), dim3(kBlock), 0, st, dst, src, m);
  return hipGetLastError();
}

hipError_t copy_pairs(const upsample_pbd_s* h, const PbdTrace* tr, int phase, hipStream_t st) {
  const int64_t n = h->n;
  hipError_t e = hipMemcpyAsync(tr->pair_cnt + phase * n, h->cnt, sizeof(uint32_t) * (size_t)n,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tr->pair_ids + phase * n * (int64_t)h->K, h->ids, sizeof(uint32_t) * (size_t)(n * h->K),
                       hipMemcpyDeviceToDevice, st);
  return e;
}

// One step (Algorithm 1).  The stabilization reads x and then alternates
// between h->xs and h->xs2, so the stabilized start positions x0 never alias
// x when there is at least one iteration and the last solver iteration can
// write the new state itself; the solver alternates between h->xt and
// h->xt2.  With a trace, every stage is copied out behind its kernel.
hipError_t pbd_step_one(upsample_pbd_s* h, float* x, float* v, float* fx, float* fv, const PbdTrace* tr,
                        hipStream_t st) {
  const int64_t n = h->n;
  const PbdConst pc = pbd_const(h->p);
  const unsigned nb = nblocks(n);
  const bool lanes16 = pair_lanes(n) == 16;
  const unsigned nb_pairs = nblocks(n * pair_lanes(n));
  const bool lanes8 = iter_lanes(n) == 8;
  const unsigned nb_iter = nblocks(n * iter_lanes(n));
  const int K = h->K;
  float* rec = tr != nullptr ? tr->base : nullptr;
  hipError_t e = hipSuccess;
  if (h->counts_dirty) {  // every grid build expects zero counts (its scan leaves them so)
    hipLaunchKernelGGL(k_zero_u32, dim3(nblocks(h->n_cells)), dim3(kBlock), 0, st, h->g.counts, h->n_cells);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    h->counts_dirty = false;
  }
  auto record = [&](const float* src, int64_t m) {
    if (rec == nullptr || e != hipSuccess) return;
    e = copy_async(rec, src, m, st);
    rec += m;
  };
  // the prediction starts the first grid build: the stabilization's on x, or
  // without stabilization the solver's on x~
  if (h->p.stab_iters > 0)
    hipLaunchKernelGGL(k_pbd_predict<kKeysOfX>, dim3(nb), dim3(kBlock), 0, st, pc, n, x, v, h->xt, h->body,
                       h->inv_m, h->w, h->gc, h->g.keys, h->g.slot, h->g.counts);
  else
    hipLaunchKernelGGL(k_pbd_predict<kKeysOfXt>, dim3(nb), dim3(kBlock), 0, st, pc, n, x, v, h->xt, h->body,
                       h->inv_m, h->w, h->gc, h->g.keys, h->g.slot, h->g.counts);
  e = hipGetLastError();
  record(h->w, n);
  record(v, 3 * n);
  record(h->xt, 3 * n);
  // 2. stabilization on the start positions
  const float* x0 = x;
  if (h->p.stab_iters == 0 && tr != nullptr && e == hipSuccess) {
    // no stabilization pairs: the trace's lists of that phase are empty
    hipLaunchKernelGGL(k_zero_u32, dim3(nb), dim3(kBlock), 0, st, tr->pair_cnt, n);
    e = hipGetLastError();
  }
  if (h->p.stab_iters > 0) {
    if (e == hipSuccess) e = launch_build_grid_points(h->gc, x, h->body, n, h->n_cells, h->g, st, true);
    if (e == hipSuccess)
      hipLaunchKernelGGL(lanes16 ? k_pbd_pairs<16> : k_pbd_pairs<8>, dim3(nb_pairs), dim3(kBlock), 0, st, h->gc,
                         h->g.lr_sorted, h->g.cell_start, n, K, h->cnt, h->ids, h->overflow);
    if (e == hipSuccess && tr != nullptr) e = copy_pairs(h, tr, 0, st);
    float* out = h->xs;
    for (int it = 0; it < h->p.stab_iters && e == hipSuccess; ++it) {
      // the last iteration starts the solver phase's grid build on its x~
      const bool keys = it == h->p.stab_iters - 1;
      auto kern = keys ? (lanes8 ? k_pbd_stab<true, 8> : k_pbd_stab<true, 4>)
                       : (lanes8 ? k_pbd_stab<false, 8> : k_pbd_stab<false, 4>);
      hipLaunchKernelGGL(kern, dim3(nb_iter), dim3(kBlock), 0, st, pc, n, x0, out, h->xt, h->w, K, h->cnt, h->ids,
                         h->gc, h->g.keys, h->g.slot, h->g.counts);
      e = hipGetLastError();
      x0 = out;
      out = out == h->xs ? h->xs2 : h->xs;
      record(x0, 3 * n);
      record(h->xt, 3 * n);
    }
  }
  // 3. solver iterations on x~
  float* ta = h->xt;
  float* tb = h->xt2;
  if (e == hipSuccess) e = launch_build_grid_points(h->gc, ta, h->body, n, h->n_cells, h->g, st, true);
  if (e == hipSuccess)
    hipLaunchKernelGGL(lanes16 ? k_pbd_pairs<16> : k_pbd_pairs<8>, dim3(nb_pairs), dim3(kBlock), 0, st, h->gc,
                       h->g.lr_sorted, h->g.cell_start, n, K, h->cnt, h->ids, h->overflow);
  if (e == hipSuccess && tr != nullptr) e = copy_pairs(h, tr, 1, st);
  const bool fuse = x0 != x && h->p.solve_iters > 0;
  const FinishArgs fin{x, v, fx, fv};
  for (int it = 0; it < h->p.solve_iters && e == hipSuccess; ++it) {
    if (h->n_bodies > 0)
      hipLaunchKernelGGL(k_pbd_shape, dim3((unsigned)h->n_bodies), dim3(kShapeThreads), 0, st, n, ta, h->members,
                         h->body_ptr, h->rest, h->osum, h->cr);
    const bool last = fuse && it == h->p.solve_iters - 1;
    auto kern = last ? (lanes8 ? k_pbd_solve<true, 8> : k_pbd_solve<true, 4>)
                     : (lanes8 ? k_pbd_solve<false, 8> : k_pbd_solve<false, 4>);
    hipLaunchKernelGGL(kern, dim3(nb_iter), dim3(kBlock), 0, st, pc, n, ta, tb, x0, h->w, K, h->cnt, h->ids,
                       h->body, h->rest, h->cr, fin);
    e = hipGetLastError();
    float* t = ta;
    ta = tb;
    tb = t;
    record(h->cr, 12 * (int64_t)h->n_bodies);
    record(ta, 3 * n);
  }
  // 4. velocities, unless the last solver iteration wrote them
  if (e == hipSuccess && !fuse) {
    hipLaunchKernelGGL(k_pbd_finish, dim3(nb), dim3(kBlock), 0, st, pc, n, x0, ta, h->body, x, v, fx, fv);
    e = hipGetLastError();
  }
  record(x, 3 * n);
  record(v, 3 * n);
  return e;
}

}  // namespace

extern "C" {

int upsample_pbd_default_params(upsample_pbd_params* p) {
  if (p == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->r = 0.02f;
  p->dt = 0.005f;
  p->g[1] = -9.81f;
  p->mu_s = 0.35f;
  p->mu_k = 0.3f;
  p->stab_iters = 2;
  p->solve_iters = 5;
  p->mass_scaling = 1;
  for (int a = 0; a < 3; ++a) p->domain_hi[a] = 1.0f;
  p->max_neighbors = 32;
  return UPSAMPLE_OK;
}

int upsample_pbd_init(const upsample_pbd_params* p, int64_t n, const int32_t* body, const float* inv_mass,
                      const float* rest, upsample_pbd* out) {
  if (p == nullptr || out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (!(std::isfinite(p->r) && p->r > 0.0f && std::isfinite(p->dt) && p->dt > 0.0f)) return UPSAMPLE_ERR_INVALID_ARG;
  if (!(std::isfinite(p->mu_s) && std::isfinite(p->mu_k) && p->mu_s >= 0.0f && p->mu_k >= 0.0f))
    return UPSAMPLE_ERR_INVALID_ARG;
  if (p->stab_iters < 0 || p->solve_iters < 0 || p->max_neighbors < 1 || p->max_neighbors > 1024)
    return UPSAMPLE_ERR_INVALID_ARG;
  if (n < 0 || n >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_INVALID_ARG;
  if (n > 0 && (body == nullptr || inv_mass == nullptr || rest == nullptr)) return UPSAMPLE_ERR_INVALID_ARG;
  // the neighbour grid: cells of 2r (times 1.0001: float32 rounding never
  // moves a contact partner beyond the 27-cell stencil)
  const double cs = 2.0 * (double)p->r * 1.0001;
  GridConst gc;
  int64_t n_cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (!(std::isfinite(p->domain_lo[a]) && std::isfinite(p->domain_hi[a]) && p->domain_hi[a] > p->domain_lo[a]))
      return UPSAMPLE_ERR_INVALID_ARG;
    const double ext = ((double)p->domain_hi[a] - (double)p->domain_lo[a]) / cs;
    if (!(ext < 1048576.0)) return UPSAMPLE_ERR_GRID_TOO_LARGE;
    const int d = std::max(1, (int)std::ceil(ext));
    gc.dims[a] = d;
    gc.lo[a] = p->domain_lo[a];
    n_cells *= d;
  }
  if (n_cells >= ((int64_t)1 << 31)) return UPSAMPLE_ERR_GRID_TOO_LARGE;
  gc.inv_cs = (float)(1.0 / cs);
  gc.cs = (float)cs;
  gc.reach = 1;
  gc.h2 = (float)(4.0 * (double)p->r * (double)p->r);
  gc.inv_h2 = 0.0f;
  // rigid bodies: members grouped by body id (ids 0 .. n_bodies - 1)
  int n_bodies = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (body[i] < kStatic) return UPSAMPLE_ERR_INVALID_ARG;
    if (body[i] >= 0) n_bodies = std::max(n_bodies, body[i] + 1);
    if (body[i] != kStatic && !(std::isfinite(inv_mass[i]) && inv_mass[i] >= 0.0f)) return UPSAMPLE_ERR_INVALID_ARG;
  }
  std::vector<uint32_t> ptr((size_t)n_bodies + 1, 0u), members;
  for (int64_t i = 0; i < n; ++i)
    if (body[i] >= 0) ptr[(size_t)body[i] + 1] += 1u;
  for (int b = 0; b < n_bodies; ++b) {
    if (ptr[(size_t)b + 1] == 0u) return UPSAMPLE_ERR_INVALID_ARG;  // body ids must be dense
    ptr[(size_t)b + 1] += ptr[(size_t)b];
  }
  members.resize(ptr[(size_t)n_bodies]);
  {
    std::vector<uint32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      if (body[i] >= 0) members[fill[(size_t)body[i]]++] = (uint32_t)i;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return UPSAMPLE_ERR_NO_DEVICE;
  upsample_pbd h = new (std::nothrow) upsample_pbd_s();
  if (h == nullptr) return UPSAMPLE_ERR_OOM;
  h->p = *p;
  h->n = n;
  h->n_bodies = n_bodies;
  h->K = p->max_neighbors;
  h->gc = gc;
  h->n_cells = n_cells;
  const int64_t n_chunks = (n_cells + kScanChunk - 1) / kScanChunk;
  hipError_t e = hipSuccess;
#define ALLOC(ptr_, cnt_) \
  if (e == hipSuccess) e = dalloc(&(ptr_), (cnt_));
  ALLOC(h->g.keys, n)
  ALLOC(h->g.slot, n)
  ALLOC(h->g.tmp, n)
  ALLOC(h->g.perm, n)
  ALLOC(h->g.counts, n_cells)
  ALLOC(h->g.local, n_cells)
  ALLOC(h->g.chunk_sum, n_chunks + 1)
  ALLOC(h->g.cell_start, n_cells + 1)
  ALLOC(h->g.lr_sorted, n)
  ALLOC(h->body, n)
  ALLOC(h->inv_m, n)
  ALLOC(h->rest, 3 * n)
  ALLOC(h->members, (int64_t)members.size())
  ALLOC(h->body_ptr, n_bodies + 1)
  ALLOC(h->osum, 3 * (int64_t)n_bodies)
  ALLOC(h->cr, 12 * (int64_t)n_bodies)
  ALLOC(h->w, n)
  ALLOC(h->xt, 3 * n)
  ALLOC(h->xt2, 3 * n)
  ALLOC(h->xs, 3 * n)
  ALLOC(h->xs2, 3 * n)
  ALLOC(h->cnt, n)
  ALLOC(h->ids, n * (int64_t)h->K)
  ALLOC(h->overflow, 1)
#undef ALLOC
  if (e == hipSuccess && n > 0) e = hipMemcpy(h->body, body, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess && n > 0) e = hipMemcpy(h->inv_m, inv_mass, sizeof(float) * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess && n > 0) e = hipMemcpy(h->rest, rest, sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess && !members.empty())
    e = hipMemcpy(h->members, members.data(), sizeof(uint32_t) * members.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->body_ptr, ptr.data(), sizeof(uint32_t) * ptr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_bodies > 0) {
    std::vector<double> os((size_t)n_bodies * 3, 0.0);
    for (int64_t i = 0; i < n; ++i)
      if (body[i] >= 0)
        for (int a = 0; a < 3; ++a) os[(size_t)body[i] * 3 + a] += (double)rest[a * n + i];
    e = hipMemcpy(h->osum, os.data(), sizeof(double) * os.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(h->g.counts, 0, sizeof(uint32_t) * (size_t)n_cells);
  if (e == hipSuccess) e = hipMemset(h->overflow, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    pbd_free(h);
    delete h;
    return e == hipErrorOutOfMemory ? UPSAMPLE_ERR_OOM : UPSAMPLE_ERR_HIP;
  }
  *out = h;
  return UPSAMPLE_OK;
}

int upsample_pbd_step(upsample_pbd h, float* x, float* v, int32_t n_steps, float* frames_x, float* frames_v,
                      void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (n_steps < 0) return pbd_fail(h, UPSAMPLE_ERR_INVALID_ARG, "n_steps < 0");
  if (h->n > 0 && (x == nullptr || v == nullptr)) return pbd_fail(h, UPSAMPLE_ERR_INVALID_ARG, "x / v is NULL");
  if ((frames_x == nullptr) != (frames_v == nullptr))
    return pbd_fail(h, UPSAMPLE_ERR_INVALID_ARG, "frames_x and frames_v: both or neither");
  const int64_t n = h->n;
  if (n == 0 || n_steps == 0) return UPSAMPLE_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int32_t s = 0; s < n_steps && e == hipSuccess; ++s) {
    float* fx = frames_x != nullptr ? frames_x + (size_t)s * 3 * (size_t)n : nullptr;
    float* fv = frames_v != nullptr ? frames_v + (size_t)s * 3 * (size_t)n : nullptr;
    e = pbd_step_one(h, x, v, fx, fv, nullptr, st);
    if (e != hipSuccess) h->counts_dirty = true;
  }
  if (e != hipSuccess) return pbd_fail(h, UPSAMPLE_ERR_HIP, std::string("pbd_step: ") + hipGetErrorString(e));
  return UPSAMPLE_OK;
}

int upsample_pbd_debug_step(upsample_pbd h, float* x, float* v, float* trace, int64_t trace_len,
                            uint32_t* pair_cnt, uint32_t* pair_ids, void* stream) {
  if (h == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  if (trace_len != trace_floats(h)) return pbd_fail(h, UPSAMPLE_ERR_INVALID_ARG, "trace_len does not match");
  if (h->n > 0 && (x == nullptr || v == nullptr || trace == nullptr || pair_cnt == nullptr || pair_ids == nullptr))
    return pbd_fail(h, UPSAMPLE_ERR_INVALID_ARG, "NULL buffer");
  if (h->n == 0) return UPSAMPLE_OK;
  hipStream_t st = (hipStream_t)stream;
  const PbdTrace tr{trace, pair_cnt, pair_ids};
  hipError_t e = pbd_step_one(h, x, v, nullptr, nullptr, &tr, st);
  if (e != hipSuccess) h->counts_dirty = true;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return pbd_fail(h, UPSAMPLE_ERR_HIP, std::string("pbd_debug_step: ") + hipGetErrorString(e));
  return UPSAMPLE_OK;
}

int upsample_pbd_info(upsample_pbd h, int64_t* out) {
  if (h == nullptr || out == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  out[0] = h->n;
  out[1] = h->n_bodies;
  out[2] = h->K;
  out[3] = h->n_cells;
  out[4] = trace_floats(h);
  return UPSAMPLE_OK;
}

int upsample_pbd_status(upsample_pbd h, int64_t* overflow, void* stream) {
  if (h == nullptr || overflow == nullptr) return UPSAMPLE_ERR_INVALID_ARG;
  uint32_t f = 0;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&f, h->overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return pbd_fail(h, UPSAMPLE_ERR_HIP, std::string("pbd_status: ") + hipGetErrorString(e));
  *overflow = f;
  return UPSAMPLE_OK;
}

int upsample_pbd_destroy(upsample_pbd h) {
  if (h == nullptr) return UPSAMPLE_OK;
  (void)hipDeviceSynchronize();
  pbd_free(h);
  delete h;
  return UPSAMPLE_OK;
}

const char* upsample_pbd_last_error(upsample_pbd h) {
  if (h == nullptr) return "null handle";
  return h->last_error.c_str();
}

}  // extern "C"
