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
// uniform grid of cells at least 2r wide, stable counting sort).
//
// Per step: k_pbd_predict, grid + k_pbd_pairs on the start positions,
// stab_iters x k_pbd_stab, grid + k_pbd_pairs on the predicted positions,
// solve_iters x (k_pbd_shape per rigid body, k_pbd_solve), k_pbd_finish.
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
__global__ __launch_bounds__(kBlock) void k_pbd_predict(PbdConst pc, int64_t n, const float* __restrict__ x,
                                                        float* __restrict__ v, float* __restrict__ xt,
                                                        const int32_t* __restrict__ body,
                                                        const float* __restrict__ inv_m, float* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const bool stat = body[i] == kStatic;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float va = stat ? 0.0f : fmaf(pc.dt, pc.g[a], v[a * n + i]);
    v[a * n + i] = va;
    xt[a * n + i] = fmaf(pc.dt, va, x[a * n + i]);
  }
  float wi = stat ? 0.0f : inv_m[i];
  if (pc.mass_scaling) wi *= expf(x[n + i] - pc.ground_y);
  w[i] = wi;
}

// Contact list of each particle: the other particles closer than 2r
// (squared distance rounded as in the upsampling's membership predicate,
// against fl32(4 r^2)), without static-static and same-body pairs, in grid
// walk order.  A list longer than K sets *overflow.
__global__ __launch_bounds__(kBlock) void k_pbd_pairs(GridConst gc, const LRPoint* __restrict__ sorted,
                                                      const uint32_t* __restrict__ cell_start, int64_t n,
                                                      const float* __restrict__ P, const int32_t* __restrict__ body,
                                                      int K, uint32_t* __restrict__ cnt, uint32_t* __restrict__ ids,
                                                      uint32_t* overflow) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float x = P[i], y = P[n + i], z = P[2 * n + i];
  const int bi = body[i];
  const int cx = cell_coord(x, gc.lo[0], gc.inv_cs, gc.dims[0]);
  const int cy = cell_coord(y, gc.lo[1], gc.inv_cs, gc.dims[1]);
  const int cz = cell_coord(z, gc.lo[2], gc.inv_cs, gc.dims[2]);
  const int R = gc.reach;
  uint32_t c = 0;
  for (int zz = max(cz - R, 0); zz <= min(cz + R, gc.dims[2] - 1); ++zz)
    for (int yy = max(cy - R, 0); yy <= min(cy + R, gc.dims[1] - 1); ++yy) {
      const uint32_t row = (uint32_t)gc.dims[0] * ((uint32_t)yy + (uint32_t)gc.dims[1] * (uint32_t)zz);
      const uint32_t b = cell_start[row + (uint32_t)max(cx - R, 0)];
      const uint32_t e = cell_start[row + (uint32_t)min(cx + R, gc.dims[0] - 1) + 1u];
      for (uint32_t q = b; q < e; ++q) {
        const LRPoint L = sorted[q];
        const uint32_t j = __float_as_uint(L.v.w);
        if (j == (uint32_t)i) continue;
        const int bj = body[j];
        if ((bi == kStatic && bj == kStatic) || (bi >= 0 && bi == bj)) continue;
        if (sq_dist(L.p.x, L.p.y, L.p.z, x, y, z) < gc.h2) {
          if ((int)c < K) ids[(int64_t)i * K + c] = j;
          ++c;
        }
      }
    }
  if ((int)c > K) atomicOr(overflow, 1u);
  cnt[i] = min(c, (uint32_t)K);
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
// contact displacement goes to x (xs_out) and to x~ (in place).
__global__ __launch_bounds__(kBlock) void k_pbd_stab(PbdConst pc, int64_t n, const float* __restrict__ xs_in,
                                                     float* __restrict__ xs_out, float* __restrict__ xt,
                                                     const float* __restrict__ w, int K,
                                                     const uint32_t* __restrict__ cnt,
                                                     const uint32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float Pi[3];
  load3(xs_in, n, i, Pi);
  const float wi = w[i];
  float acc[3] = {0.f, 0.f, 0.f};
  int na = 0;
  const uint32_t c = cnt[i];
  for (uint32_t k = 0; k < c; ++k) {
    const int64_t j = ids[i * K + k];
    float Pj[3];
    load3(xs_in, n, j, Pj);
    const float wj = w[j];
    PairGeo g;
    if (!contact_geo(Pi, Pj, wi, wj, pc.r2, g)) continue;
    const float mi = wi / (wi + wj);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] -= mi * g.s * g.xij[a];
    ++na;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = na > 0 ? acc[a] / (float)na : 0.0f;
    xs_out[a * n + i] = Pi[a] + u;
    xt[a * n + i] += u;
  }
}

// Shape matching, per rigid body (one block each): centre c = mean of the
// body's x~, C = sum (x~ - c) o^T in double, and the rotation R of the polar
// decomposition of C (from the eigenvectors of C^T C, cyclic Jacobi in
// double): R = sum_k u_k v_k^T with u_k = C v_k / sigma_k for the two largest
// singular values and u_3 = u_1 x u_2, v_3 signed so that det R = +1.
// Writes (c, R) as 12 floats per body.
__device__ void jacobi_eig3(double A[3][3], double V[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) V[a][b] = a == b ? 1.0 : 0.0;
  const double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    if (!(off > 1e-30 * scale)) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- J^T A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
}

__global__ __launch_bounds__(kBlock) void k_pbd_shape(int64_t n, const float* __restrict__ xt,
                                                      const uint32_t* __restrict__ members,
                                                      const uint32_t* __restrict__ body_ptr,
                                                      const float* __restrict__ rest, float* __restrict__ cr) {
  __shared__ double red[kBlock][9];
  __shared__ double cen[3];
  const int b = blockIdx.x;
  const uint32_t p0 = body_ptr[b], p1 = body_ptr[b + 1];
  const int t = threadIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  for (uint32_t q = p0 + t; q < p1; q += kBlock) {
    const int64_t i = members[q];
    for (int a = 0; a < 3; ++a) s[a] += (double)xt[a * n + i];
  }
  for (int a = 0; a < 3; ++a) red[t][a] = s[a];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (t < h)
      for (int a = 0; a < 3; ++a) red[t][a] += red[t + h][a];
    __syncthreads();
  }
  if (t == 0)
    for (int a = 0; a < 3; ++a) cen[a] = red[0][a] / (double)(p1 - p0);
  __syncthreads();
  double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (uint32_t q = p0 + t; q < p1; q += kBlock) {
    const int64_t i = members[q];
    double dxa[3], o[3];
    for (int a = 0; a < 3; ++a) {
      dxa[a] = (double)xt[a * n + i] - cen[a];
      o[a] = (double)rest[a * n + i];
    }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) C[3 * a + c] += dxa[a] * o[c];
  }
  __syncthreads();
  for (int k = 0; k < 9; ++k) red[t][k] = C[k];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (t < h)
      for (int k = 0; k < 9; ++k) red[t][k] += red[t + h][k];
    __syncthreads();
  }
  if (t != 0) return;
  double M[3][3], A[3][3], V[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) M[a][c] = red[0][3 * a + c];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += M[k][a] * M[k][c];
      A[a][c] = acc;
    }
  jacobi_eig3(A, V);
  // order the eigenpairs by decreasing eigenvalue
  int ord[3] = {0, 1, 2};
  for (int x = 0; x < 2; ++x)
    for (int y = x + 1; y < 3; ++y)
      if (A[ord[y]][ord[y]] > A[ord[x]][ord[x]]) {
        const int tmp = ord[x];
        ord[x] = ord[y];
        ord[y] = tmp;
      }
  double v[3][3], u[3][3];
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 3; ++a) v[k][a] = V[a][ord[k]];
  for (int k = 0; k < 2; ++k) {
    double nrm = 0.0;
    for (int a = 0; a < 3; ++a) {
      double acc = 0.0;
      for (int c = 0; c < 3; ++c) acc += M[a][c] * v[k][c];
      u[k][a] = acc;
      nrm += acc * acc;
    }
    nrm = sqrt(nrm);
    for (int a = 0; a < 3; ++a) u[k][a] = nrm > 0.0 ? u[k][a] / nrm : (a == k ? 1.0 : 0.0);
  }
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  const double detv = v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) -
                      v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
                      v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
  if (detv < 0.0)
    for (int a = 0; a < 3; ++a) v[2][a] = -v[2][a];
  float* o = cr + 12 * b;
  for (int a = 0; a < 3; ++a) o[a] = (float)cen[a];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += u[k][a] * v[k][c];
      o[3 + 3 * a + c] = (float)acc;
    }
}

// 3. One solver iteration: contact and friction of each pair (one constraint)
// plus the shape-matching displacement of rigid particles, averaged.
__global__ __launch_bounds__(kBlock) void k_pbd_solve(PbdConst pc, int64_t n, const float* __restrict__ xt_in,
                                                      float* __restrict__ xt_out, const float* __restrict__ x0,
                                                      const float* __restrict__ w, int K,
                                                      const uint32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ ids,
                                                      const int32_t* __restrict__ body,
                                                      const float* __restrict__ rest, const float* __restrict__ cr) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float Pi[3], X0i[3];
  load3(xt_in, n, i, Pi);
  load3(x0, n, i, X0i);
  const float wi = w[i];
  float acc[3] = {0.f, 0.f, 0.f};
  int na = 0;
  const uint32_t c = cnt[i];
  for (uint32_t k = 0; k < c; ++k) {
    const int64_t j = ids[i * K + k];
    float Pj[3], X0j[3];
    load3(xt_in, n, j, Pj);
    const float wj = w[j];
    PairGeo g;
    if (!contact_geo(Pi, Pj, wi, wj, pc.r2, g)) continue;
    load3(x0, n, j, X0j);
    const float mi = wi / (wi + wj), mj = wj / (wi + wj);
    float Dx[3], ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ci[a] = -mi * g.s * g.xij[a];
      const float cj = mj * g.s * g.xij[a];
      Dx[a] = ((Pi[a] + ci[a]) - X0i[a]) - ((Pj[a] + cj) - X0j[a]);
    }
    // friction on the part of Dx perpendicular to x_ij
    const float dn = fmaf(Dx[2], g.xij[2], fmaf(Dx[1], g.xij[1], Dx[0] * g.xij[0])) / g.d2;
    float Dt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Dt[a] = Dx[a] - dn * g.xij[a];
    const float lt = sqrtf(fmaf(Dt[2], Dt[2], fmaf(Dt[1], Dt[1], Dt[0] * Dt[0])));
    const float scale = lt < pc.mu_s2r ? 1.0f : fminf(pc.mu_k2r / lt, 1.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] += ci[a] - mi * (Dt[a] * scale);
    ++na;
  }
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
    ++na;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) xt_out[a * n + i] = Pi[a] + (na > 0 ? acc[a] / (float)na : 0.0f);
}

// 4. v = (x~ - x0) / dt, x = x~ (static particles keep x0, v = 0), x0 the
// stabilized start positions; optionally the new state into a frame buffer.
// x0 may alias x (not restrict-qualified): each thread reads its element
// before writing it.
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
  float* cr;
  float *w, *xt, *xt2, *xs;
  uint32_t *cnt, *ids, *overflow;
  std::string last_error;
};

namespace {

int pbd_fail(upsample_pbd h, int code, const std::string& m) {
  if (h != nullptr) h->last_error = m;
  return code;
}

void pbd_free(upsample_pbd h) {
  void* ptrs[] = {h->g.keys, h->g.slot, h->g.tmp, h->g.perm, h->g.counts, h->g.local, h->g.chunk_sum,
                  h->g.cell_start, h->g.lr_sorted, h->body, h->inv_m, h->rest, h->members, h->body_ptr, h->cr,
                  h->w, h->xt, h->xt2, h->xs, h->cnt, h->ids, h->overflow};
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

// One step (Algorithm 1).  The stabilization ping-pongs between x and h->xs,
// the solver between h->xt and h->xt2.  With a trace, every stage is copied
// out behind its kernel.
hipError_t pbd_step_one(upsample_pbd_s* h, float* x, float* v, float* fx, float* fv, const PbdTrace* tr,
                        hipStream_t st) {
  const int64_t n = h->n;
  const PbdConst pc = pbd_const(h->p);
  const unsigned nb = nblocks(n);
  const int K = h->K;
  float* rec = tr != nullptr ? tr->base : nullptr;
  hipError_t e = hipSuccess;
  auto record = [&](const float* src, int64_t m) {
    if (rec == nullptr || e != hipSuccess) return;
    e = copy_async(rec, src, m, st);
    rec += m;
  };
  hipLaunchKernelGGL(k_pbd_predict, dim3(nb), dim3(kBlock), 0, st, pc, n, x, v, h->xt, h->body, h->inv_m, h->w);
  e = hipGetLastError();
  record(h->w, n);
  record(v, 3 * n);
  record(h->xt, 3 * n);
  // 2. stabilization on the start positions
  float* sa = x;
  float* sb = h->xs;
  if (e == hipSuccess) e = launch_build_grid(h->gc, sa, sa, nullptr, n, h->n_cells, h->g, st);
  if (e == hipSuccess)
    hipLaunchKernelGGL(k_pbd_pairs, dim3(nb), dim3(kBlock), 0, st, h->gc, h->g.lr_sorted, h->g.cell_start, n, sa,
                       h->body, K, h->cnt, h->ids, h->overflow);
  if (e == hipSuccess && tr != nullptr) e = copy_pairs(h, tr, 0, st);
  for (int it = 0; it < h->p.stab_iters && e == hipSuccess; ++it) {
    hipLaunchKernelGGL(k_pbd_stab, dim3(nb), dim3(kBlock), 0, st, pc, n, sa, sb, h->xt, h->w, K, h->cnt, h->ids);
    e = hipGetLastError();
    float* t = sa;
    sa = sb;
    sb = t;
    record(sa, 3 * n);
    record(h->xt, 3 * n);
  }
  const float* x0 = sa;  // stabilized start positions
  // 3. solver iterations on x~
  float* ta = h->xt;
  float* tb = h->xt2;
  if (e == hipSuccess) e = launch_build_grid(h->gc, ta, ta, nullptr, n, h->n_cells, h->g, st);
  if (e == hipSuccess)
    hipLaunchKernelGGL(k_pbd_pairs, dim3(nb), dim3(kBlock), 0, st, h->gc, h->g.lr_sorted, h->g.cell_start, n, ta,
                       h->body, K, h->cnt, h->ids, h->overflow);
  if (e == hipSuccess && tr != nullptr) e = copy_pairs(h, tr, 1, st);
  for (int it = 0; it < h->p.solve_iters && e == hipSuccess; ++it) {
    if (h->n_bodies > 0)
      hipLaunchKernelGGL(k_pbd_shape, dim3((unsigned)h->n_bodies), dim3(kBlock), 0, st, n, ta, h->members,
                         h->body_ptr, h->rest, h->cr);
    hipLaunchKernelGGL(k_pbd_solve, dim3(nb), dim3(kBlock), 0, st, pc, n, ta, tb, x0, h->w, K, h->cnt, h->ids,
                       h->body, h->rest, h->cr);
    e = hipGetLastError();
    float* t = ta;
    ta = tb;
    tb = t;
    record(h->cr, 12 * (int64_t)h->n_bodies);
    record(ta, 3 * n);
  }
  // 4. velocities; x0 may be x itself (an even number of stabilization
  // iterations): each thread reads its own element before writing it
  if (e == hipSuccess) {
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
  ALLOC(h->cr, 12 * (int64_t)n_bodies)
  ALLOC(h->w, n)
  ALLOC(h->xt, 3 * n)
  ALLOC(h->xt2, 3 * n)
  ALLOC(h->xs, 3 * n)
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
