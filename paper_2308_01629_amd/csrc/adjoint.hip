// Adjoint of the upsampling step (an extension: the paper does not
// differentiate it).  Per HR particle: a first stencil walk recomputes the
// weighted sums, the argmax of the weights and the alpha branch; the forward
// blend, integration and walls are replayed to record which walls acted; the
// upstream gradient is pulled back through the walls, the integration and the
// blend; a second stencil walk distributes the weight gradients to the LR
// particles (float atomics into the caller's [3][n_lr] arrays, by original
// index) and to the HR position.
//
// Held fixed (piecewise differentiation): alpha branch, neighbour membership,
// argmax of w (ties: smallest original LR index), wall activations.
#include "kernels.hpp"

namespace ups {
namespace {

struct Pass1 {
  float S, Ux, Uy, Uz, M;
  uint32_t arg;
  bool gran;
};

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

__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a, WallTable wt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const GridConst& gc = a.gc;
  const float x = a.hx[i], y = a.hx[n + i], z = a.hx[2 * n + i];
  const float vx = a.hv[i], vy = a.hv[n + i], vz = a.hv[2 * n + i];
  int lo[3], hi[3];
  stencil_bounds(gc, x, y, z, lo, hi);

  // ---- pass 1: sums, argmax
  Pass1 p{0.f, 0.f, 0.f, 0.f, 0.f, 0xffffffffu, false};
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
          p.S += w;
          p.Ux = fmaf(w, V.x, p.Ux);
          p.Uy = fmaf(w, V.y, p.Uy);
          p.Uz = fmaf(w, V.z, p.Uz);
          if (w > p.M || (w == p.M && id < p.arg)) {
            p.M = w;
            p.arg = id;
          }
          p.gran |= (P.w == 0.0f);
        }
      }
    }
  if (!p.gran) {
    p.S = p.Ux = p.Uy = p.Uz = p.M = 0.f;
  }

  // ---- forward replay
  float tx = 0.f, ty = 0.f, tz = 0.f;
  bool A = true;
  if (p.S > 0.0f) {
    tx = p.Ux / p.S;
    ty = p.Uy / p.S;
    tz = p.Uz / p.S;
    A = (p.M <= a.sc.c1) || (p.M / p.S >= a.sc.c2);
  }
  const float alpha = A ? 1.0f - p.M : 0.0f;
  const float dt = a.sc.dt;
  const float fx = fmaf(dt, a.sc.g[0], vx), fy = fmaf(dt, a.sc.g[1], vy), fz = fmaf(dt, a.sc.g[2], vz);
  float nvx = fmaf(alpha, fx - tx, tx), nvy = fmaf(alpha, fy - ty, ty), nvz = fmaf(alpha, fz - tz, tz);
  float nx = fmaf(dt, nvx, x), ny = fmaf(dt, nvy, y), nz = fmaf(dt, nvz, z);
  uint32_t pushed = 0u, clipped = 0u;
  for (int k = 0; k < a.sc.n_walls; ++k) {
    const float* w = &wt.w[k * UPSAMPLE_WALL_FLOATS];
    const float wnx = w[0], wny = w[1], wnz = w[2], d = w[3];
    bool act = fmaf(w[6], nz, fmaf(w[5], ny, w[4] * nx)) >= w[7];
    if (w[11] > 0.0f) {
      const float rx = nx - w[8], ry = ny - w[9], rz = nz - w[10];
      const float rn = fmaf(wnz, rz, fmaf(wny, ry, wnx * rx));
      const float ix = fmaf(-rn, wnx, rx), iy = fmaf(-rn, wny, ry), iz = fmaf(-rn, wnz, rz);
      act = act && (sqrtf(fmaf(iz, iz, fmaf(iy, iy, ix * ix))) >= w[11]);
    }
    act = act && (fmaf(wnz, z, fmaf(wny, y, wnx * x)) - d >= 0.0f);
    const float pen = fmaf(wnz, nz, fmaf(wny, ny, wnx * nx)) - d;
    if (act && pen < a.sc.r_hr) {
      pushed |= 1u << k;
      const float push = a.sc.r_hr - pen;
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

  // ---- pull the upstream gradient back
  float gx = a.gx_out[i], gy = a.gx_out[n + i], gz = a.gx_out[2 * n + i];
  float hx = a.gv_out[i], hy = a.gv_out[n + i], hz = a.gv_out[2 * n + i];
  for (int k = a.sc.n_walls - 1; k >= 0; --k) {
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
  const float om = 1.0f - alpha;
  const float gM = A ? -g_alpha : 0.0f;
  float gUx = 0.f, gUy = 0.f, gUz = 0.f, gS = 0.f;
  if (p.S > 0.0f) {
    const float inv = 1.0f / p.S;
    gUx = om * qx * inv;
    gUy = om * qy * inv;
    gUz = om * qz * inv;
    gS = -(gUx * tx + gUy * ty + gUz * tz);
  }

  // ---- pass 2: weight gradients to LR and HR positions, LR velocities
  if (p.gran) {
    const float k2 = -6.0f * gc.inv_h2;  // dw/ds = -3 t^2 / h2, times 2 for d(s)/d(X)
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
            float gw = fmaf(gUz, V.z, fmaf(gUy, V.y, gUx * V.x)) + gS;
            if (id == p.arg) gw += gM;
            unsafeAtomicAdd(&a.g_lr_v[id], w * gUx);
            unsafeAtomicAdd(&a.g_lr_v[nl + id], w * gUy);
            unsafeAtomicAdd(&a.g_lr_v[2 * nl + id], w * gUz);
            const float c = gw * k2 * t * t;
            const float dx = P.x - x, dy = P.y - y, dz = P.z - z;
            unsafeAtomicAdd(&a.g_lr_x[id], c * dx);
            unsafeAtomicAdd(&a.g_lr_x[nl + id], c * dy);
            unsafeAtomicAdd(&a.g_lr_x[2 * nl + id], c * dz);
            gx = fmaf(-c, dx, gx);
            gy = fmaf(-c, dy, gy);
            gz = fmaf(-c, dz, gz);
          }
        }
      }
  }
  a.gx_in[i] = gx;
  a.gx_in[n + i] = gy;
  a.gx_in[2 * n + i] = gz;
  a.gv_in[i] = alpha * qx;
  a.gv_in[n + i] = alpha * qy;
  a.gv_in[2 * n + i] = alpha * qz;
}

}  // namespace

hipError_t launch_adjoint(const AdjointArgs& a, const WallTable& walls, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adjoint, dim3(blocks), dim3(kBlock), 0, st, a, walls);
  return hipGetLastError();
}

}  // namespace ups
