"""Plain CPU oracle for the LR simulation step (Section 3 and Algorithm 1):
position-based dynamics with contact and friction constraints, constraint
averaging, stabilization iterations, height-scaled masses, and shape-matching
constraints that couple rigid bodies to the granular material.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.  Float64 NumPy; numpy's SVD gives the polar
decomposition.

One step of dt (Algorithm 1), LR particles of radius r:

1. Dynamic particles: v += dt g; every particle: x~ = x + dt v.  The inverse
   of the scaled mass is w*_i = w_i exp(h(x_i)) (m* = m exp(-h)), h the height
   above the ground plane, from the positions at the start of the step.
2. Stabilization: the contact pairs of the start positions x are generated;
   in each stabilization iteration every pair that still overlaps gives its
   contact displacement (below), each particle's displacements are averaged
   (divided by its number of active constraints) and added to x and to x~.
3. The contact pairs of x~ are generated, plus one shape-matching constraint
   per rigid particle; in each solver iteration every constraint is evaluated
   at the same x~ (Jacobi), the displacements averaged and added to x~.
4. v = (x~ - x) / dt, x = x~ (static particles keep x and v = 0).

Contact of a pair (i, j), x_ij = x~_j - x~_i, d = |x_ij| < 2r (Section 3):
    dx_i = -w_i/(w_i + w_j) (2r - d) x_ij / d,   dx_j = +w_j/(w_i + w_j) (2r - d) x_ij / d
with the scaled inverse masses.  Friction of the same pair (solver
iterations): the relative displacement Dx = (x'_i - x0_i) - (x'_j - x0_j),
x' the positions after the pair's contact displacement and x0 the positions
at the start of the step (after stabilization); its part perpendicular to
x_ij, Dt; f = Dt if |Dt| < 2 r mu_s, else Dt min(2 r mu_k / |Dt|, 1); then
dx_i -= w_i/(w_i+w_j) f, dx_j += w_j/(w_i+w_j) f.  Contact and friction of a
pair count as one constraint of each particle.

Shape matching of a rigid body (its particles have equal masses): c the mean
of its particles' x~, C = sum (x~_i - c) o_i^T with the rest offsets o_i,
R the rotation of the polar decomposition of C (C = U S V^T, R = U V^T, the
sign of U's last column flipped if det R < 0), dx_i = R o_i + c - x~_i.

Readings (listed with the others in the design notes):

* "relative height" h is the height above the ground plane in metres, unscaled.
* The paper prints the friction thresholds as 2 r_LR mu_s and 2 r_LR mu_k
  (its text speaks of the penetration depth): the printed formulas are
  followed.  The printed relative displacement (x~_i - x_i) - (x~_j - x_j) is
  read with x the positions at the start of the step, as in the method the
  paper builds on; read as the pair's own contact displacements it would be
  normal to x_ij and leave no tangential part.
* Stabilization pairs come from the start positions, solver pairs from x~
  after stabilization (each generated once per step; a generated pair acts
  while it overlaps).  Pairs of two static particles or of two particles of
  one rigid body are not generated.
* Static (boundary) particles have inverse mass 0; all constraints of one
  iteration are evaluated at the positions the iteration starts from.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree

F64 = np.float64
GRANULAR = -1
STATIC = -2


@dataclass
class PBDParams:
    r: float
    dt: float = 0.005                   # Section 5.2: default LR time step
    g: Tuple[float, float, float] = (0.0, -9.81, 0.0)
    mu_s: float = 0.35                  # Section 5.2: static friction
    mu_k: float = 0.3                   # Section 5.2: kinetic friction
    ground_y: float = 0.0
    stab_iters: int = 2                 # Algorithm 1
    solve_iters: int = 5
    mass_scaling: bool = True


def scaled_inv_mass(x, inv_m, prm: PBDParams) -> np.ndarray:
    """w* = w exp(h), h = y - ground (m* = m exp(-h))."""
    if not prm.mass_scaling:
        return np.asarray(inv_m, dtype=F64).copy()
    return np.asarray(inv_m, dtype=F64) * np.exp(np.asarray(x, dtype=F64)[1] - prm.ground_y)


def contact_pairs(P, body, r) -> np.ndarray:
    """Pairs (i < j) closer than 2r, without static-static and same-body
    pairs; P [3, N]."""
    P = np.asarray(P, dtype=F64)
    if P.shape[1] < 2:
        return np.zeros((0, 2), dtype=np.int64)
    pr = np.array(sorted(cKDTree(P.T).query_pairs(2.0 * r * (1 + 1e-9))), dtype=np.int64).reshape(-1, 2)
    if pr.size == 0:
        return pr
    i, j = pr[:, 0], pr[:, 1]
    d = np.linalg.norm(P[:, j] - P[:, i], axis=0)
    bi, bj = body[i], body[j]
    keep = (d < 2.0 * r) & ~((bi == STATIC) & (bj == STATIC)) & ~((bi >= 0) & (bi == bj))
    return pr[keep]


def _contact(P, pairs, w, r):
    """Per-pair contact displacements (dx_i, dx_j) [3, K] and the active mask."""
    i, j = pairs[:, 0], pairs[:, 1]
    xij = P[:, j] - P[:, i]
    d = np.linalg.norm(xij, axis=0)
    wi, wj = w[i], w[j]
    ws = wi + wj
    act = (d < 2.0 * r) & (d > 0.0) & (ws > 0.0)
    s = np.where(act, (2.0 * r - d) / np.where(d > 0, d, 1.0), 0.0)
    mi = np.where(act, wi / np.where(ws > 0, ws, 1.0), 0.0)
    mj = np.where(act, wj / np.where(ws > 0, ws, 1.0), 0.0)
    return -mi * s * xij, mj * s * xij, act, xij, mi, mj


def polar_rotation(C) -> np.ndarray:
    """Rotation of the polar decomposition C = R S (S symmetric positive)."""
    U, _, Vt = np.linalg.svd(C)
    R = U @ Vt
    if np.linalg.det(R) < 0.0:
        U[:, 2] *= -1.0
        R = U @ Vt
    return R


def shape_matching(P, body, rest):
    """Shape-matching displacements [3, N] (zero for non-rigid particles)."""
    dx = np.zeros_like(P)
    for b in np.unique(body[body >= 0]):
        idx = np.nonzero(body == b)[0]
        c = P[:, idx].mean(axis=1)
        o = rest[:, idx]
        C = (P[:, idx] - c[:, None]) @ o.T
        R = polar_rotation(C)
        dx[:, idx] = R @ o + c[:, None] - P[:, idx]
    return dx


def step(x, v, body, inv_m, rest, prm: PBDParams, return_info: bool = False):
    """One LR step (Algorithm 1).  x, v: [3, N]; body: int [N] (GRANULAR = -1,
    STATIC = -2, rigid body ids >= 0); inv_m: [N] (0 for static); rest: [3, N]
    rest offsets of rigid particles from their body's centre (ignored
    otherwise).  Returns float64 (x, v) after the step."""
    x = np.asarray(x, dtype=F64).copy()
    v = np.asarray(v, dtype=F64).copy()
    body = np.asarray(body)
    rest = np.asarray(rest, dtype=F64)
    g = np.asarray(prm.g, dtype=F64)
    dyn = body != STATIC
    r, dt = F64(prm.r), F64(prm.dt)
    # 1. prediction and scaled masses
    v[:, dyn] += dt * g[:, None]
    v[:, ~dyn] = 0.0
    xt = x + dt * v
    w = scaled_inv_mass(x, inv_m, prm)
    w[~dyn] = 0.0
    N = x.shape[1]
    info = {"stab_pairs": 0, "solve_pairs": 0, "min_margin": np.inf}
    # 2. stabilization on the start positions, applied to x and x~
    sp = contact_pairs(x, body, r)
    info["stab_pairs"] = sp.shape[0]
    for _ in range(prm.stab_iters):
        di, dj, act, _, _, _ = _contact(x, sp, w, r)
        acc = np.zeros((3, N))
        cnt = np.zeros(N)
        np.add.at(acc.T, sp[:, 0], di.T)
        np.add.at(acc.T, sp[:, 1], dj.T)
        np.add.at(cnt, sp[:, 0], act.astype(F64))
        np.add.at(cnt, sp[:, 1], act.astype(F64))
        upd = np.where(cnt > 0, acc / np.maximum(cnt, 1.0), 0.0)
        x += upd
        xt += upd
    x0 = x.copy()
    # 3. solver iterations on x~: contact + friction per pair, shape matching
    pairs = contact_pairs(xt, body, r)
    info["solve_pairs"] = pairs.shape[0]
    rigid = body >= 0
    for _ in range(prm.solve_iters):
        di, dj, act, xij, mi, mj = _contact(xt, pairs, w, r)
        i, j = pairs[:, 0], pairs[:, 1]
        Dx = (xt[:, i] + di - x0[:, i]) - (xt[:, j] + dj - x0[:, j])
        n2 = np.sum(xij * xij, axis=0)
        Dt = Dx - np.sum(Dx * xij, axis=0) / np.where(n2 > 0, n2, 1.0) * xij
        lt = np.linalg.norm(Dt, axis=0)
        static_f = lt < 2.0 * r * prm.mu_s
        scale = np.where(static_f, 1.0, np.minimum(2.0 * r * prm.mu_k / np.where(lt > 0, lt, 1.0), 1.0))
        f = Dt * scale
        di = di - mi * f
        dj = dj + mj * f
        di[:, ~act] = 0.0
        dj[:, ~act] = 0.0
        acc = np.zeros((3, N))
        cnt = np.zeros(N)
        np.add.at(acc.T, i, di.T)
        np.add.at(acc.T, j, dj.T)
        np.add.at(cnt, i, act.astype(F64))
        np.add.at(cnt, j, act.astype(F64))
        if rigid.any():
            acc += shape_matching(xt, body, rest)
            cnt += rigid.astype(F64)
        if act.any():
            dd = np.linalg.norm(xij[:, act], axis=0)
            info["min_margin"] = min(info["min_margin"], float(np.min(np.abs(dd - 2.0 * r))),
                                     float(np.min(np.abs(lt[act] - 2.0 * r * prm.mu_s))))
        xt += np.where(cnt > 0, acc / np.maximum(cnt, 1.0), 0.0)
    # 4. velocities from the positions
    vn = np.where(dyn, (xt - x) / dt, 0.0)
    xn = np.where(dyn, xt, x)
    if return_info:
        return xn, vn, info
    return xn, vn
