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

``predict``, ``stab_iteration``, ``solve_iteration`` and ``finish`` are these
steps one at a time; ``step`` chains them.  ``force_act`` / ``force_static``
fix a pair's contact or friction decision, so that a test can recompute a
stage with the other decision of a pair that sits on a threshold.

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

from dataclasses import dataclass
from typing import Tuple

import numpy as np
from scipy.spatial import cKDTree

F32 = np.float32
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


def contact_pairs(P, body, r, f32: bool = False) -> np.ndarray:
    """Pairs (i < j) closer than 2r, without static-static and same-body
    pairs; P [3, N].  With f32=True the distance test is taken in float32 like
    the GPU's (the float32 positions, d = fl(P_j - P_i) per axis, separately
    rounded squares and sums, against fl32(4 r^2)), so that both sides decide
    each pair identically."""
    P = np.asarray(P, dtype=F32 if f32 else F64)
    if P.shape[1] < 2:
        return np.zeros((0, 2), dtype=np.int64)
    pr = np.array(sorted(cKDTree(P.T.astype(F64)).query_pairs(2.0 * float(r) * (1 + 1e-6))),
                  dtype=np.int64).reshape(-1, 2)
    if pr.size == 0:
        return pr
    i, j = pr[:, 0], pr[:, 1]
    if f32:
        d = P[:, j] - P[:, i]
        s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        close = s < F32(4.0 * F64(F32(r)) ** 2)
    else:
        close = np.linalg.norm(P[:, j] - P[:, i], axis=0) < 2.0 * r
    bi, bj = body[i], body[j]
    keep = close & ~((bi == STATIC) & (bj == STATIC)) & ~((bi >= 0) & (bi == bj))
    return pr[keep]


def _forced(own, force):
    """A decision per pair: the oracle's own, or the one ``force`` fixes
    (int8 per pair: -1 own, 0 false, 1 true)."""
    if force is None:
        return own
    force = np.asarray(force)
    return np.where(force < 0, own, force > 0)


def _contact(P, pairs, w, r, force_act=None):
    """Per-pair contact displacements (dx_i, dx_j) [3, K], the active mask and
    the signed distance margin d - 2r."""
    i, j = pairs[:, 0], pairs[:, 1]
    xij = P[:, j] - P[:, i]
    d = np.linalg.norm(xij, axis=0)
    wi, wj = w[i], w[j]
    ws = wi + wj
    act = _forced((d < 2.0 * r) & (d > 0.0) & (ws > 0.0), force_act) & (d > 0.0) & (ws > 0.0)
    s = np.where(act, (2.0 * r - d) / np.where(d > 0, d, 1.0), 0.0)
    mi = np.where(act, wi / np.where(ws > 0, ws, 1.0), 0.0)
    mj = np.where(act, wj / np.where(ws > 0, ws, 1.0), 0.0)
    return -mi * s * xij, mj * s * xij, act, xij, mi, mj, d - 2.0 * r


def polar_rotation(C) -> np.ndarray:
    """Rotation of the polar decomposition C = R S (S symmetric positive)."""
    U, _, Vt = np.linalg.svd(C)
    R = U @ Vt
    if np.linalg.det(R) < 0.0:
        U[:, 2] *= -1.0
        R = U @ Vt
    return R


def shape_matching(P, body, rest, return_frames: bool = False):
    """Shape-matching displacements [3, N] (zero for non-rigid particles);
    with return_frames also each body's (c, R), bodies 0 .. B-1."""
    dx = np.zeros_like(P)
    frames = {}
    for b in np.unique(body[body >= 0]):
        idx = np.nonzero(body == b)[0]
        c = P[:, idx].mean(axis=1)
        o = rest[:, idx]
        C = (P[:, idx] - c[:, None]) @ o.T
        R = polar_rotation(C)
        dx[:, idx] = R @ o + c[:, None] - P[:, idx]
        frames[int(b)] = (c, R)
    if return_frames:
        return dx, frames
    return dx


def _average(N, pairs, di, dj, act, extra=None, extra_cnt=None):
    """Each particle's summed displacements divided by its number of active
    constraints (constraint averaging)."""
    acc = np.zeros((3, N))
    cnt = np.zeros(N)
    np.add.at(acc.T, pairs[:, 0], di.T)
    np.add.at(acc.T, pairs[:, 1], dj.T)
    np.add.at(cnt, pairs[:, 0], act.astype(F64))
    np.add.at(cnt, pairs[:, 1], act.astype(F64))
    if extra is not None:
        acc += extra
        cnt += extra_cnt
    return np.where(cnt > 0, acc / np.maximum(cnt, 1.0), 0.0)


def predict(x, v, body, inv_m, prm: PBDParams):
    """Step 1: velocities with gravity (zero for static particles), the
    predicted positions x~ and the scaled inverse masses (0 for static)."""
    x = np.asarray(x, dtype=F64)
    v = np.asarray(v, dtype=F64).copy()
    dyn = np.asarray(body) != STATIC
    v[:, dyn] += F64(prm.dt) * np.asarray(prm.g, dtype=F64)[:, None]
    v[:, ~dyn] = 0.0
    xt = x + F64(prm.dt) * v
    w = scaled_inv_mass(x, inv_m, prm)
    w[~dyn] = 0.0
    return v, xt, w


def stab_iteration(x, xt, pairs, w, r, force_act=None):
    """Step 2, one stabilization iteration: the averaged contact displacements
    of the pairs at x, added to x and to x~.  Returns (x, x~, per-pair
    distance margin d - 2r)."""
    x = np.asarray(x, dtype=F64)
    xt = np.asarray(xt, dtype=F64)
    di, dj, act, _, _, _, margin = _contact(x, pairs, w, F64(r), force_act)
    upd = _average(x.shape[1], pairs, di, dj, act)
    return x + upd, xt + upd, margin


def solve_iteration(xt, x0, pairs, w, body, rest, prm: PBDParams, force_act=None, force_static=None):
    """Step 3, one solver iteration on x~ (Jacobi): contact and friction of
    each pair as one constraint, one shape-matching constraint per rigid
    particle, averaged.  Returns (x~, info) with the per-pair distance margin
    d - 2r, the friction margin |Dt| - 2 r mu_s and the bodies' (c, R)."""
    xt = np.asarray(xt, dtype=F64)
    x0 = np.asarray(x0, dtype=F64)
    body = np.asarray(body)
    r = F64(prm.r)
    di, dj, act, xij, mi, mj, margin = _contact(xt, pairs, w, r, force_act)
    i, j = pairs[:, 0], pairs[:, 1]
    Dx = (xt[:, i] + di - x0[:, i]) - (xt[:, j] + dj - x0[:, j])
    n2 = np.sum(xij * xij, axis=0)
    Dt = Dx - np.sum(Dx * xij, axis=0) / np.where(n2 > 0, n2, 1.0) * xij
    lt = np.linalg.norm(Dt, axis=0)
    static_f = _forced(lt < 2.0 * r * prm.mu_s, force_static)
    scale = np.where(static_f, 1.0, np.minimum(2.0 * r * prm.mu_k / np.where(lt > 0, lt, 1.0), 1.0))
    f = Dt * scale
    di = di - mi * f
    dj = dj + mj * f
    di[:, ~act] = 0.0
    dj[:, ~act] = 0.0
    rigid = body >= 0
    frames = {}
    sm, sm_cnt = None, None
    if rigid.any():
        sm, frames = shape_matching(xt, body, np.asarray(rest, dtype=F64), return_frames=True)
        sm_cnt = rigid.astype(F64)
    upd = _average(xt.shape[1], pairs, di, dj, act, sm, sm_cnt)
    info = {"act": act, "act_margin": margin, "fric_margin": lt - 2.0 * r * prm.mu_s, "frames": frames}
    return xt + upd, info


def finish(x, xt, body, dt):
    """Step 4: v = (x~ - x) / dt, x = x~; static particles keep x, v = 0."""
    x = np.asarray(x, dtype=F64)
    xt = np.asarray(xt, dtype=F64)
    dyn = np.asarray(body) != STATIC
    return np.where(dyn, xt, x), np.where(dyn, (xt - x) / F64(dt), 0.0)


def step(x, v, body, inv_m, rest, prm: PBDParams, return_info: bool = False):
    """One LR step (Algorithm 1).  x, v: [3, N]; body: int [N] (GRANULAR = -1,
    STATIC = -2, rigid body ids >= 0); inv_m: [N] (0 for static); rest: [3, N]
    rest offsets of rigid particles from their body's centre (ignored
    otherwise).  Returns float64 (x, v) after the step."""
    x = np.asarray(x, dtype=F64)
    body = np.asarray(body)
    r = F64(prm.r)
    info = {"stab_pairs": 0, "solve_pairs": 0, "min_margin": np.inf}
    # 1. prediction and scaled masses
    v, xt, w = predict(x, v, body, inv_m, prm)
    # 2. stabilization on the start positions, applied to x and x~
    sp = contact_pairs(x, body, r)
    info["stab_pairs"] = sp.shape[0]
    for _ in range(prm.stab_iters):
        x, xt, _ = stab_iteration(x, xt, sp, w, r)
    x0 = x.copy()
    # 3. solver iterations on x~: contact + friction per pair, shape matching
    pairs = contact_pairs(xt, body, r)
    info["solve_pairs"] = pairs.shape[0]
    for _ in range(prm.solve_iters):
        xt_new, it = solve_iteration(xt, x0, pairs, w, body, rest, prm)
        act = it["act"]
        if act.any():
            info["min_margin"] = min(info["min_margin"], float(np.min(np.abs(it["act_margin"][act]))),
                                     float(np.min(np.abs(it["fric_margin"][act]))))
        xt = xt_new
    # 4. velocities from the positions
    xn, vn = finish(x, xt, body, prm.dt)
    if return_info:
        return xn, vn, info
    return xn, vn
