"""Plain CPU oracle for the high-resolution (HR) upsampling step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP library
never calls it, and this module shares no code with the HIP path: it is
written from the paper (Section 4, "HR Upsampling") and from the boundary's
contract for the integer stages, in float64 NumPy, deliberately slow and plain.

What it computes, per HR particle i given the LR guide particles j (Section 4):

* weight   w_ij = max(0, (1 - |x_ij|^2 / (9 r_LR^2))^3)                 (support h = 3 r_LR)
* Shepard  v~_i = sum_j w_ij v_j / sum_j w_ij
* blend    alpha_i = 1 - max_j w_ij  if max w <= c1 or max w / sum w >= c2, else 0
           with c1 = 512/729 (the weight at distance r_LR) and c2 = 0.6
* velocity v_i^{t+1} = (1 - alpha_i) v~_i^{t+1} + alpha_i (v_i^t + dt_HR g)
* position x_i^{t+1} = x_i^t + dt_HR v_i^{t+1}            (symplectic Euler)
* LR particles of rigid bodies / boundaries take part only when at least one
  granular LR particle is in the vicinity (end of Section 4).

Readings where the paper is silent (each listed in the design notes):

* empty neighbourhood: v~ = 0, so max w = 0 <= c1 and alpha = 1 (pure free fall);
* "vicinity" of the rigid rule = the kernel support;
* membership is decided by the float32 predicate ``fl32(|X_j - x_i|^2) < fl32(9 r^2)``
  with each float32 operation rounded separately (the integer contract shared with
  the GPU); the weights themselves are float64;
* the domain walls (the paper gives none for HR particles) are the boundary's
  planar-wall contract, applied in order after integration;
* the adjoint (not in the paper) differentiates the step with the alpha branch,
  neighbour membership, the argmax of the weights and the wall activations held
  fixed; argmax ties go to the smallest LR index.

Arrays are structure-of-arrays ``[3, N]``; float32 inputs are widened exactly to
float64 before any floating-point work except the integer-contract stages.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass
from typing import Dict, Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree

F32 = np.float32
F64 = np.float64

C1 = 512.0 / 729.0   # weight at |x_ij| = r_LR (Section 4)
C2 = 0.6             # empirically chosen ratio threshold (Section 4)

DEFAULT_CELL_FACTOR = 1.0001
BAND = 1e-5          # alpha-branch band: either branch is accepted inside it
WALL_BAND = 4e-6     # wall-decision band (metres)
WORKERS = min(16, os.cpu_count() or 1)   # KD-tree query threads (numpy work is single-threaded)


# ---------------------------------------------------------------------------
# Kernel weight (Section 4).
# ---------------------------------------------------------------------------

def weight(s: np.ndarray, r_lr: float) -> np.ndarray:
    """w = max(0, (1 - s / (9 r^2))^3) for squared distance s (float64)."""
    s = np.asarray(s, dtype=F64)
    return np.maximum(0.0, (1.0 - s / (9.0 * F64(r_lr) ** 2)) ** 3)


# ---------------------------------------------------------------------------
# Grid contract (integer stages).  The neighbour search of the paper is a
# compact-hashing uniform grid with cell size tied to the search radius
# (Section 5.1); the boundary fixes its float32 arithmetic so that the keys,
# the stable sorted order and the per-cell ranges are reproducible bit for bit.
# ---------------------------------------------------------------------------

@dataclass
class GridSpec:
    h: float              # support radius 3 r (float64)
    cs: float             # cell size (float64)
    inv_cs: np.float32    # fl32(1 / cs)
    lo: np.ndarray        # float32[3]
    dims: Tuple[int, int, int]
    reach: int            # stencil half-width in cells
    h2_f: np.float32      # fl32(9 r^2)

    @property
    def n_cells(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]


def grid_spec(r_lr: float, domain_lo, domain_hi, cell_factor: float = 0.0) -> GridSpec:
    r = F64(F32(r_lr))
    kappa = F64(F32(cell_factor if cell_factor > 0 else DEFAULT_CELL_FACTOR))
    h = 3.0 * r
    cs = kappa * h
    lo = np.asarray(domain_lo, dtype=F32)
    hi = np.asarray(domain_hi, dtype=F32)
    dims = tuple(max(1, int(math.ceil((F64(hi[a]) - F64(lo[a])) / cs))) for a in range(3))
    gmax = max(dims)
    reach = int(math.ceil(h / cs + 16.0 * gmax * 2.0 ** -24))
    return GridSpec(h=h, cs=cs, inv_cs=F32(1.0 / cs), lo=lo, dims=dims, reach=reach,
                    h2_f=F32(9.0 * r * r))


def cell_coords(X: np.ndarray, spec: GridSpec) -> np.ndarray:
    """Integer cell coordinates [3, N]: clamp(floor(fl32(fl32(X - lo) * inv_cs)), 0, G-1)."""
    X = np.asarray(X, dtype=F32)
    out = np.empty(X.shape, dtype=np.int64)
    for a in range(3):
        t = (X[a] - spec.lo[a]) * spec.inv_cs           # two separately rounded float32 ops
        f = np.floor(t.astype(F64))
        out[a] = np.clip(f, 0, spec.dims[a] - 1).astype(np.int64)
    return out


def cell_keys(X: np.ndarray, spec: GridSpec) -> np.ndarray:
    c = cell_coords(X, spec)
    gx, gy, _ = spec.dims
    return (c[0] + gx * (c[1] + gy * c[2])).astype(np.uint32)


def sort_by_cell(keys: np.ndarray, n_cells: int) -> Tuple[np.ndarray, np.ndarray]:
    """Stable counting sort: order by (key, original index); cell_start[G + 1]."""
    perm = np.argsort(keys, kind="stable").astype(np.uint32)
    counts = np.bincount(keys.astype(np.int64), minlength=n_cells)
    cell_start = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    return perm, cell_start


# ---------------------------------------------------------------------------
# Neighbour sets under the float32 membership predicate.
# ---------------------------------------------------------------------------

def sq_dist_f32(Xj: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz)), d = fl32(X_j - x_i).

    Xj, xi broadcastable float32 arrays of shape [3, ...]."""
    d = np.asarray(Xj, dtype=F32) - np.asarray(xi, dtype=F32)
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]


def _csr(lists) -> Tuple[np.ndarray, np.ndarray]:
    indptr = np.zeros(len(lists) + 1, dtype=np.int64)
    indptr[1:] = np.cumsum([len(l) for l in lists])
    idx = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists]) if lists else np.zeros(0, np.int64)
    return indptr, idx


def neighbours_bruteforce(lr_x: np.ndarray, hr_x: np.ndarray, h2_f) -> Tuple[np.ndarray, np.ndarray]:
    """All pairs: for each HR i the ascending LR ids j with s_f < h2_f (tiny inputs)."""
    lr_x = np.asarray(lr_x, dtype=F32)
    hr_x = np.asarray(hr_x, dtype=F32)
    lists = []
    for i in range(hr_x.shape[1]):
        s = sq_dist_f32(lr_x, hr_x[:, i:i + 1])
        lists.append(np.nonzero(s < F32(h2_f))[0])
    return _csr(lists)


def neighbours_kdtree(lr_x: np.ndarray, hr_x: np.ndarray, h: float, h2_f,
                      predicate: str = "f32") -> Tuple[np.ndarray, np.ndarray]:
    """KD-tree candidates within h (1 + 1e-5), filtered by the membership predicate.
    ``predicate="f64"`` uses the exact float64 test s < 9 r^2 = h^2 instead."""
    lr_x = np.asarray(lr_x, dtype=F32)
    hr_x = np.asarray(hr_x, dtype=F32)
    n_hr = hr_x.shape[1]
    if lr_x.shape[1] == 0 or n_hr == 0:
        return np.zeros(n_hr + 1, np.int64), np.zeros(0, np.int64)
    tree = cKDTree(lr_x.T.astype(F64))
    cand = tree.query_ball_point(hr_x.T.astype(F64), r=h * (1.0 + 1e-5), workers=WORKERS)
    counts = np.fromiter((len(c) for c in cand), dtype=np.int64, count=n_hr)
    ii = np.repeat(np.arange(n_hr), counts)
    jj = np.concatenate([np.asarray(c, dtype=np.int64) for c in cand]) if counts.sum() else np.zeros(0, np.int64)
    if predicate == "f32":
        keep = sq_dist_f32(lr_x[:, jj], hr_x[:, ii]) < F32(h2_f)
    else:
        d = lr_x[:, jj].astype(F64) - hr_x[:, ii].astype(F64)
        keep = np.sum(d * d, axis=0) < h * h
    ii, jj = ii[keep], jj[keep]
    order = np.lexsort((jj, ii))
    ii, jj = ii[order], jj[order]
    indptr = np.zeros(n_hr + 1, dtype=np.int64)
    indptr[1:] = np.cumsum(np.bincount(ii, minlength=n_hr))
    return indptr, jj


def neighbours_grid(lr_x: np.ndarray, hr_x: np.ndarray, spec: GridSpec) -> Tuple[np.ndarray, np.ndarray]:
    """The same sets through the uniform grid: the (2R+1)^3 cell stencil around each
    HR cell, candidates filtered by the float32 predicate.  Plain loops (small N)."""
    lr_x = np.asarray(lr_x, dtype=F32)
    hr_x = np.asarray(hr_x, dtype=F32)
    keys = cell_keys(lr_x, spec)
    perm, cell_start = sort_by_cell(keys, spec.n_cells)
    hc = cell_coords(hr_x, spec)
    gx, gy, gz = spec.dims
    R = spec.reach
    lists = []
    for i in range(hr_x.shape[1]):
        found = []
        for cz in range(max(hc[2, i] - R, 0), min(hc[2, i] + R, gz - 1) + 1):
            for cy in range(max(hc[1, i] - R, 0), min(hc[1, i] + R, gy - 1) + 1):
                for cx in range(max(hc[0, i] - R, 0), min(hc[0, i] + R, gx - 1) + 1):
                    k = cx + gx * (cy + gy * cz)
                    for p in range(cell_start[k], cell_start[k + 1]):
                        j = int(perm[p])
                        if sq_dist_f32(lr_x[:, j], hr_x[:, i]) < spec.h2_f:
                            found.append(j)
        lists.append(sorted(found))
    return _csr(lists)


# ---------------------------------------------------------------------------
# Planar walls (the boundary's contract; the paper has no HR boundary step).
# A wall row is n(3), d, a(3), b, o(3), R.
# ---------------------------------------------------------------------------

def apply_walls(x_old: np.ndarray, x: np.ndarray, v: np.ndarray, walls: np.ndarray, r_hr: float,
                flip: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """In place on float64 (N, 3) x and v.  For each wall in order: the wall acts on
    particle i when a.x >= b, the in-plane distance from o is >= R (or R = 0) and the
    pre-step position satisfied n.x_old - d >= 0.  An acting wall with n.x - d < r_HR
    pushes x to n.x - d = r_HR and removes an inward normal velocity.

    ``flip`` (N, n_walls) bool inverts the push decision (used to enumerate the
    alternative result for particles inside the decision band).  Returns the per
    wall push / clip masks and the band mask."""
    n_w = walls.shape[0]
    N = x.shape[0]
    pushed = np.zeros((N, n_w), dtype=bool)
    clipped = np.zeros((N, n_w), dtype=bool)
    band = np.zeros((N, n_w), dtype=bool)
    for k in range(n_w):
        row = walls[k].astype(F64)
        n, d, a, b, o, R = row[0:3], row[3], row[4:7], row[7], row[8:11], row[11]
        ax = x @ a
        act = ax >= b
        act_band = np.abs(ax - b) <= WALL_BAND
        if R > 0.0:
            rel = x - o
            inpl = rel - np.outer(rel @ n, n)
            dist = np.sqrt(np.sum(inpl * inpl, axis=1))
            act &= dist >= R
            act_band |= np.abs(dist - R) <= WALL_BAND
        side = x_old @ n - d
        act &= side >= 0.0
        act_band |= np.abs(side) <= WALL_BAND
        pen = x @ n - d
        hit = act & (pen < r_hr)
        # a decision inside the float32 rounding band of its threshold may go either way
        band[:, k] = ((pen < r_hr + WALL_BAND) & act_band) | (act & (np.abs(pen - r_hr) <= WALL_BAND))
        if flip is not None:
            hit ^= flip[:, k]
        x[hit] += np.outer(r_hr - pen[hit], n)
        vn = v @ n
        clip = hit & (vn < 0.0)
        v[clip] -= np.outer(vn[clip], n)
        pushed[:, k] = hit
        clipped[:, k] = clip
    return {"pushed": pushed, "clipped": clipped, "band": band}


# ---------------------------------------------------------------------------
# Forward step (Section 4).
# ---------------------------------------------------------------------------

def _pairs(indptr: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(indptr.shape[0] - 1), np.diff(indptr))


def step(lr_x, lr_v, lr_rigid, hr_x, hr_v, prm: dict, nbrs=None, force_A=None,
         wall_flip=None, predicate: str = "f32", keep: bool = False) -> Dict[str, np.ndarray]:
    """One upsampling step.  ``lr_*`` is the LR frame the HR particles are advanced
    against (positions, velocities, rigid flags); ``hr_x``/``hr_v`` the HR state at t.

    ``prm``: r_lr, r_hr, dt, g(3), c1, c2, walls (n, 12).
    ``force_A`` optional bool [N_H] replacing the alpha condition (band alternatives).
    Returns float64 ``x``, ``v`` [3, N_H] and per-HR diagnostics."""
    r = F64(F32(prm["r_lr"]))
    h = 3.0 * r
    h2 = 9.0 * r * r
    h2_f = F32(9.0 * r * r)
    c1 = F64(prm.get("c1", C1))
    c2 = F64(prm.get("c2", C2))
    dt = F64(prm["dt"])
    g = np.asarray(prm["g"], dtype=F64)
    X = np.asarray(lr_x, dtype=F64).T
    V = np.asarray(lr_v, dtype=F64).T
    x = np.asarray(hr_x, dtype=F64).T.copy()
    v = np.asarray(hr_v, dtype=F64).T.copy()
    N = x.shape[0]
    rigid = np.zeros(X.shape[0], dtype=bool) if lr_rigid is None else np.asarray(lr_rigid).astype(bool)

    if nbrs is None:
        nbrs = neighbours_kdtree(lr_x, hr_x, h, h2_f, predicate=predicate)
    indptr, jj = nbrs
    ii = _pairs(indptr)

    # rigid LR count only where a granular LR is in the vicinity (Section 4, last paragraph)
    n_gran = np.bincount(ii, weights=(~rigid[jj]).astype(F64), minlength=N)
    keep_pair = n_gran[ii] > 0
    ii, jj = ii[keep_pair], jj[keep_pair]

    d = X[jj] - x[ii]
    s = np.sum(d * d, axis=1)
    w = weight(s, r)

    S = np.bincount(ii, weights=w, minlength=N)
    U = np.stack([np.bincount(ii, weights=w * V[jj, a], minlength=N) for a in range(3)], axis=1)
    M = np.zeros(N)
    np.maximum.at(M, ii, w)

    has = S > 0.0
    vt = np.zeros((N, 3))
    vt[has] = U[has] / S[has, None]
    ratio = np.zeros(N)
    ratio[has] = M[has] / S[has]
    A = (M <= c1) | (has & (ratio >= c2))
    band = (np.abs(M - c1) <= BAND) | (has & (np.abs(ratio - c2) <= BAND))
    if force_A is not None:
        A = np.asarray(force_A, dtype=bool)
    alpha = np.where(A, 1.0 - M, 0.0)

    vf = v + dt * g
    v_new = (1.0 - alpha)[:, None] * vt + alpha[:, None] * vf
    x_new = x + dt * v_new
    walls = np.asarray(prm.get("walls", np.zeros((0, 12))), dtype=F32)
    wrec = apply_walls(x, x_new, v_new, walls, F64(prm["r_hr"]), flip=wall_flip)

    out = {"x": x_new.T, "v": v_new.T, "S": S, "M": M, "alpha": alpha, "A": A,
           "band": band, "wall_band": wrec["band"], "count": np.diff(indptr)}
    if keep:
        out.update(ii=ii, jj=jj, s=s, w=w, U=U, vt=vt, vf=vf, wall=wrec)
    return out


# ---------------------------------------------------------------------------
# Adjoint of one step (a reading: the paper does not differentiate).
# ---------------------------------------------------------------------------

def step_backward(lr_x, lr_v, lr_rigid, hr_x, hr_v, prm: dict, gx_out, gv_out,
                  predicate: str = "f32", nbrs=None) -> Dict[str, np.ndarray]:
    """Vector-Jacobian product of :func:`step` with the alpha branch, membership,
    argmax and wall activations held at their forward values.

    gx_out, gv_out: dL/dx^{t+1}, dL/dv^{t+1} [3, N_H].
    Returns gx, gv (dL/dx^t, dL/dv^t) and g_lr_x, g_lr_v (dL/dX, dL/dV) [3, N]."""
    fw = step(lr_x, lr_v, lr_rigid, hr_x, hr_v, prm, nbrs=nbrs, predicate=predicate, keep=True)
    r = F64(F32(prm["r_lr"]))
    h2 = 9.0 * r * r
    dt = F64(prm["dt"])
    X = np.asarray(lr_x, dtype=F64).T
    V = np.asarray(lr_v, dtype=F64).T
    x = np.asarray(hr_x, dtype=F64).T
    N, NL = x.shape[0], X.shape[0]
    walls = np.asarray(prm.get("walls", np.zeros((0, 12))), dtype=F64)

    gx = np.asarray(gx_out, dtype=F64).T.copy()
    gv = np.asarray(gv_out, dtype=F64).T.copy()
    # walls, last first: a push maps x -> x + (r_HR - (n.x - d)) n, Jacobian I - n n^T;
    # a velocity clip maps v -> v - (n.v) n, Jacobian I - n n^T.
    for k in range(walls.shape[0] - 1, -1, -1):
        n = walls[k, 0:3]
        p = fw["wall"]["pushed"][:, k]
        c = fw["wall"]["clipped"][:, k]
        gx[p] -= np.outer(gx[p] @ n, n)
        gv[c] -= np.outer(gv[c] @ n, n)

    # x' = x + dt v'  ->  dL/dv' gains dt dL/dx'
    gvp = gv + dt * gx
    alpha = fw["alpha"]
    g_x = gx.copy()
    g_v = alpha[:, None] * gvp
    g_alpha = np.sum(gvp * (fw["vf"] - fw["vt"]), axis=1)
    g_vt = (1.0 - alpha)[:, None] * gvp
    g_M = np.where(fw["A"], -g_alpha, 0.0)
    S = fw["S"]
    has = S > 0.0
    g_U = np.zeros((N, 3))
    g_S = np.zeros(N)
    g_U[has] = g_vt[has] / S[has, None]
    g_S[has] = -np.sum(g_vt[has] * fw["vt"][has], axis=1) / S[has]

    ii, jj, s, w = fw["ii"], fw["jj"], fw["s"], fw["w"]
    # argmax of w per HR, ties to the smallest LR index
    arg = np.full(N, -1, dtype=np.int64)
    if ii.size:
        order = np.lexsort((jj, -w, ii))
        first = np.ones(order.size, dtype=bool)
        first[1:] = ii[order][1:] != ii[order][:-1]
        arg[ii[order][first]] = jj[order][first]
    is_arg = jj == arg[ii]

    g_w = np.sum(g_U[ii] * V[jj], axis=1) + g_S[ii] + np.where(is_arg, g_M[ii], 0.0)
    g_lr_v = np.zeros((NL, 3))
    for a in range(3):
        g_lr_v[:, a] = np.bincount(jj, weights=w * g_U[ii, a], minlength=NL)
    t = np.maximum(0.0, 1.0 - s / h2)
    g_s = g_w * (-3.0 / h2) * t * t
    d = X[jj] - x[ii]
    g_lr_x = np.zeros((NL, 3))
    for a in range(3):
        g_lr_x[:, a] = np.bincount(jj, weights=2.0 * g_s * d[:, a], minlength=NL)
        g_x[:, a] -= np.bincount(ii, weights=2.0 * g_s * d[:, a], minlength=N)
    return {"gx": g_x.T, "gv": g_v.T, "g_lr_x": g_lr_x.T, "g_lr_v": g_lr_v.T, "fw": fw}


# ---------------------------------------------------------------------------
# Rollouts.
# ---------------------------------------------------------------------------

def rollout(frames, lr_rigid, x0, v0, prm: dict, predicate: str = "f32"):
    """Advance (x0, v0) through LR frames [(X, V), ...]; returns the list of states
    [(x^0, v^0), (x^1, v^1), ...] in float64 and the per-step band masks."""
    states = [(np.asarray(x0, dtype=F64), np.asarray(v0, dtype=F64))]
    bands = []
    for (X, V) in frames:
        x, v = states[-1]
        o = step(X, V, lr_rigid, x, v, prm, predicate=predicate)
        states.append((o["x"], o["v"]))
        bands.append(o["band"] | np.any(o["wall_band"], axis=1))
    return states, bands


def rollout_loss_grad(frames, lr_rigid, x0, v0, prm: dict, target, predicate: str = "f32"):
    """Loss L = mean_i |x_i^T - y_i|^2 over the rollout and its gradients with respect
    to every frame's LR positions and velocities (lists, [3, N_L] each)."""
    states, _ = rollout(frames, lr_rigid, x0, v0, prm, predicate=predicate)
    xT = states[-1][0]
    y = np.asarray(target, dtype=F64)
    N = xT.shape[1]
    diff = xT - y
    loss = float(np.sum(diff * diff) / N)
    gx = 2.0 * diff / N
    gv = np.zeros_like(gx)
    g_X, g_V = [None] * len(frames), [None] * len(frames)
    for t in range(len(frames) - 1, -1, -1):
        X, V = frames[t]
        x, v = states[t]
        b = step_backward(X, V, lr_rigid, x, v, prm, gx, gv, predicate=predicate)
        gx, gv = b["gx"], b["gv"]
        g_X[t], g_V[t] = b["g_lr_x"], b["g_lr_v"]
    return loss, g_X, g_V, gx, gv
