"""Helpers shared by the GPU parity tests: device upload of seeded scenes and the
element-wise comparison of a GPU step against the oracle, with the tolerance
and the two-results-allowed bands written out here."""
from __future__ import annotations

import sys

import numpy as np

from oracle import upsample_oracle as O

# Tolerances per step: |dx| <= 1e-6 box lengths, |dv| <= 1e-5 max(|v_ref|, 1 m/s).
TOL_X = 1e-6
TOL_V = 1e-5


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _close(gx, gv, ox, ov, L, n_steps):
    ex = np.abs(gx - ox).max(axis=0)
    ev = (np.abs(gv - ov) / np.maximum(np.abs(ov), 1.0)).max(axis=0)
    return (ex <= TOL_X * L * n_steps) & (ev <= TOL_V * n_steps), ex, ev


def compare_step(gx, gv, lr_x, lr_v, rigid, hr_x, hr_v, prm, L, n_steps=1, idx=None, oracle_out=None,
                 max_band_frac=1e-3):
    """Compare GPU outputs gx, gv ([3, N] float32) with the oracle's step of
    (hr_x, hr_v) at columns ``idx`` (all if None).  Particles inside an alpha or
    wall decision band may match the other branch instead.  Returns a summary."""
    if idx is None:
        idx = np.arange(hr_x.shape[1])
    o = oracle_out if oracle_out is not None else O.step(lr_x, lr_v, rigid, hr_x[:, idx], hr_v[:, idx], prm)
    ok, ex, ev = _close(gx[:, idx], gv[:, idx], o["x"], o["v"], L, n_steps)
    bad = np.nonzero(~ok)[0]
    band_hits = 0
    if bad.size:
        sub = idx[bad]
        alpha_band = o["band"][bad]
        wall_band = o["wall_band"][bad]
        # alternative 1: the other alpha branch
        fA = o["A"].copy()[bad] ^ alpha_band
        o1 = O.step(lr_x, lr_v, rigid, hr_x[:, sub], hr_v[:, sub], prm, force_A=fA)
        ok1, _, _ = _close(gx[:, sub], gv[:, sub], o1["x"], o1["v"], L, n_steps)
        # alternative 2: the other wall decision for walls inside their band
        o2 = O.step(lr_x, lr_v, rigid, hr_x[:, sub], hr_v[:, sub], prm, wall_flip=wall_band)
        ok2, _, _ = _close(gx[:, sub], gv[:, sub], o2["x"], o2["v"], L, n_steps)
        in_band = alpha_band | wall_band.any(axis=1)
        rescued = in_band & (ok1 | ok2)
        band_hits = int(rescued.sum())
        still = bad[~rescued]
        if still.size:
            j = still[0]
            i = idx[j]
            raise AssertionError(
                f"{still.size} of {idx.size} HR outside tolerance; first: hr={i} x_gpu={gx[:, i]} "
                f"x_ref={o['x'][:, j]} v_gpu={gv[:, i]} v_ref={o['v'][:, j]} |dx|={ex[j]:.3e} "
                f"rel|dv|={ev[j]:.3e} alpha={o['alpha'][j]} M={o['M'][j]} S={o['S'][j]} "
                f"band={o['band'][j]} wall_band={o['wall_band'][j].any()}")
    assert band_hits <= max(2, max_band_frac * idx.size), band_hits
    return {"n": int(idx.size), "max_dx": float(ex.max(initial=0)), "max_rel_dv": float(ev.max(initial=0)),
            "band": band_hits, "alpha_band": int(o["band"].sum())}


def hilbert_index(f, bits):
    """Index along a 3-D Hilbert curve of integer cells f [3, N] in a cube of
    2^bits cells per axis (Skilling 2004, transpose form), axis 0 the most
    significant bit of each triple.  Pinned by tests/test_abi.py: a bijection
    onto [0, 8^bits) whose consecutive indices are face neighbours."""
    X = [np.asarray(f[a], dtype=np.int64).copy() for a in range(3)]
    q = 1 << (bits - 1)
    while q > 1:
        p = q - 1
        for i in range(3):
            hit = (X[i] & q) != 0
            t = (X[0] ^ X[i]) & p
            x0 = np.where(hit, X[0] ^ p, X[0] ^ t)
            if i:
                X[i] = np.where(hit, X[i], X[i] ^ t)
            X[0] = x0
        q >>= 1
    X[1] ^= X[0]
    X[2] ^= X[1]
    t = np.zeros_like(X[0])
    q = 1 << (bits - 1)
    while q > 1:
        t = np.where((X[2] & q) != 0, t ^ (q - 1), t)
        q >>= 1
    key = np.zeros_like(X[0])
    for b in range(bits - 1, -1, -1):
        for i in range(3):
            key = (key << 1) | (((X[i] ^ t) >> b) & 1)
    return key


def morton_sort_keys(x, spec, sub, mode=1):
    """The HR reorder key of positions x [3, N] for a grid spec (float32
    arithmetic): mode 1 the Z-order code of fine cells, mode 0 the grid cell
    then the Z-order of its sub-cells, mode 2 the Hilbert index of fine cells.
    Used to check the reorder's output."""
    x = np.asarray(x, dtype=np.float32)
    bits, fine = [], []
    for a in range(3):
        t = (x[a] - spec.lo[a]) * spec.inv_cs
        c = np.clip(np.floor(t), 0, spec.dims[a] - 1).astype(np.float32)
        f = np.clip(np.floor((t - c) * np.float32(sub)), 0, sub - 1)
        fine.append(c.astype(np.int64) * sub + f.astype(np.int64))
        bits.append(int(np.ceil(np.log2(spec.dims[a] * sub))) if spec.dims[a] * sub > 1 else 0)
    if mode == 2:
        return hilbert_index(fine, max(bits))
    if mode == 0:
        c = [f // sub for f in fine]
        sb = [f % sub for f in fine]
        cell = c[0] + spec.dims[0] * (c[1] + spec.dims[1] * c[2])
        m = np.zeros_like(cell)
        for b in range(2):
            for a in range(3):
                m |= ((sb[a] >> b) & 1) << (3 * b + a)
        return cell * sub ** 3 + m
    key = np.zeros(x.shape[1], dtype=np.int64)
    pos = 0
    for b in range(max(bits)):
        for a in range(3):
            if b < bits[a]:
                key |= ((fine[a] >> b) & 1) << pos
                pos += 1
    return key


# Two GPU runs that group particles into waves differently (another HR order,
# another per-wave path) may round differently: the weights of a compact wave
# are computed relative to its box centre.  They agree far inside the oracle
# tolerance.
SAME_X = 2e-7
SAME_V = 3e-6


def assert_same_step(x_a, v_a, x_b, v_b, L):
    """x, v: torch tensors [3, N] of two GPU results of the same step."""
    import torch
    dx = (x_a - x_b).abs().max().item()
    dv = ((v_a - v_b).abs() / torch.clamp(v_b.abs(), min=1.0)).max().item()
    assert dx <= SAME_X * L and dv <= SAME_V, (dx, dv)


def _decisions(o):
    """The discrete decisions of an oracle step: alpha branch and wall pushes."""
    return np.concatenate([o["A"][:, None], o["wall"]["pushed"]], axis=1)


def band_along(frames, states, idx, prm, rigid=None, drift=None):
    """Whether each particle idx met a decision threshold at some step of a
    trajectory: states[t] = (x, v) [3, N] before frame t.  At step t a
    particle counts when the oracle's step puts its alpha or wall decision
    inside the band of either branch, or -- with ``drift`` (a function of t
    giving a distance in metres) -- when moving its position by drift(t)
    along any axis changes one of its decisions.  Two float32 runs that
    group particles into other waves drift apart by rounding, by at most
    their comparison tolerance so far; a particle whose decision is that
    sensitive may take the other branch in one of them and from then on
    follow another valid trajectory."""
    hit = np.zeros(len(idx), bool)
    for t, ((X, V), (x, v)) in enumerate(zip(frames, states)):
        xs, vs = np.asarray(x)[:, idx].astype(np.float64), np.asarray(v)[:, idx].astype(np.float64)
        o = O.step(X, V, rigid, xs, vs, prm, keep=True)
        hit |= o["band"] | o["wall_band"].any(axis=1)
        if drift is not None:
            base = _decisions(o)
            d = float(drift(t))
            for a in range(3):
                for sgn in (-1.0, 1.0):
                    xp = xs.copy()
                    xp[a] += sgn * d
                    hit |= (_decisions(O.step(X, V, rigid, xp, vs, prm, keep=True)) != base).any(axis=1)
    return hit


# Weight of a list entry on which the kernel's test (computed weight > 0) and
# the exact membership predicate disagree: such an entry sits where
# 1 - s / h^2 is within the rounding of the kernel's weight argument, at most
# 16 float32 units of its largest term (about 1e-6), so its weight is below
# (1e-6)^3 = 1e-18; ten times that is allowed.
W_DISAGREE_MAX = 1e-17
