"""Plain CPU oracle for the randomized volume sampling of initial particle
states (Section 4, the sampling paragraph before the upsampling formulas).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and is written from the paper's description:

1. The bounding box of the hull is divided into cubic cells of side
   2 r / sqrt(3) (r the radius of the particles being sampled, LR or HR), so
   a cell's diagonal is 2 r: two non-overlapping particles never share a cell.
2. Many random candidate positions, uniform inside the hull, are assigned to
   the cells they fall in.
3. For each cell an attempt is made to select one of its candidates that does
   not overlap an already sampled position (distance at least 2 r).

Readings (listed with the others in the design notes):

* The candidates are an input (their random numbers are drawn by the caller,
  inside the hull, which is an analytic shape here: the paper's meshes are
  not available); a cell tries its candidates in input order and takes the
  first that fits.
* The paper leaves the order of the cells open.  Here the cells are visited
  in 27 colour phases, colour (cx mod 3) + 3 (cy mod 3) + 9 (cz mod 3), and
  within a phase in cell-key order.  Two cells of one colour differ by at
  least 3 in some axis, so their points are at least 2 side lengths = 2.31 r
  apart and can never conflict: within a phase every cell can choose at once
  and the result is still that of this sequential order.
* Overlap is decided in float32, like the neighbour predicate of the step:
  a candidate p fits if fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz)) >= fl32(4 r^2)
  for every sample q, d = fl(p - q); cell coordinates are
  clamp(floor(fl(fl(p - lo) * fl32(1 / side))), 0, G - 1) with
  G = ceil((hi - lo) / side) per axis and side = 2 r / sqrt(3) in float64.
  A conflict can only come from the 5 x 5 x 5 cells around a cell (2 r is
  1.73 side lengths).
* The samples are returned in cell-key order.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

F32 = np.float32
F64 = np.float64


def sampling_grid(r: float, lo, hi):
    """Side (float64), fl32(1/side), lo (float32) and dims of the sampling cells."""
    side = 2.0 * F64(F32(r)) / math.sqrt(3.0)
    lo32 = np.asarray(lo, dtype=F32)
    hi32 = np.asarray(hi, dtype=F32)
    dims = tuple(max(1, int(math.ceil((F64(hi32[a]) - F64(lo32[a])) / side))) for a in range(3))
    return side, F32(1.0 / side), lo32, dims


def cells_of(P, inv_side, lo32, dims) -> np.ndarray:
    """Integer cell coordinates [3, N] of float32 positions [3, N]."""
    P = np.asarray(P, dtype=F32)
    c = np.empty(P.shape, dtype=np.int64)
    for a in range(3):
        t = (P[a] - lo32[a]) * inv_side
        c[a] = np.clip(np.floor(t.astype(F64)), 0, dims[a] - 1).astype(np.int64)
    return c


def _fits(p, q, d2) -> bool:
    """Non-overlap test of positions p, q (float32 [3]) in the float32 contract."""
    d = p.astype(F32) - q.astype(F32)
    s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    return bool(s >= d2)


def sample_volume_sequential(cand, r: float, lo, hi) -> np.ndarray:
    """The reading above as one sequential pass over the cells in (colour,
    key) order, a plain dictionary of the samples taken so far.  Small inputs
    only.  cand: float32 [3, M] -> samples float32 [3, K] in key order."""
    side, inv_side, lo32, dims = sampling_grid(r, lo, hi)
    cand = np.asarray(cand, dtype=F32)
    d2 = F32(4.0 * F64(F32(r)) ** 2)
    c = cells_of(cand, inv_side, lo32, dims)
    key = c[0] + dims[0] * (c[1] + dims[1] * c[2])
    colour = (c[0] % 3) + 3 * (c[1] % 3) + 9 * (c[2] % 3)
    by_cell = {}
    for i in range(cand.shape[1]):                      # input order within a cell
        by_cell.setdefault(int(key[i]), []).append(i)
    cells = sorted(by_cell, key=lambda k: (int(colour[by_cell[k][0]]), k))
    taken = {}                                           # cell key -> sample index
    for k in cells:
        cz, rem = divmod(k, dims[0] * dims[1])
        cy, cx = divmod(rem, dims[0])
        for i in by_cell[k]:
            ok = True
            for dz in range(-2, 3):
                for dy in range(-2, 3):
                    for dx in range(-2, 3):
                        x, y, z = cx + dx, cy + dy, cz + dz
                        if not (0 <= x < dims[0] and 0 <= y < dims[1] and 0 <= z < dims[2]):
                            continue
                        j = taken.get(x + dims[0] * (y + dims[1] * z))
                        if j is not None and not _fits(cand[:, i], cand[:, j], d2):
                            ok = False
            if ok:
                taken[k] = i
                break
    order = sorted(taken)
    return cand[:, [taken[k] for k in order]] if order else np.zeros((3, 0), F32)


def sample_volume(cand, r: float, lo, hi) -> Tuple[np.ndarray, np.ndarray]:
    """The same result, one colour phase at a time: in a phase every cell of
    the colour takes its first candidate that fits the samples of the earlier
    phases (numpy over the cells of the phase, one candidate rank after the
    other).  Returns the samples float32 [3, K] in key order and the index of
    each sample in ``cand``."""
    side, inv_side, lo32, dims = sampling_grid(r, lo, hi)
    cand = np.asarray(cand, dtype=F32)
    M = cand.shape[1]
    d2 = F32(4.0 * F64(F32(r)) ** 2)
    c = cells_of(cand, inv_side, lo32, dims)
    key = c[0] + dims[0] * (c[1] + dims[1] * c[2])
    order = np.argsort(key, kind="stable")               # by cell, input order inside
    skey = key[order]
    first = np.ones(M, dtype=bool)
    first[1:] = skey[1:] != skey[:-1]
    rank = np.arange(M) - np.maximum.accumulate(np.where(first, np.arange(M), 0))
    n_cells = dims[0] * dims[1] * dims[2]
    taken = np.full(n_cells, -1, dtype=np.int64)         # cell key -> candidate index
    sc = c[:, order]
    colour = (sc[0] % 3) + 3 * (sc[1] % 3) + 9 * (sc[2] % 3)
    offs = [(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)]
    for col in range(27):
        in_phase = colour == col
        for k in range(int(rank[in_phase].max(initial=-1)) + 1):
            sel = np.nonzero(in_phase & (rank == k))[0]
            sel = sel[taken[skey[sel]] < 0]                # cells still without a sample
            if sel.size == 0:
                continue
            idx = order[sel]
            p = cand[:, idx]
            ok = np.ones(sel.size, dtype=bool)
            for dx, dy, dz in offs:
                x, y, z = sc[0, sel] + dx, sc[1, sel] + dy, sc[2, sel] + dz
                inb = (x >= 0) & (x < dims[0]) & (y >= 0) & (y < dims[1]) & (z >= 0) & (z < dims[2])
                nk = np.where(inb, x + dims[0] * (y + dims[1] * z), 0)
                j = np.where(inb, taken[nk], -1)
                has = j >= 0
                if has.any():
                    q = cand[:, np.where(has, j, 0)]
                    d = p - q
                    s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                    ok &= ~has | (s >= d2)
            taken[skey[sel[ok]]] = idx[ok]
    cells = np.nonzero(taken >= 0)[0]
    return cand[:, taken[cells]], taken[cells]
