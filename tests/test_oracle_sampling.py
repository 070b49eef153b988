"""Pins of the volume-sampling oracle (oracle/sampling_oracle.py, Section 4's
sampling paragraph) against what the description and geometry fix: no two
samples closer than 2r (brute force in float64), at most one sample per cell
of side 2r/sqrt(3), every sample a candidate of its own cell, every candidate
left out either never tried (its cell took an earlier one) or overlapping a
sample of an earlier phase, and the phase-at-a-time route equal to a plain
sequential pass over the cells on small inputs."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import sampling_oracle as S


def _cands(rng, m, lo, hi, clustered=False):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    if clustered:
        centres = rng.uniform(lo, hi, (8, 3))
        P = centres[rng.integers(0, 8, m)] + rng.normal(0, 0.03 * (hi - lo).max(), (m, 3))
        P = np.clip(P, lo, hi)
    else:
        P = rng.uniform(lo, hi, (m, 3))
    return np.ascontiguousarray(P.T, dtype=np.float32)


@pytest.mark.parametrize("seed,clustered", [(0, False), (1, False), (2, True), (3, True)])
def test_phases_equal_sequential_pass(seed, clustered):
    rng = np.random.default_rng(seed)
    lo, hi, r = (0.0, 0.0, 0.0), (0.3, 0.2, 0.25), 0.02
    cand = _cands(rng, 3000, lo, hi, clustered)
    a = S.sample_volume_sequential(cand, r, lo, hi)
    b, idx = S.sample_volume(cand, r, lo, hi)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(b, cand[:, idx])
    assert b.shape[1] > 10


@pytest.mark.parametrize("seed", [4, 5])
def test_samples_do_not_overlap_and_one_per_cell(seed):
    rng = np.random.default_rng(seed)
    lo, hi, r = (-0.5, 0.0, 0.2), (0.5, 0.6, 0.9), 0.011
    cand = _cands(rng, 120000, lo, hi)
    P, idx = S.sample_volume(cand, r, lo, hi)
    X = P.T.astype(np.float64)
    pairs = cKDTree(X).query_pairs(2 * r * (1 - 1e-6))
    assert not pairs, f"{len(pairs)} overlapping samples"
    side, inv, lo32, dims = S.sampling_grid(r, lo, hi)
    assert abs(side * math.sqrt(3) - 2 * np.float32(r)) < 1e-12   # cell diagonal 2r
    c = S.cells_of(P, inv, lo32, dims)
    key = c[0] + dims[0] * (c[1] + dims[1] * c[2])
    assert np.all(np.diff(key) > 0)                    # one per cell, in key order
    ci = S.cells_of(cand[:, idx], inv, lo32, dims)
    np.testing.assert_array_equal(ci, c)
    # packing fraction of the spheres of radius r: below the densest packing
    # (pi / sqrt 18), and a dense candidate set gets near the random
    # sequential jamming density (about 0.38)
    vol = np.prod(np.asarray(hi, float) - np.asarray(lo, float))
    phi = P.shape[1] * 4.0 / 3.0 * math.pi * r ** 3 / vol
    assert 0.15 < phi < math.pi / math.sqrt(18.0)


def test_left_out_candidates_were_not_tried_or_overlap_an_earlier_phase():
    rng = np.random.default_rng(6)
    lo, hi, r = (0.0, 0.0, 0.0), (0.25, 0.25, 0.25), 0.015
    cand = _cands(rng, 20000, lo, hi)
    P, idx = S.sample_volume(cand, r, lo, hi)
    side, inv, lo32, dims = S.sampling_grid(r, lo, hi)
    c = S.cells_of(cand, inv, lo32, dims)
    key = c[0] + dims[0] * (c[1] + dims[1] * c[2])
    colour = (c[0] % 3) + 3 * (c[1] % 3) + 9 * (c[2] % 3)
    chosen = dict(zip(key[idx].tolist(), idx.tolist()))
    d2 = np.float32(4.0 * float(np.float32(r)) ** 2)
    X = cand.T.astype(np.float64)
    tree = cKDTree(X[idx])
    for i in range(cand.shape[1]):
        k = int(key[i])
        j = chosen.get(k)
        if j == i or (j is not None and j < i):
            continue                                   # taken, or never tried
        # tried and rejected: some sample of an earlier colour overlaps it
        near = tree.query_ball_point(X[i], 2.0 * r * (1 + 1e-6))
        hit = False
        for n in near:
            q = idx[n]
            if colour[q] < colour[i]:
                d = cand[:, i] - cand[:, q]
                hit |= bool(((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) < d2)
        assert hit, f"candidate {i} rejected without an overlapping earlier sample"


def test_one_cell_and_phase_order():
    r = 0.05
    side = 2 * np.float32(r) / math.sqrt(3)
    # every candidate in one cell: the first one is the sample
    c = np.array([[0.01, 0.02, 0.015], [0.01, 0.011, 0.02], [0.02, 0.01, 0.01]], np.float32)
    P, idx = S.sample_volume(c, r, (0, 0, 0), (1, 1, 1))
    assert list(idx) == [0]
    # two candidates in neighbouring cells, closer than 2r: the cell of the
    # earlier colour (x-index 0, colour 0) keeps its candidate, listed second
    a = np.array([0.5 * side, 0.5 * side, 0.5 * side])
    b = a + np.array([side, 0.0, 0.0])
    cand = np.ascontiguousarray(np.stack([b, a], axis=1).astype(np.float32))
    P, idx = S.sample_volume(cand, r, (0, 0, 0), (1, 1, 1))
    assert list(idx) == [1]
    np.testing.assert_array_equal(S.sample_volume_sequential(cand, r, (0, 0, 0), (1, 1, 1)), P)
