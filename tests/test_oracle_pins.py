"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU).

Each test checks the oracle against something other than itself: exact fractions
derived by hand from the Section 4 formulas (tests/golden/), closed forms
(free fall, one and two neighbours), invariants (partition of unity, uniform
field reproduction) and brute force.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import upsample_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _frac(p):
    return Fraction(p[0], p[1])


def _vec(rows):
    return np.array([float(_frac(c)) for c in rows], dtype=np.float64)


# ---------------------------------------------------------------- constants

def test_paper_constants_fixture():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    c1 = Fraction(c["c1"]["num"], c["c1"]["den"])
    # c1 is the weight at distance r_LR: (1 - r^2 / (9 r^2))^3 = (8/9)^3 exactly
    assert (1 - Fraction(1, c["support_factor_sq"]["value"])) ** 3 == c1
    assert O.C1 == float(c1)
    assert O.C2 == c["c2"]["value"]
    rmin, rmax = c["radius_ratio"]["min"], c["radius_ratio"]["max"]
    # Section 5.2's upscaling factors 15..125 are the cubes of 1/0.4 .. 1/0.2
    assert round((1 / rmax) ** 3) == 16 and round((1 / rmin) ** 3) == 125


def test_weight_closed_form_and_shape():
    for r in (0.5, 0.02, 0.0125, 1.0 / 3.0):
        assert O.weight(0.0, r) == 1.0
        assert abs(O.weight(r * r, r) - 512.0 / 729.0) < 1e-15
        assert abs(O.weight(4 * r * r, r) - 125.0 / 729.0) < 1e-15
        assert O.weight(9 * r * r, r) < 1e-30   # zero up to the rounding of 9 r^2
        assert O.weight(9.5 * r * r, r) == 0.0
        assert O.weight(100 * r * r, r) == 0.0
        d = np.linspace(0.0, 3 * r, 1001)
        w = O.weight(d * d, r)
        assert np.all(np.diff(w) <= 0.0) and w.min() >= 0.0 and w.max() <= 1.0
        # C1 at the support radius: slope -> 0
        eps = 1e-6 * r
        slope = (O.weight((3 * r) ** 2, r) - O.weight((3 * r - eps) ** 2, r)) / eps
        assert abs(slope) < 1e-9 / r


# ---------------------------------------------------------------- golden cases

def _case_inputs(case):
    lr_x = np.array([[float(_frac(c)) for c in p] for p in case["lr_x"]]).T.astype(np.float32)
    lr_v = np.array([[float(_frac(c)) for c in p] for p in case["lr_v"]]).T.astype(np.float32)
    hr_x = _vec(case["hr_x"]).reshape(3, 1).astype(np.float32)
    hr_v = _vec(case["hr_v"]).reshape(3, 1).astype(np.float32)
    return lr_x, lr_v, np.array(case["lr_rigid"], dtype=np.uint8), hr_x, hr_v


def test_golden_closed_form_cases():
    fx = json.load(open(os.path.join(GOLDEN, "closed_form_cases.json")))
    prm = dict(r_lr=float(_frac(fx["r_lr"])), r_hr=0.1, dt=float(_frac(fx["dt"])),
               g=_vec(fx["g"]), c1=O.C1, c2=O.C2, walls=np.zeros((0, 12), np.float32))
    for case in fx["cases"]:
        lr_x, lr_v, rigid, hr_x, hr_v = _case_inputs(case)
        o = O.step(lr_x, lr_v, rigid, hr_x, hr_v, prm)
        assert abs(o["alpha"][0] - float(_frac(case["alpha"]))) < 1e-15, case["name"]
        np.testing.assert_allclose(o["v"][:, 0], _vec(case["v_new"]), rtol=0, atol=1e-14,
                                   err_msg=case["name"])
        np.testing.assert_allclose(o["x"][:, 0], _vec(case["x_new"]), rtol=0, atol=1e-14,
                                   err_msg=case["name"])


# ---------------------------------------------------------------- closed forms

def _prm(r=0.02, dt=1.0 / 60.0, g=(0.0, -9.81, 0.0), walls=None, r_hr=0.005):
    return dict(r_lr=r, r_hr=r_hr, dt=dt, g=np.array(g), c1=O.C1, c2=O.C2,
                walls=np.zeros((0, 12), np.float32) if walls is None else walls)


def test_free_fall_closed_form():
    rng = np.random.default_rng(0)
    n, steps = 64, 12
    x0 = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    v0 = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    prm = _prm()
    empty = np.zeros((3, 0), np.float32)
    x, v = x0.astype(np.float64), v0.astype(np.float64)
    for _ in range(steps):
        o = O.step(empty, empty, np.zeros(0, np.uint8), x, v, prm)
        x, v = o["x"], o["v"]
        assert np.all(o["alpha"] == 1.0)
    g = np.array(prm["g"])[:, None]
    dt = prm["dt"]
    x0, v0 = x0.astype(np.float64), v0.astype(np.float64)
    v_ref = v0 + steps * dt * g
    x_ref = x0 + steps * dt * v0 + dt * dt * g * steps * (steps + 1) / 2.0
    np.testing.assert_allclose(v, v_ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("d_over_r", [0.0, 0.3, 0.999, 1.0, 1.5, 2.5, 2.99])
def test_single_neighbour(d_over_r):
    r = 0.02
    prm = _prm(r=r)
    rng = np.random.default_rng(int(d_over_r * 1000))
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    hr_x = np.array([[0.3], [0.4], [0.5]], np.float32)
    lr_x = (hr_x[:, 0] + d_over_r * r * direction).astype(np.float32).reshape(3, 1)
    V = rng.normal(size=(3, 1)).astype(np.float32)
    v = rng.normal(size=(3, 1)).astype(np.float32)
    o = O.step(lr_x, V, np.zeros(1, np.uint8), hr_x, v, prm)
    d2 = np.sum((lr_x.astype(np.float64) - hr_x.astype(np.float64)) ** 2)
    w = (1.0 - d2 / (9 * np.float64(np.float32(r)) ** 2)) ** 3
    # max w / sum w = 1 >= c2, so alpha = 1 - w for every distance inside the support
    assert abs(o["alpha"][0] - (1.0 - w)) < 1e-14
    v_ref = w * V[:, 0] + (1.0 - w) * (v[:, 0] + prm["dt"] * prm["g"])
    np.testing.assert_allclose(o["v"][:, 0], v_ref, atol=1e-13)
    np.testing.assert_allclose(o["x"][:, 0], hr_x[:, 0] + prm["dt"] * v_ref, atol=1e-13)


@pytest.mark.parametrize("d_over_r", [0.2, 0.7, 0.99, 1.01, 1.7, 2.6])
def test_two_symmetric_neighbours(d_over_r):
    r = 0.5  # power of two: the mirrored LR sit at exactly equal distances
    prm = _prm(r=r)
    hr_x = np.zeros((3, 1), np.float32)
    e = np.array([0.0, 0.0, 1.0])
    lr_x = np.stack([d_over_r * r * e, -d_over_r * r * e], axis=1).astype(np.float32)
    V = np.array([[1.0, -2.0], [0.5, 0.25], [3.0, 1.0]], np.float32)
    v = np.array([[0.1], [0.2], [0.3]], np.float32)
    o = O.step(lr_x, V, np.zeros(2, np.uint8), hr_x, v, prm)
    dd = np.float64(np.float32(d_over_r * r))
    w = (1.0 - dd * dd / (9 * r * r)) ** 3
    vt = V.astype(np.float64).mean(axis=1)
    # max w / sum w = 1/2 < c2: alpha = 1 - w only when w <= c1, i.e. d >= r
    alpha = (1.0 - w) if d_over_r >= 1.0 else 0.0
    assert abs(o["alpha"][0] - alpha) < 1e-14
    v_ref = (1 - alpha) * vt + alpha * (v[:, 0] + prm["dt"] * prm["g"])
    np.testing.assert_allclose(o["v"][:, 0], v_ref, atol=1e-13)


def test_sparse_many_neighbours_alpha_is_one_minus_max():
    # six LR on the axes at 2r: each w = 125/729 <= c1, max/sum = 1/6 < c2 -> alpha = 1 - 125/729
    r = 0.5
    prm = _prm(r=r)
    pts = []
    for ax in range(3):
        for s in (1.0, -1.0):
            p = np.zeros(3)
            p[ax] = 2 * r * s
            pts.append(p)
    lr_x = np.array(pts).T.astype(np.float32)
    V = np.ones((3, 6), np.float32)
    o = O.step(lr_x, V, np.zeros(6, np.uint8), np.zeros((3, 1), np.float32),
               np.zeros((3, 1), np.float32), prm)
    assert abs(o["alpha"][0] - (1 - 125 / 729)) < 1e-15
    # and dense packing: 6 LR at r/2 -> max w > c1 and max/sum = 1/6 -> alpha = 0
    o = O.step(lr_x / 4, V, np.zeros(6, np.uint8), np.zeros((3, 1), np.float32),
               np.zeros((3, 1), np.float32), prm)
    assert o["alpha"][0] == 0.0
    np.testing.assert_allclose(o["v"][:, 0], 1.0, atol=1e-15)


def _random_scene(seed, n_lr=400, n_hr=3000, r=0.05, box=1.0):
    rng = np.random.default_rng(seed)
    lr_x = rng.uniform(0, box, (3, n_lr)).astype(np.float32)
    lr_v = rng.normal(size=(3, n_lr)).astype(np.float32)
    hr_x = rng.uniform(0, box, (3, n_hr)).astype(np.float32)
    hr_v = rng.normal(size=(3, n_hr)).astype(np.float32)
    return lr_x, lr_v, hr_x, hr_v


def test_partition_of_unity_and_uniform_field():
    lr_x, lr_v, hr_x, hr_v = _random_scene(1)
    prm = _prm(r=0.05)
    o = O.step(lr_x, lr_v, None, hr_x, hr_v, prm, keep=True)
    S = o["S"]
    has = S > 0
    ratio_sum = np.bincount(o["ii"], weights=o["w"] / S[o["ii"]], minlength=S.size)
    np.testing.assert_allclose(ratio_sum[has], 1.0, atol=1e-14)
    # a uniform LR field is reproduced exactly where alpha = 0 (Shepard reproduces constants)
    Vc = np.array([0.3, -1.2, 2.5], np.float32)
    uni = np.repeat(Vc[:, None], lr_x.shape[1], axis=1)
    o2 = O.step(lr_x, uni, None, hr_x, hr_v, prm)
    dense = o2["alpha"] == 0.0
    assert dense.sum() > 100
    np.testing.assert_allclose(o2["v"][:, dense], np.repeat(Vc[:, None].astype(np.float64), dense.sum(), 1),
                               atol=1e-14)
    # elsewhere the closed form of the blend holds
    a = o2["alpha"]
    ref = (1 - a) * np.where(o2["S"] > 0, 1.0, 0.0) * Vc[:, None].astype(np.float64) + \
        a * (hr_v.astype(np.float64) + prm["dt"] * prm["g"][:, None])
    np.testing.assert_allclose(o2["v"], ref, atol=1e-13)


def test_alpha_rule_all_branches():
    lr_x, lr_v, hr_x, hr_v = _random_scene(2, n_lr=800, n_hr=4000)
    prm = _prm(r=0.05)
    o = O.step(lr_x, lr_v, None, hr_x, hr_v, prm)
    S, M, a = o["S"], o["M"], o["alpha"]
    c1, c2 = 512 / 729, 0.6
    sparse = M <= c1
    lonely = (S > 0) & (M / np.where(S > 0, S, 1) >= c2)
    np.testing.assert_array_equal(a > 0, (sparse | lonely) & (M < 1))
    np.testing.assert_allclose(a[sparse | lonely], 1 - M[sparse | lonely], atol=0)
    assert np.all(a[~(sparse | lonely)] == 0)
    # every branch occurs in this scene
    assert sparse.sum() and (lonely & ~sparse).sum() and (~sparse & ~lonely).sum()


# ---------------------------------------------------------------- rigid rule

def test_rigid_only_neighbours_give_free_fall():
    lr_x, lr_v, hr_x, hr_v = _random_scene(3)
    prm = _prm(r=0.05)
    rigid = np.ones(lr_x.shape[1], np.uint8)
    o = O.step(lr_x, lr_v, rigid, hr_x, hr_v, prm)
    np.testing.assert_array_equal(o["alpha"], 1.0)
    np.testing.assert_allclose(o["v"], hr_v + prm["dt"] * prm["g"][:, None], atol=1e-14)


def test_rigid_counts_only_with_granular_in_vicinity():
    lr_x, lr_v, hr_x, hr_v = _random_scene(4)
    prm = _prm(r=0.05)
    rng = np.random.default_rng(5)
    rigid = (rng.uniform(size=lr_x.shape[1]) < 0.5).astype(np.uint8)
    o = O.step(lr_x, lr_v, rigid, hr_x, hr_v, prm, keep=True)
    indptr, jj = O.neighbours_bruteforce(lr_x, hr_x, O.grid_spec(0.05, [0] * 3, [1] * 3).h2_f)
    ii = np.repeat(np.arange(hr_x.shape[1]), np.diff(indptr))
    has_gran = np.bincount(ii, weights=(rigid[jj] == 0), minlength=hr_x.shape[1]) > 0
    has_any = np.diff(indptr) > 0
    # HR with only rigid neighbours fall freely
    only_rigid = has_any & ~has_gran
    assert only_rigid.sum() > 10
    np.testing.assert_allclose(o["v"][:, only_rigid],
                               hr_v[:, only_rigid] + prm["dt"] * prm["g"][:, None], atol=1e-14)
    # HR with a granular neighbour use all neighbours, rigid ones included
    mixed = has_gran
    cnt = np.bincount(o["ii"], minlength=hr_x.shape[1])
    np.testing.assert_array_equal(cnt[mixed], np.diff(indptr)[mixed])


# ---------------------------------------------------------------- neighbours / grid

def _adversarial_points(rng, spec, n):
    """Points on cell faces, outside the box, coincident with each other."""
    lo = spec.lo.astype(np.float64)
    faces = lo[:, None] + spec.cs * rng.integers(-1, max(spec.dims) + 1, size=(3, n))
    P = rng.uniform(-0.1, 1.1, (3, n))
    pick = rng.uniform(size=(3, n)) < 0.4
    P[pick] = faces[pick]
    P[:, : n // 10] = P[:, n // 10: 2 * (n // 10)]
    return P.astype(np.float32)


@pytest.mark.parametrize("cell_factor", [0.0, 1.5, 0.5, 0.34])
def test_neighbour_routes_agree(cell_factor):
    rng = np.random.default_rng(7)
    r = 0.04
    spec = O.grid_spec(r, [0, 0, 0], [1, 1, 1], cell_factor)
    lr_x = _adversarial_points(rng, spec, 300)
    hr_x = _adversarial_points(rng, spec, 400)
    # HR at exactly the support distance from an LR, and at r
    hr_x[:, :20] = (lr_x[:, :20].astype(np.float64) + np.array([[3 * r], [0], [0]])).astype(np.float32)
    hr_x[:, 20:40] = (lr_x[:, 20:40].astype(np.float64) + np.array([[0], [r], [0]])).astype(np.float32)
    b = O.neighbours_bruteforce(lr_x, hr_x, spec.h2_f)
    k = O.neighbours_kdtree(lr_x, hr_x, spec.h, spec.h2_f)
    g = O.neighbours_grid(lr_x, hr_x, spec)
    for other in (k, g):
        np.testing.assert_array_equal(b[0], other[0])
        np.testing.assert_array_equal(b[1], other[1])
    assert b[1].size > 200


def test_grid_keys_locate_cells():
    rng = np.random.default_rng(8)
    spec = O.grid_spec(0.0125, [0, 0, 0], [1, 2.4, 1])
    X = rng.uniform(-0.05, 2.45, (3, 20000)).astype(np.float32)
    c = O.cell_coords(X, spec)
    for a in range(3):
        lo = spec.lo[a] + c[a] * spec.cs
        hi = lo + spec.cs
        x = X[a].astype(np.float64)
        inside = (x >= spec.lo[a]) & (x < spec.lo[a] + spec.dims[a] * spec.cs)
        tol = 1e-6
        assert np.all(x[inside] >= lo[inside] - tol) and np.all(x[inside] < hi[inside] + tol)
        assert np.all(c[a][x < spec.lo[a]] == 0)
        assert np.all(c[a][x >= spec.lo[a] + spec.dims[a] * spec.cs + tol] == spec.dims[a] - 1)
    keys = O.cell_keys(X, spec)
    gx, gy, gz = spec.dims
    np.testing.assert_array_equal(keys % gx, c[0])
    np.testing.assert_array_equal((keys // gx) % gy, c[1])
    np.testing.assert_array_equal(keys // (gx * gy), c[2])
    perm, cs = O.sort_by_cell(keys, spec.n_cells)
    assert np.array_equal(np.sort(perm), np.arange(X.shape[1]))
    ks = keys[perm]
    assert np.all(np.diff(ks.astype(np.int64)) >= 0)
    ties = np.diff(ks.astype(np.int64)) == 0
    assert np.all(np.diff(perm.astype(np.int64))[ties] > 0)
    assert cs[0] == 0 and cs[-1] == X.shape[1]
    for k in rng.integers(0, spec.n_cells, 200):
        assert cs[k + 1] - cs[k] == np.count_nonzero(keys == k)
        assert np.all(keys[perm[cs[k]:cs[k + 1]]] == k)


def test_grid_spec_reach_covers_support():
    for kappa in (0.0, 1.0, 1.0001, 0.5, 0.49, 0.34, 2.0):
        spec = O.grid_spec(0.01, [0, 0, 0], [3, 3, 3], kappa)
        assert spec.reach * spec.cs >= spec.h * (1 + 1e-6)
        assert (spec.reach - 1) * spec.cs < spec.h * (1 + 1e-3)
    assert O.grid_spec(0.01, [0, 0, 0], [1, 1, 1], 1.0).reach == 2
    assert O.grid_spec(0.01, [0, 0, 0], [1, 1, 1], 1.0001).reach == 1


# ---------------------------------------------------------------- walls

def _floor_and_plate():
    from workloads.generators import wall
    floor = wall((0, 1, 0), 0.0)
    plate = wall((0, 1, 0), 0.6, o=(0.5, 0.6, 0.5), R=0.1)
    return np.stack([floor, plate])


def test_walls_push_clip_and_orifice():
    walls = _floor_and_plate()
    r_hr = 0.01
    # particle 0: lands on the plate outside the hole -> pushed to y = 0.61, vy clipped to 0
    # particle 1: above the hole -> passes through
    # particle 2: below the plate moving up through it -> one-sided, not stopped
    # particle 3: hits the floor
    x_old = np.array([[0.8, 0.5, 0.8, 0.3], [0.62, 0.62, 0.58, 0.02], [0.8, 0.52, 0.8, 0.3]])
    x_new = x_old + np.array([[0.0, 0.0, 0.0, 0.01], [-0.05, -0.05, 0.05, -0.03], [0, 0, 0, 0]])
    v_new = np.array([[0.0, 0.0, 0.0, 0.6], [-3.0, -3.0, 3.0, -1.8], [0.0, 0.0, 0.0, 0.0]])
    x, v = x_new.T.copy(), v_new.T.copy()
    rec = O.apply_walls(x_old.T, x, v, walls.astype(np.float32), r_hr)
    np.testing.assert_allclose(x[0], [0.8, 0.61, 0.8], atol=1e-7)
    np.testing.assert_allclose(v[0], [0.0, 0.0, 0.0], atol=0)
    np.testing.assert_allclose(x[1], x_new[:, 1], atol=0)
    np.testing.assert_allclose(x[2], x_new[:, 2], atol=0)
    np.testing.assert_allclose(x[3], [0.31, 0.01, 0.3], atol=1e-7)
    np.testing.assert_allclose(v[3], [0.6, 0.0, 0.0], atol=0)
    assert rec["pushed"][0, 1] and rec["pushed"][3, 0] and not rec["pushed"][1].any()


def test_walls_invariants_on_drain():
    from workloads import configs
    sc = configs.drain(scale=1.0 / 512)
    prm = sc.params()
    x, v = sc.hr_x0.astype(np.float64), sc.hr_v0.astype(np.float64)
    rng = np.random.default_rng(9)
    for t in range(1, 6):
        X, V = sc.lr_frame(t)
        v = v + rng.normal(0, 2.0, v.shape)      # kick HR hard into the walls
        o = O.step(X, V, sc.lr_rigid, x, v, prm, keep=True)
        xn = o["x"].T
        for k in range(sc.walls.shape[0]):
            n, d = sc.walls[k, :3].astype(np.float64), float(sc.walls[k, 3])
            p = o["wall"]["pushed"][:, k]
            later = o["wall"]["pushed"][:, k + 1:].any(axis=1)
            ok = p & ~later
            assert np.all(xn[ok] @ n - d >= prm["r_hr"] - 1e-8)   # |n| = 1 to float32 rounding
            c = o["wall"]["clipped"][:, k] & ~later
            assert np.all(o["v"].T[c] @ n >= -1e-6)
        x, v = o["x"], o["v"]
