"""Pins of the LR simulation oracle (oracle/pbd_oracle.py; Section 3,
Algorithm 1) against closed forms: free fall, a head-on overlap resolved to
exactly 2r with the mass ratio of Section 3's contact, a static partner,
constraint averaging, the static and kinetic friction branches, the centre of
mass conserved by isolated pairs, the scaled mass of Algorithm 1, the
polar-decomposition rotation, shape matching leaving a rigid motion
unchanged and restoring a deformed body, and stabilization not changing
velocities; the contact pairs against all pairs tested one by one (float64
and the float32 contract), and a forced decision taking the other branch."""
import json
import math
import os

import numpy as np
import pytest

from oracle import pbd_oracle as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _prm(**kw):
    base = dict(r=0.02, dt=0.005, g=(0.0, 0.0, 0.0), mass_scaling=False)
    base.update(kw)
    return P.PBDParams(**base)


def _one(x, v=None, body=None, inv_m=None, rest=None, **kw):
    x = np.asarray(x, float)
    n = x.shape[1]
    v = np.zeros_like(x) if v is None else np.asarray(v, float)
    body = np.full(n, P.GRANULAR) if body is None else np.asarray(body)
    inv_m = np.ones(n) if inv_m is None else np.asarray(inv_m, float)
    rest = np.zeros_like(x) if rest is None else rest
    return P.step(x, v, body, inv_m, rest, _prm(**kw))


def test_paper_defaults():
    g = json.load(open(GOLDEN))
    prm = P.PBDParams(r=0.02)
    assert prm.dt == g["dt_lr"]["value"]
    assert abs(np.linalg.norm(prm.g) - g["gravity_magnitude"]["value"]) < 1e-12
    assert (prm.mu_s, prm.mu_k) == (0.35, 0.3) and (prm.stab_iters, prm.solve_iters) == (2, 5)


def test_free_fall():
    x0 = np.array([[0.5], [0.7], [0.5]])
    v0 = np.array([[0.1], [0.0], [-0.2]])
    x, v = x0.copy(), v0.copy()
    dt, g = 0.005, np.array([0.0, -9.81, 0.0])
    for n in range(1, 6):
        x, v = _one(x, v, g=tuple(g))
        np.testing.assert_allclose(v[:, 0], v0[:, 0] + n * dt * g, atol=1e-12)
        np.testing.assert_allclose(x[:, 0], x0[:, 0] + n * dt * v0[:, 0] + dt * dt * g * n * (n + 1) / 2, atol=1e-12)


def test_head_on_overlap_resolves_to_contact_distance():
    r = 0.02
    # overlap 0.01: equal masses move 0.005 each; the pair is isolated (one
    # constraint each), so the first iteration already separates it to 2r
    x = np.array([[0.5, 0.5 + 2 * r - 0.01], [0.3, 0.3], [0.5, 0.5]])
    xn, vn = _one(x, stab_iters=0)
    np.testing.assert_allclose(xn[0], [0.5 - 0.005, 0.5 + 2 * r - 0.01 + 0.005], atol=1e-15)
    np.testing.assert_allclose(vn[0], [-0.005 / 0.005, 0.005 / 0.005], atol=1e-12)
    # mass ratio 3:1 (w 1 and 3): the lighter particle takes 3/4 of the overlap
    xn, _ = _one(x, inv_m=[1.0, 3.0], stab_iters=0)
    np.testing.assert_allclose(xn[0] - x[0], [-0.0025, 0.0075], atol=1e-15)
    # a static partner does not move; the dynamic particle takes it all
    xn, vn = _one(x, body=[P.STATIC, P.GRANULAR], inv_m=[0.0, 1.0], stab_iters=0)
    np.testing.assert_allclose(xn[0], [0.5, 0.5 + 2 * r], atol=1e-15)
    assert np.all(vn[:, 0] == 0.0)


def test_constraint_averaging():
    r = 0.02
    # particle 1 between 0 and 2, overlapping both by 0.004: its two contact
    # displacements cancel (averaged: 0); the ends move outward by half each
    x = np.array([[0.5 - 2 * r + 0.004, 0.5, 0.5 + 2 * r - 0.004], [0.3] * 3, [0.5] * 3])
    xn, _ = _one(x, stab_iters=0, solve_iters=1)
    np.testing.assert_allclose(xn[0] - x[0], [-0.002, 0.0, 0.002], atol=1e-15)
    # particle 1 overlaps 0 along x (by 0.004) and 2 along y (by 0.002): its
    # two displacements are averaged, the others take theirs whole
    x = np.array([[0.5, 0.5 + 2 * r - 0.004, 0.5 + 2 * r - 0.004], [0.3, 0.3, 0.3 + 2 * r - 0.002],
                  [0.5] * 3])
    assert np.linalg.norm(x[:, 2] - x[:, 0]) > 2 * r   # 0 and 2 do not touch
    xn, _ = _one(x, stab_iters=0, solve_iters=1)
    np.testing.assert_allclose(xn - x, [[-0.002, 0.001, 0.0], [0.0, -0.0005, 0.001], [0.0, 0.0, 0.0]],
                               atol=1e-15)


def test_friction_static_and_kinetic_branches():
    r, mu_s, mu_k = 0.02, 0.35, 0.3
    dt = 0.005
    # two overlapping particles (by 0.01 along x) sliding tangentially (z),
    # still in contact at the predicted positions
    x = np.array([[0.5, 0.5 + 2 * r - 0.01], [0.3, 0.3], [0.5, 0.5]])
    for vz, static in ((0.5, True), (2.0, False)):
        v = np.array([[0.0, 0.0], [0.0, 0.0], [vz, -vz]])
        xn, vn = _one(x, v, stab_iters=0, solve_iters=1)
        xt = x + dt * v                          # predicted positions: the collision vector
        n = xt[:, 1] - xt[:, 0]
        n /= np.linalg.norm(n)
        perp = lambda a: a - (a @ n) * n
        before = perp((xt[:, 0] - x[:, 0]) - (xt[:, 1] - x[:, 1]))    # contact moves along n only
        after = perp((xn[:, 0] - x[:, 0]) - (xn[:, 1] - x[:, 1]))
        assert (np.linalg.norm(before) < 2 * r * mu_s) == static
        if static:
            # static friction cancels the relative tangential displacement
            assert np.linalg.norm(after) < 1e-15
        else:
            # kinetic: the correction is 2 r mu_k long (half to each, equal masses)
            assert abs(np.linalg.norm(before) - np.linalg.norm(after) - 2 * r * mu_k) < 1e-15
            np.testing.assert_allclose(after / np.linalg.norm(after), before / np.linalg.norm(before), atol=1e-12)


def test_isolated_pairs_conserve_the_centre_of_mass():
    rng = np.random.default_rng(1)
    r = 0.02
    # well separated pairs, each overlapping by a random amount, random velocities
    base = rng.uniform(0.1, 0.9, (3, 40)) * np.array([[1.0], [1.0], [1.0]])
    base = base[:, np.argsort(base[0])]
    base[0] = np.linspace(0.05, 0.95, 40) * 10   # far apart in x
    dirn = rng.normal(size=(3, 40))
    dirn /= np.linalg.norm(dirn, axis=0)
    other = base + dirn * rng.uniform(1.5 * r, 1.99 * r, 40)
    x = np.concatenate([base, other], axis=1)
    v = rng.normal(0, 0.3, x.shape)
    xn, vn = _one(x, v)
    np.testing.assert_allclose(xn.mean(axis=1), (x + 0.005 * v).mean(axis=1), atol=1e-14)


def test_scaled_mass_of_algorithm_one():
    prm = P.PBDParams(r=0.02, ground_y=0.1)
    x = np.array([[0.0, 0.0], [0.1, 0.6], [0.0, 0.0]])
    w = P.scaled_inv_mass(x, np.array([2.0, 2.0]), prm)
    np.testing.assert_allclose(w, [2.0, 2.0 * math.exp(0.5)], rtol=1e-15)
    # a higher particle (lighter scaled mass) takes more of a shared overlap
    r = 0.02
    x = np.array([[0.5, 0.5], [0.2, 0.2 + 2 * r - 0.004], [0.5, 0.5]])
    xn, _ = P.step(x, np.zeros_like(x), np.full(2, P.GRANULAR), np.ones(2), np.zeros_like(x),
                   P.PBDParams(r=r, g=(0.0, 0.0, 0.0), stab_iters=0, ground_y=0.0))
    wl, wu = math.exp(0.2), math.exp(0.2 + 2 * r - 0.004)
    np.testing.assert_allclose(xn[1] - x[1], [-0.004 * wl / (wl + wu), 0.004 * wu / (wl + wu)], atol=1e-15)


def test_polar_rotation_recovers_the_rotation():
    rng = np.random.default_rng(2)
    for _ in range(20):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        a, b, c, d = q
        R = np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                      [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                      [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])
        A = rng.normal(size=(3, 3))
        S = A @ A.T + 3 * np.eye(3)                 # symmetric positive definite
        np.testing.assert_allclose(P.polar_rotation(R @ S), R, atol=1e-12)


def _body(n_side=4, r=0.02):
    g = (np.arange(n_side) - (n_side - 1) / 2) * 2 * r
    X = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    return X - X.mean(axis=1, keepdims=True)


def test_shape_matching_keeps_a_rigid_motion_and_restores_a_deformed_body():
    rest = _body()
    n = rest.shape[1]
    th = 0.3
    R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
    pos = R @ rest + np.array([[0.5], [0.4], [0.5]])
    body = np.zeros(n, dtype=int)
    np.testing.assert_allclose(P.shape_matching(pos, body, rest), 0.0, atol=1e-14)
    # a rigid motion survives a whole step (no contacts: the body's particles
    # do not collide with each other)
    v = np.cross(np.array([0.0, 2.0, 0.0]), (pos - pos.mean(axis=1, keepdims=True)).T).T + 0.3
    xn, vn = P.step(pos, v, body, np.ones(n), rest, _prm())
    Rn = P.polar_rotation((xn - xn.mean(axis=1, keepdims=True)) @ rest.T)
    np.testing.assert_allclose(xn, Rn @ rest + xn.mean(axis=1, keepdims=True), atol=1e-12)
    # a deformed body is projected back onto its rest shape
    rng = np.random.default_rng(3)
    bent = pos + rng.normal(0, 0.003, pos.shape)
    xn, _ = P.step(bent, np.zeros_like(bent), body, np.ones(n), rest, _prm(solve_iters=1))
    Rn = P.polar_rotation((xn - xn.mean(axis=1, keepdims=True)) @ rest.T)
    np.testing.assert_allclose(xn, Rn @ rest + xn.mean(axis=1, keepdims=True), atol=1e-12)


def test_stabilization_moves_x_and_prediction_together():
    r = 0.02
    # an overlap at rest without gravity: stabilization separates the pair in
    # both x and x~, so the velocities stay zero
    x = np.array([[0.5, 0.5 + 2 * r - 0.006], [0.3, 0.3], [0.5, 0.5]])
    xn, vn = _one(x, stab_iters=2)
    np.testing.assert_allclose(vn, 0.0, atol=1e-12)
    np.testing.assert_allclose(xn[0, 1] - xn[0, 0], 2 * r, atol=1e-15)


def test_contact_pairs_against_brute_force():
    # every pair tested one by one, in float64 and in the float32 contract
    rng = np.random.default_rng(7)
    r = 0.02
    x = rng.uniform(0.0, 0.25, (3, 150))
    body = rng.choice([P.GRANULAR, P.STATIC, 0, 1], 150)
    x32 = x.astype(np.float32)
    d2 = np.float32(4.0 * float(np.float32(r)) ** 2)
    want64, want32 = set(), set()
    for i in range(150):
        for j in range(i + 1, 150):
            if (body[i] == P.STATIC and body[j] == P.STATIC) or (body[i] >= 0 and body[i] == body[j]):
                continue
            if math.dist(x[:, i], x[:, j]) < 2 * r:
                want64.add((i, j))
            dx, dy, dz = (x32[a, j] - x32[a, i] for a in range(3))
            if (dx * dx + dy * dy) + dz * dz < d2:
                want32.add((i, j))
    assert {tuple(p) for p in P.contact_pairs(x, body, r)} == want64 and want64
    assert {tuple(p) for p in P.contact_pairs(x32, body, np.float32(r), f32=True)} == want32


def test_forced_decisions_take_the_other_branch():
    r, dt, mu_k = 0.02, 0.005, 0.3
    # a tangential slide whose relative displacement lies between 2 r mu_k
    # and 2 r mu_s: static friction by the oracle's own decision
    x = np.array([[0.5, 0.5 + 2 * r - 0.01], [0.3, 0.3], [0.5, 0.5]])
    v = np.array([[0.0, 0.0], [0.0, 0.0], [1.45, -1.45]])
    prm = _prm()
    body = np.full(2, P.GRANULAR)
    _, xt, w = P.predict(x, v, body, np.ones(2), prm)
    pairs = P.contact_pairs(xt, body, r)
    rest = np.zeros_like(x)
    own, info = P.solve_iteration(xt, x, pairs, w, body, rest, prm)
    n = (xt[:, 1] - xt[:, 0]) / np.linalg.norm(xt[:, 1] - xt[:, 0])
    Dx = (xt[:, 0] - x[:, 0]) - (xt[:, 1] - x[:, 1])
    Dt = Dx - (Dx @ n) * n
    lt = np.linalg.norm(Dt)
    assert 2 * r * mu_k < lt < 2 * r * 0.35
    assert info["act"][0] and abs(info["fric_margin"][0] - (lt - 2 * r * 0.35)) < 1e-15
    # contact switched off: the pair is no constraint, x~ stays as predicted
    off, _ = P.solve_iteration(xt, x, pairs, w, body, rest, prm, force_act=[0])
    np.testing.assert_array_equal(off, xt)
    # kinetic branch forced: the correction along Dt is shorter by
    # (|Dt| - 2 r mu_k) / 2 (equal masses)
    kin, _ = P.solve_iteration(xt, x, pairs, w, body, rest, prm, force_static=[0])
    np.testing.assert_allclose(kin[:, 0] - own[:, 0], 0.5 * (lt - 2 * r * mu_k) * Dt / lt, atol=1e-15)
    np.testing.assert_allclose(kin[:, 1] - own[:, 1], -0.5 * (lt - 2 * r * mu_k) * Dt / lt, atol=1e-15)
    # the stabilization iteration honours a forced decision too
    xs, xts, m = P.stab_iteration(x, xt, P.contact_pairs(x, body, r), w, r, force_act=[0])
    np.testing.assert_array_equal(xs, x)
    np.testing.assert_array_equal(xts, xt)
    assert abs(m[0] + 0.01) < 1e-15
