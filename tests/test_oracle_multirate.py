"""Pins of the LR sub-stepping oracle (oracle/multirate_oracle.py) against what
the paper and the mathematics fix: Section 5.2's time steps (dt_LR = 0.005 s,
dt_HR = 0.0167 s, tests/golden/paper_constants.json) bracketed with exact
rational arithmetic, uniform motion reproduced exactly by the interpolation,
the frames themselves at theta = 0, the float32 contract within rounding of
the float64 definition, and the multi-rate rollout reducing to the
single-rate one when both time steps agree."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import multirate_oracle as MR
from oracle import upsample_oracle as O
from workloads.generators import build_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _paper_dts():
    g = json.load(open(GOLDEN))
    return g["dt_lr"]["value"], g["dt_hr"]["value"]


def test_bracket_paper_time_steps_against_rationals():
    """Every HR step of Section 5.2's time steps ends between the two LR frames
    the schedule names, at the rational weight (frames at k dt_LR)."""
    dt_lr, dt_hr = _paper_dts()
    n_steps, n_frames = 600, 2100
    sched = MR.hr_schedule(0.0, dt_hr, n_steps, 0.0, dt_lr, n_frames)
    q_lr, q_hr = Fraction(dt_lr), Fraction(dt_hr)
    per_frame = []
    for n, (k, th) in enumerate(sched):
        s = (n + 1) * q_hr / q_lr            # exact position in LR steps
        assert 0.0 <= th <= 1.0
        assert abs(Fraction(k) + Fraction(th) - s) <= Fraction(1, 10 ** 9)
        per_frame.append(math.floor(s) - (math.floor(n * q_hr / q_lr) if n else 0))
    # dt_HR / dt_LR = 3.34: each HR frame covers three or four LR steps
    assert set(per_frame) <= {3, 4} and abs(np.mean(per_frame) - dt_hr / dt_lr) < 0.01


def test_bracket_edges():
    assert MR.bracket(0.0, 0.0, 0.005, 4) == (0, 0.0)
    k, th = MR.bracket(0.015, 0.0, 0.005, 4)     # on the last frame (to float64 rounding)
    assert k == 2 and abs(th - 1.0) < 1e-9
    assert MR.bracket(0.0125, 0.0, 0.005, 4) == (2, pytest.approx(0.5, abs=1e-12))
    with pytest.raises(ValueError):
        MR.bracket(0.0151, 0.0, 0.005, 4)
    with pytest.raises(ValueError):
        MR.bracket(-1e-6, 0.0, 0.005, 4)


def test_uniform_motion_reproduced_exactly():
    """LR particles in uniform motion X(t) = a + b t, V = b: the interpolated
    state at any time is the motion itself."""
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 1, (3, 50))
    b = rng.normal(0, 1, (3, 50))
    dt = 0.005
    frames = [(a + b * (k * dt), b.copy()) for k in range(6)]
    for t in rng.uniform(0, 5 * dt, 40):
        k, th = MR.bracket(t, 0.0, dt, 6)
        X, V = MR.lerp_frame(*frames[k], *frames[k + 1], th)
        np.testing.assert_allclose(X, a + b * t, rtol=0, atol=1e-14)
        np.testing.assert_array_equal(V, b)


def test_theta_zero_is_the_frame_and_f32_contract_rounds():
    rng = np.random.default_rng(2)
    X0, X1 = rng.uniform(0, 2, (2, 3, 1000)).astype(np.float32)
    V0, V1 = rng.normal(0, 1, (2, 3, 1000)).astype(np.float32)
    x, v = MR.lerp_frame_f32(X0, V0, X1, V1, 0.0)
    np.testing.assert_array_equal(x, X0)
    np.testing.assert_array_equal(v, V0)
    for th in (0.25, 1.0 / 3.0, 0.999999, 1.0):
        x32, v32 = MR.lerp_frame_f32(X0, V0, X1, V1, th)
        x64, v64 = MR.lerp_frame(X0, V0, X1, V1, th)
        # three roundings of float32 magnitude at most 2: within 4 units of 2^-23
        assert np.abs(x32 - x64).max() <= 4 * 2.0 ** -23 * 2
        assert np.abs(v32 - v64).max() <= 4 * 2.0 ** -23 * 4
        assert x32.dtype == np.float32


def _plain_scene():
    return build_scene("plain", 512, 4096, seed=[7, 1], r_lr=0.02)


def test_multirate_equals_single_rate_when_steps_agree():
    """With dt_LR = dt_HR every HR step ends on an LR frame: the multi-rate
    rollout is the single-rate rollout over the frames."""
    sc = _plain_scene()
    prm = sc.params()
    T = 4
    frames = [(sc.lr_x0, np.zeros_like(sc.lr_x0))] + [sc.lr_frame(t) for t in range(1, T + 1)]
    # float64 interpolation: a schedule weight of 1 - 1e-16 then gives the
    # frame to float64 rounding (its float32 contract may round an LR
    # position by one unit)
    states, sched = MR.rollout_multirate(frames, 0.0, prm["dt"], 0.0, T, None, sc.hr_x0, sc.hr_v0, prm,
                                         f32_frames=False)
    ref, _ = O.rollout(frames[1:], None, sc.hr_x0, sc.hr_v0, prm)
    for (k, th), n in zip(sched, range(T)):
        assert (k, th) in ((n + 1, 0.0), (n, 1.0)) or abs(k + th - (n + 1)) < 1e-12
    for (x, v), (xr, vr) in zip(states, ref):
        np.testing.assert_allclose(x, xr, rtol=0, atol=1e-12)
        np.testing.assert_allclose(v, vr, rtol=0, atol=1e-10)


def test_time_varying_uniform_field_is_followed():
    """Every LR particle moving with the same velocity V(t), linear in time:
    the interpolated field is V(t_{n+1}) exactly, so an HR particle whose blend
    parameter is zero (dense support) takes exactly that velocity (Section 4,
    uniform field reproduced by the Shepard average)."""
    sc = _plain_scene()
    prm = dict(sc.params())
    prm["walls"] = np.zeros((0, 12), np.float32)
    dt_lr = 0.005
    c0, c1 = np.array([0.3, -0.2, 0.1]), np.array([-1.0, 0.5, 2.0])   # V(t) = c0 + c1 t
    X = sc.lr_x0.astype(np.float64)
    frames = []
    for k in range(12):
        t = k * dt_lr
        frames.append((X + (c0[:, None] * t + 0.5 * c1[:, None] * t * t), np.repeat((c0 + c1 * t)[:, None],
                                                                                     X.shape[1], axis=1)))
    states, sched = MR.rollout_multirate(frames, 0.0, dt_lr, 0.0, 3, None, sc.hr_x0, sc.hr_v0, prm,
                                         f32_frames=False)
    for n, (k, th) in enumerate(sched):
        t = (n + 1) * prm["dt"]
        Xn, Vn = MR.lerp_frame(*frames[k], *frames[k + 1], th)
        np.testing.assert_allclose(Vn, np.repeat((c0 + c1 * t)[:, None], X.shape[1], axis=1), atol=1e-12)
        o = O.step(Xn, Vn, None, states[n][0], states[n][1], prm)
        dense = o["alpha"] == 0.0
        assert dense.sum() > 100
        np.testing.assert_allclose(o["v"][:, dense], np.repeat((c0 + c1 * t)[:, None], dense.sum(), axis=1),
                                   atol=1e-12)
