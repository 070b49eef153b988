"""Plain CPU oracle for LR sub-stepping: the LR state at the HR time level.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and is written from the paper:

* Section 5.2 runs the LR simulation with its own time step dt_LR (0.005 s by
  default, CFL-limited) and the HR upsampling with dt_HR = 0.0167 s, and times
  one HR frame as the LR steps that cover one dt_HR.  So an HR step does not in
  general start or end on an LR step.
* Section 4 advances an HR particle from t to t + 1 with the LR velocity field
  at t + 1 (the weights use the LR positions of that time level too).

Reading (listed with the others in the design notes): LR frames k sit at times
t_k = t_LR0 + k dt_LR; the LR state at a time t between two frames is the
linear interpolation in time of positions and of velocities between the two
frames that bracket it,

    X(t) = X_k + theta (X_{k+1} - X_k),   V(t) = V_k + theta (V_{k+1} - V_k),
    k = floor((t - t_LR0) / dt_LR),       theta = (t - t_LR0) / dt_LR - k,

which is exact for LR particles in uniform motion, and equals frame k at
theta = 0.  HR step n (0-based) advances t_HR0 + n dt_HR to
t_HR0 + (n + 1) dt_HR against the LR state at the step's end.

``lerp_frame`` is the definition in float64.  The library interpolates in
float32; so that its grid keys and neighbour sets stay bit-exact, the
boundary fixes that arithmetic (``lerp_frame_f32``: theta rounded to float32,
then d = fl(X_{k+1} - X_k), fl(theta d), fl(X_k + fl(theta d)), each operation
rounded separately), like the grid keys of the upsampling oracle.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from . import upsample_oracle as O

F32 = np.float32
F64 = np.float64


def bracket(t: float, t_lr0: float, dt_lr: float, n_frames: int) -> Tuple[int, float]:
    """Frame index k and weight theta of the LR state at time t, from frames
    0 .. n_frames - 1 at t_lr0 + k dt_lr (float64).  A time on the last frame
    is (n_frames - 2, 1.0); times outside the frames raise ValueError."""
    s = (F64(t) - F64(t_lr0)) / F64(dt_lr)
    k = math.floor(s)
    theta = float(s - k)
    if k == n_frames - 1 and theta == 0.0 and n_frames >= 2:
        return n_frames - 2, 1.0
    if k < 0 or k > n_frames - 2:
        raise ValueError(f"time {t} outside the LR frames")
    return int(k), theta


def hr_schedule(t_hr0: float, dt_hr: float, n_steps: int, t_lr0: float, dt_lr: float,
                n_frames: int) -> List[Tuple[int, float]]:
    """(k, theta) of the LR state used by HR steps 0 .. n_steps - 1: the state
    at the end of each step, t_hr0 + (n + 1) dt_hr."""
    return [bracket(F64(t_hr0) + F64(n + 1) * F64(dt_hr), t_lr0, dt_lr, n_frames) for n in range(n_steps)]


def lerp_frame(X0, V0, X1, V1, theta: float):
    """The definition: linear interpolation in time, float64 [3, N]."""
    X0, V0, X1, V1 = (np.asarray(a, dtype=F64) for a in (X0, V0, X1, V1))
    th = F64(theta)
    return X0 + th * (X1 - X0), V0 + th * (V1 - V0)


def lerp_frame_f32(X0, V0, X1, V1, theta: float):
    """The boundary's float32 arithmetic of the same interpolation: theta
    rounded to float32, each operation rounded separately.  -> float32 [3, N]."""
    th = F32(theta)
    out = []
    for a0, a1 in ((X0, X1), (V0, V1)):
        a0 = np.asarray(a0, dtype=F32)
        a1 = np.asarray(a1, dtype=F32)
        d = a1 - a0
        p = th * d
        out.append(a0 + p)
    return out[0], out[1]


def rollout_multirate(frames: Sequence[Tuple[np.ndarray, np.ndarray]], t_lr0: float, dt_lr: float,
                      t_hr0: float, n_steps: int, lr_rigid, x0, v0, prm: dict, f32_frames: bool = True):
    """HR rollout with LR frames at their own time step: ``frames`` k = 0 ..
    at t_lr0 + k dt_lr; each HR step of prm["dt"] uses the LR state at its end
    (the float32 contract of the interpolation by default, the float64
    definition with f32_frames=False).  Returns the states [(x^0, v^0), ...]
    (float64) and the schedule."""
    sched = hr_schedule(t_hr0, prm["dt"], n_steps, t_lr0, dt_lr, len(frames))
    states = [(np.asarray(x0, dtype=F64), np.asarray(v0, dtype=F64))]
    lerp = lerp_frame_f32 if f32_frames else lerp_frame
    for k, th in sched:
        X, V = lerp(frames[k][0], frames[k][1], frames[k + 1][0], frames[k + 1][1], th)
        x, v = states[-1]
        o = O.step(X, V, lr_rigid, x, v, prm)
        states.append((o["x"], o["v"]))
    return states, sched
