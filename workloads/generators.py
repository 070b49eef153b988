"""Seeded synthetic inputs for the granular upsampling step.

Input machinery shared by the tests, the bench and the oracle checks: particle
lattices, random placements, prescribed velocity fields for the low-resolution
(LR) guide particles and the wall tables that describe each geometry.  It holds
none of the upsampling arithmetic (kernel weights, Shepard interpolation, the
gravity blend, time integration, the projection of high-resolution particles on
walls); the CPU oracle and the HIP library each implement that on their own.

The paper's scenes (sandcastle, excavator, hourglass, squirrel meshes; Section
5.2) are not available, so analytic geometries stand in for them:

* ``plain``  -- a jittered LR lattice block in a unit box,
* ``column`` -- a 0.5 x 1.0 x 0.5 column that slumps outward,
* ``drain``  -- a silo over a 60 degree hopper and an orifice plate,
* ``heap``   -- a 30 degree cone in a unit box.

They keep the paper's proportions (Section 5.2): LR packed at spacing 2 r_LR
(Section 4 sampling), r_HR / r_LR in 0.2 .. 0.4, dt_HR about 1/60 s.

LR trajectories are a stand-in for the paper's PBD solver (Section 3, Algorithm
1), which keeps particles from interpenetrating.  A stand-in that integrated
gravity without contacts would stack every LR particle into one sheet on the
floor, so the stand-in moves LR particles with volume-preserving prescribed
flows (a slump for column and heap, a converging sink for the drain) plus a
divergence-free smooth field and Gaussian noise.

Arrays handed to the library and the oracle are float32, structure-of-arrays
``[3, N]`` (row 0 = x, row 1 = y, row 2 = z), C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

F32 = np.float32
GRAVITY = (0.0, -9.81, 0.0)  # |g| = 9.81 m/s^2 (Algorithm 1), y up
DT_60 = 1.0 / 60.0           # dt_HR about 0.0167 s (Section 5.2)
NO_CLIP = -3.0e38            # wall clip offset that never deactivates a wall

# Seed stream order for a config: SeedSequence(cfg).spawn(5)
STREAM_JITTER, STREAM_FIELD, STREAM_NOISE, STREAM_HR, STREAM_TARGET = range(5)


# ---------------------------------------------------------------------------
# Wall tables.  A wall is 12 float32: n(3), d, a(3), b, o(3), R.  The plane is
# n.x = d with unit normal n pointing into the admissible side; (a, b) clip the
# wall's extent to a.x >= b; a disc of radius R around o is an open hole
# (R = 0: no hole).  The library and the oracle both read this format.
# ---------------------------------------------------------------------------

def wall(n, d, a=(0.0, 0.0, 0.0), b=NO_CLIP, o=(0.0, 0.0, 0.0), R=0.0) -> np.ndarray:
    n = np.asarray(n, dtype=np.float64)
    n = n / np.linalg.norm(n)
    return np.array([*n, d, *a, b, *o, R], dtype=F32)


def box_walls(lo, hi) -> List[np.ndarray]:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = []
    for ax in range(3):
        n = np.zeros(3)
        n[ax] = 1.0
        out.append(wall(n, lo[ax]))
        out.append(wall(-n, -hi[ax]))
    return out


# ---------------------------------------------------------------------------
# Smooth divergence-free velocity field: F(x) = 1/4 sum_k a_k sin(2 pi f_k d_k.x + phi_k)
# with unit wave directions d_k and unit amplitudes a_k perpendicular to d_k
# (transverse waves are divergence-free), so |F| <= 1 m/s.
# ---------------------------------------------------------------------------

def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@dataclass
class SmoothField:
    d: np.ndarray
    a: np.ndarray
    f: np.ndarray
    phi: np.ndarray

    @classmethod
    def draw(cls, rng: np.random.Generator, n_waves: int = 4) -> "SmoothField":
        d = _unit_vectors(rng, n_waves)
        a = _unit_vectors(rng, n_waves)
        a = a - np.sum(a * d, axis=1, keepdims=True) * d
        a = a / np.linalg.norm(a, axis=1, keepdims=True)
        f = rng.uniform(0.5, 2.0, size=n_waves)
        phi = rng.uniform(0.0, 2.0 * math.pi, size=n_waves)
        return cls(d=d, a=a, f=f, phi=phi)

    def __call__(self, X: np.ndarray) -> np.ndarray:
        """X: (N, 3) float64 -> (N, 3) float64."""
        phase = 2.0 * math.pi * (X @ self.d.T) * self.f + self.phi
        return 0.25 * (np.sin(phase) @ self.a)


# ---------------------------------------------------------------------------
# Geometries: shape membership, LR lattice fill, LR confinement, HR region.
# ---------------------------------------------------------------------------

HOPPER_ANGLE = math.radians(60.0)


@dataclass
class Geometry:
    name: str
    lo: np.ndarray
    hi: np.ndarray
    walls: List[np.ndarray]
    fill_lo: np.ndarray          # bounding box of the region LR are filled into
    fill_hi: np.ndarray
    params: dict = field(default_factory=dict)

    # -- shape membership (for lattice fill and HR placement), X: (N,3) --
    def inside(self, X: np.ndarray, margin: float) -> np.ndarray:
        lo, hi = self.fill_lo + margin, self.fill_hi - margin
        ok = np.all((X >= lo) & (X <= hi), axis=1)
        if self.name == "heap":
            c = self.params["center"]
            rad = np.hypot(X[:, 0] - c[0], X[:, 2] - c[2])
            ok &= X[:, 1] <= (self.params["base_radius"] - rad) * math.tan(math.radians(30.0)) - margin
        elif self.name == "drain":
            y0, th = self.params["plate_y"], self.params["throat"]
            hw = th + (X[:, 1] - y0) / math.tan(HOPPER_ANGLE) - margin / math.sin(HOPPER_ANGLE)
            ok &= X[:, 1] >= y0 + margin
            ok &= (np.abs(X[:, 0] - 0.5) <= hw) & (np.abs(X[:, 2] - 0.5) <= hw)
        return ok

    # -- LR confinement of the stand-in trajectory (not the HR wall step) --
    def confine(self, Xn: np.ndarray, Xo: np.ndarray, r: float) -> np.ndarray:
        Xn = np.clip(Xn, self.lo + r, self.hi - r)
        if self.name == "drain":
            y0, th, R = self.params["plate_y"], self.params["throat"], self.params["orifice"]
            above = Xo[:, 1] >= y0
            rho = np.hypot(Xn[:, 0] - 0.5, Xn[:, 2] - 0.5)
            blocked = above & (Xn[:, 1] < y0 + r) & (rho > R - r)
            Xn[blocked, 1] = y0 + r
            inh = Xn[:, 1] >= y0
            hw = th + (Xn[:, 1] - y0) / math.tan(HOPPER_ANGLE) - r
            hw = np.maximum(hw, 0.0)
            for ax in (0, 2):
                off = Xn[:, ax] - 0.5
                Xn[inh, ax] = 0.5 + np.clip(off[inh], -hw[inh], hw[inh])
        return Xn


def make_geometry(name: str, with_walls: bool = True) -> Geometry:
    if name == "plain":
        lo, hi = np.zeros(3), np.ones(3)
        g = Geometry(name, lo, hi, box_walls(lo, hi) if with_walls else [],
                     np.array([0.18, 0.0, 0.18]), np.array([0.82, 0.32, 0.82]))
    elif name == "column":
        lo, hi = np.zeros(3), np.array([2.0, 1.5, 2.0])
        g = Geometry(name, lo, hi, box_walls(lo, hi) if with_walls else [],
                     np.array([0.75, 0.0, 0.75]), np.array([1.25, 1.0, 1.25]),
                     {"center": np.array([1.0, 0.0, 1.0]), "slump": 0.15})
    elif name == "heap":
        lo, hi = np.zeros(3), np.ones(3)
        br = 0.49
        g = Geometry(name, lo, hi, box_walls(lo, hi) if with_walls else [],
                     np.array([0.5 - br, 0.0, 0.5 - br]),
                     np.array([0.5 + br, br * math.tan(math.radians(30.0)), 0.5 + br]),
                     {"center": np.array([0.5, 0.0, 0.5]), "base_radius": br, "slump": 0.1})
    elif name == "drain":
        lo, hi = np.zeros(3), np.array([1.0, 2.4, 1.0])
        y0, th, R = 0.6, 0.1, 0.1
        walls = box_walls(lo, hi) if with_walls else []
        if with_walls:
            o = (0.5, y0, 0.5)
            walls.append(wall((0.0, 1.0, 0.0), y0, o=o, R=R))         # orifice plate
            s, c = math.sin(HOPPER_ANGLE), math.cos(HOPPER_ANGLE)
            for ax, sign in ((0, 1.0), (0, -1.0), (2, 1.0), (2, -1.0)):
                n = np.zeros(3)
                n[ax] = -sign * s
                n[1] = c
                edge = np.array([0.5, y0, 0.5])
                edge[ax] = 0.5 + sign * th
                walls.append(wall(n, float(n @ edge), a=(0.0, 1.0, 0.0), b=y0))
        g = Geometry(name, lo, hi, walls, np.array([0.0, y0, 0.0]), np.array([1.0, 2.4, 1.0]),
                     {"plate_y": y0, "throat": th, "orifice": R, "o": np.array([0.5, y0, 0.5]),
                      "sink_q": 0.0225, "sink_cap": 3.0})
    else:
        raise ValueError(f"unknown geometry {name!r}")
    return g


def fill_lattice(geom: Geometry, r: float, n: int, rng: np.random.Generator,
                 jitter: float = 0.1) -> np.ndarray:
    """LR sites on a cubic lattice of spacing 2r inside the shape, filled
    bottom-up (by layer) to n sites, then jittered by U(+-jitter*r). -> (N,3)."""
    sp = 2.0 * r
    axes = [np.arange(geom.fill_lo[a] + r, geom.fill_hi[a] - r + 1e-9, sp) for a in range(3)]
    gx, gy, gz = np.meshgrid(*axes, indexing="ij")
    P = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    P = P[geom.inside(P, 0.5 * r)]
    order = np.lexsort((P[:, 0], P[:, 2], np.round(P[:, 1] / sp).astype(np.int64)))
    P = P[order]
    if P.shape[0] < n:
        raise ValueError(f"{geom.name}: lattice holds {P.shape[0]} sites < {n}")
    P = P[:n].copy()
    P += rng.uniform(-jitter * r, jitter * r, size=P.shape)
    return P


def place_hr(geom: Geometry, lr: np.ndarray, r_lr: float, n: int,
             rng: np.random.Generator, cell: float) -> np.ndarray:
    """n HR positions uniform in the LR-occupied region (the shape below the top of
    the LR fill), emitted in grid-cell order (cells of side ``cell``) like a
    per-cell volume sampler.  -> (n,3)."""
    lo = geom.fill_lo.copy()
    hi = geom.fill_hi.copy()
    top = float(lr[:, 1].max()) + r_lr
    hi[1] = min(hi[1], top)
    chunks, have = [], 0
    while have < n:
        m = max(1024, int(1.3 * (n - have)) + 1024)
        C = rng.uniform(lo, hi, size=(m, 3))
        C = C[geom.inside(C, 0.0)]
        chunks.append(C)
        have += C.shape[0]
    P = np.concatenate(chunks)[:n]
    c = np.floor((P - lo) / cell).astype(np.int64)
    dims = c.max(axis=0) + 1
    key = (c[:, 2] * dims[1] + c[:, 1]) * dims[0] + c[:, 0]
    return P[np.argsort(key, kind="stable")]


def volume_candidates(geometry: str, n: int, seed, top: Optional[float] = None) -> np.ndarray:
    """n random candidate positions uniform inside a geometry's fill region
    (below ``top`` if given), float32 [3, n]: the random input of the volume
    sampling of initial states.  -> also the box (lo, hi) they lie in."""
    geom = make_geometry(geometry, with_walls=False)
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    lo = geom.fill_lo.copy()
    hi = geom.fill_hi.copy()
    if top is not None:
        hi[1] = min(hi[1], top)
    chunks, have = [], 0
    while have < n:
        m = max(1024, int(1.3 * (n - have)) + 1024)
        C = rng.uniform(lo, hi, size=(m, 3))
        C = C[geom.inside(C, 0.0)]
        chunks.append(C)
        have += C.shape[0]
    P = np.concatenate(chunks)[:n]
    return np.ascontiguousarray(P.T, dtype=F32), lo.astype(F32), hi.astype(F32)


def box_candidates(lo, hi, n: int, seed) -> np.ndarray:
    """n random candidate positions uniform in the box [lo, hi], float32
    [3, n]: the random input of the volume sampling for a box-shaped region."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    P = rng.uniform(np.asarray(lo, float), np.asarray(hi, float), size=(n, 3))
    return np.ascontiguousarray(P.T, dtype=F32)


# ---------------------------------------------------------------------------
# LR trajectory stand-in.
# ---------------------------------------------------------------------------

class LRTrajectory:
    """Frames t = 1, 2, ... of LR positions and velocities (float32 SoA), one
    per LR time step ``dt`` (frame 0 is the initial state at rest).

    V^{t+1} = flow(X^t) + F(X^t) * field_gain + eta,   eta ~ N(0, sigma^2) per component,
    X^{t+1} = confine(X^t + dt V^{t+1}).
    Rigid LR particles (boundary samples) keep their position and zero velocity.
    """

    def __init__(self, geom: Geometry, X0: np.ndarray, rigid: np.ndarray, r: float, dt: float,
                 fld: SmoothField, noise_rng: np.random.Generator, flow: str,
                 field_gain: float, sigma: float = 0.05, recycle_rng=None):
        self.geom, self.r, self.dt = geom, r, dt
        self.X = X0.astype(np.float64).copy()
        self.X0 = self.X.copy()
        self.rigid = rigid.astype(bool)
        self.field, self.rng, self.flow = fld, noise_rng, flow
        self.gain, self.sigma = field_gain, sigma
        self.recycle_rng = recycle_rng
        self.frames: List[Tuple[np.ndarray, np.ndarray]] = []

    def _flow(self, X: np.ndarray) -> np.ndarray:
        g = self.geom
        if self.flow == "none":
            return np.zeros_like(X)
        if self.flow == "slump":
            c = g.params["slump"]
            ctr = g.params["center"]
            return c * np.stack([X[:, 0] - ctr[0], -2.0 * X[:, 1], X[:, 2] - ctr[2]], axis=1)
        if self.flow == "sink":
            o = g.params["o"]
            D = X - o
            rho = np.maximum(np.linalg.norm(D, axis=1), 1e-3)
            speed = np.minimum(g.params["sink_cap"], g.params["sink_q"] / rho ** 2)
            V = -D / rho[:, None] * speed[:, None]
            below = X[:, 1] < g.params["plate_y"]
            V[below] = (0.0, -2.0, 0.0)
            return V
        raise ValueError(self.flow)

    def _advance(self) -> None:
        X = self.X
        V = self._flow(X) + self.gain * self.field(X) + self.rng.normal(0.0, self.sigma, size=X.shape)
        V[self.rigid] = 0.0
        Xn = self.geom.confine(X + self.dt * V, X, self.r)
        Xn[self.rigid] = X[self.rigid]
        if self.flow == "sink":
            out = Xn[:, 1] < self.geom.params["plate_y"] - 0.05
            k = int(out.sum())
            if k:
                Xn[out] = self.recycle_rng.uniform((0.05, 2.15, 0.05), (0.95, 2.3, 0.95), size=(k, 3))
                V[out] = (0.0, -1.0, 0.0)
        self.X = Xn
        self.frames.append((np.ascontiguousarray(Xn.T, dtype=F32),
                            np.ascontiguousarray(V.T, dtype=F32)))

    def frame(self, t: int) -> Tuple[np.ndarray, np.ndarray]:
        """LR (X, V) after t steps, each float32 [3, N_L] (t = 0: the initial
        positions at rest)."""
        if t < 0:
            raise ValueError("frames start at t = 0")
        if t == 0:
            return (np.ascontiguousarray(self.X0.T, dtype=F32),
                    np.zeros((3, self.X0.shape[0]), dtype=F32))
        while len(self.frames) < t:
            self._advance()
        return self.frames[t - 1]


# ---------------------------------------------------------------------------
# Scenes.
# ---------------------------------------------------------------------------

@dataclass
class Scene:
    name: str
    r_lr: float
    r_hr: float
    dt: float
    g: np.ndarray
    domain_lo: np.ndarray
    domain_hi: np.ndarray
    walls: np.ndarray            # (n_walls, 12) float32
    lr_x0: np.ndarray            # [3, N_L] float32
    lr_rigid: np.ndarray         # [N_L] uint8, 1 = rigid/boundary sample
    hr_x0: np.ndarray            # [3, N_H] float32
    hr_v0: np.ndarray            # [3, N_H] float32
    traj: LRTrajectory
    target: Optional[np.ndarray] = None   # [3, N_H] float32 (differentiation config)
    c1: float = 512.0 / 729.0
    c2: float = 0.6
    dt_lr: Optional[float] = None         # LR frame interval (None: one LR frame per HR step, dt)

    @property
    def n_lr(self) -> int:
        return self.lr_x0.shape[1]

    @property
    def n_hr(self) -> int:
        return self.hr_x0.shape[1]

    @property
    def box_length(self) -> float:
        return float(np.max(self.domain_hi - self.domain_lo))

    def lr_frame(self, t: int) -> Tuple[np.ndarray, np.ndarray]:
        return self.traj.frame(t)

    def params(self) -> dict:
        return dict(r_lr=self.r_lr, r_hr=self.r_hr, dt=self.dt, g=self.g, c1=self.c1, c2=self.c2,
                    domain_lo=self.domain_lo, domain_hi=self.domain_hi, walls=self.walls)


def _seeds(seed) -> List[np.random.SeedSequence]:
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return ss.spawn(5)


FLOWS = {"plain": ("none", 1.0), "column": ("slump", 0.25), "heap": ("slump", 0.25),
         "drain": ("sink", 0.25)}


def build_scene(geometry: str, n_lr: int, n_hr: int, seed, r_lr: Optional[float] = None,
                dt: float = DT_60, gravity: Sequence[float] = GRAVITY, with_walls: bool = True,
                rigid_floor: bool = False, hr_radius_ratio: Optional[float] = None,
                with_target: bool = False, name: Optional[str] = None,
                dt_lr: Optional[float] = None) -> Scene:
    """Build a seeded scene.  ``r_lr`` defaults to the radius whose lattice fill
    of the geometry's nominal volume holds about ``n_lr`` sites.  ``dt_lr``:
    the LR frames' own time step (Section 5.2: 0.005 s) when the LR
    trajectory is sub-stepped against the HR step ``dt``."""
    geom = make_geometry(geometry, with_walls)
    sj, sf, sn, sh, st = (np.random.default_rng(s) for s in _seeds(seed))
    auto = r_lr is None
    if auto:
        r_lr = auto_radius(geometry, n_lr)
    while True:
        try:
            X = fill_lattice(geom, r_lr, n_lr, sj)   # draws nothing when it fails
            break
        except ValueError:
            if not auto:
                raise
            r_lr *= 0.97   # small counts: the lattice quantises below the nominal fill
    rigid = np.zeros(n_lr, dtype=np.uint8)
    if rigid_floor:
        # boundary sampling of the floor as static rigid LR particles (Section 3)
        span_lo, span_hi = geom.fill_lo + r_lr, geom.fill_hi - r_lr
        xs = np.arange(span_lo[0], span_hi[0] + 1e-9, 2 * r_lr)
        zs = np.arange(span_lo[2], span_hi[2] + 1e-9, 2 * r_lr)
        gx, gz = np.meshgrid(xs, zs, indexing="ij")
        F = np.stack([gx.ravel(), np.full(gx.size, geom.fill_lo[1] - r_lr), gz.ravel()], axis=1)
        X = np.concatenate([X, F])
        rigid = np.concatenate([rigid, np.ones(F.shape[0], dtype=np.uint8)])
    ratio = hr_radius_ratio if hr_radius_ratio is not None else (n_lr / n_hr) ** (1.0 / 3.0)
    r_hr = r_lr * ratio
    P = place_hr(geom, X[rigid == 0], r_lr, n_hr, sh, cell=2.0 * r_lr)
    flow, gain = FLOWS[geometry]
    traj = LRTrajectory(geom, X, rigid, r_lr, dt if dt_lr is None else dt_lr, SmoothField.draw(sf), sn, flow,
                        gain, recycle_rng=np.random.default_rng(sn.integers(1 << 62)))
    target = None
    if with_target:
        target = np.ascontiguousarray((P + st.normal(0.0, 0.05, size=P.shape)).T, dtype=F32)
    walls = np.stack(geom.walls).astype(F32) if geom.walls else np.zeros((0, 12), F32)
    return Scene(name=name or geometry, r_lr=float(F32(r_lr)), r_hr=float(F32(r_hr)),
                 dt=float(F32(dt)), g=np.asarray(gravity, dtype=F32),
                 domain_lo=geom.lo.astype(F32), domain_hi=geom.hi.astype(F32), walls=walls,
                 lr_x0=np.ascontiguousarray(X.T, dtype=F32), lr_rigid=rigid,
                 hr_x0=np.ascontiguousarray(P.T, dtype=F32),
                 hr_v0=np.zeros((3, n_hr), dtype=F32), traj=traj, target=target,
                 dt_lr=None if dt_lr is None else float(dt_lr))


NOMINAL_FILL_VOLUME = {
    "plain": 0.64 * 0.32 * 0.64,
    "column": 0.5 * 1.0 * 0.5,
    "heap": math.pi * 0.48 ** 2 * 0.48 * math.tan(math.radians(30.0)) / 3.0,
    "drain": 0.28 + 1.0 * 0.6,   # hopper frustum plus 0.6 m of silo
}


def auto_radius(geometry: str, n_lr: int) -> float:
    """Radius whose 2r lattice packs n_lr sites into 75% of the nominal fill volume."""
    return 0.5 * (0.75 * NOMINAL_FILL_VOLUME[geometry] / n_lr) ** (1.0 / 3.0)
