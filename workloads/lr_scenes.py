"""Seeded initial states of LR particle systems for the LR simulation step
(Section 3, Algorithm 1): static boundary samples, granular material and rigid
bodies.

Inputs only: positions, velocities, particle types, inverse masses and the
rigid bodies' rest offsets (each particle's position minus its body's mean).
None of the method's arithmetic is here; both the oracle and the GPU path
take these arrays as they are.

* ``column_collapse``: the column workload's 16,384 granular LR particles
  (r = 0.25/21, a 0.5 x 1.0 x 0.5 column on a jittered lattice of spacing 2r)
  at rest on a floor of static samples; with no walls the column slumps.
* ``impact``: a granular bed in a box of static samples, hit by a rigid
  ellipsoid thrown into it while a rigid cube falls beside it (the shape of
  the paper's rigid-body scenes, with analytic shapes for its meshes).
* ``drain_flow``: the drain workload's 65,536 granular LR (r = 0.0125) in
  its silo, standing on static samples of the 60 degree hopper, of the
  orifice plate's corners, of the silo walls and of a floor under the
  orifice, so that the sand runs out through the orifice.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from .generators import HOPPER_ANGLE, fill_lattice, make_geometry

GRANULAR = -1
STATIC = -2
F32 = np.float32


@dataclass
class LRScene:
    name: str
    r: float
    dt: float
    g: tuple
    domain_lo: np.ndarray
    domain_hi: np.ndarray
    ground_y: float
    x: np.ndarray        # [3, n] float32
    v: np.ndarray        # [3, n] float32
    body: np.ndarray     # [n] int32: GRANULAR, STATIC or rigid body id
    inv_m: np.ndarray    # [n] float32 (0 for static)
    rest: np.ndarray     # [3, n] float32 rest offsets of rigid particles (0 otherwise)

    @property
    def n(self) -> int:
        return self.x.shape[1]

    @property
    def n_bodies(self) -> int:
        return int(self.body.max(initial=-1)) + 1

    @property
    def lr_rigid(self) -> np.ndarray:
        """uint8 [n]: 1 for static and rigid particles (the upsampling's
        rigid flag), 0 for granular."""
        return (self.body != GRANULAR).astype(np.uint8)


def _lattice(lo, hi, sp) -> np.ndarray:
    axes = [np.arange(lo[a], hi[a] + 1e-9, sp) if hi[a] > lo[a] else np.array([lo[a]]) for a in range(3)]
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.ravel() for a in g], axis=1)


def _assemble(name, r, dt, g, lo, hi, ground_y, parts: List[tuple]) -> LRScene:
    """parts: (positions (N,3), velocities (N,3) or None, body id, inverse mass)."""
    xs, vs, bs, ms, rs = [], [], [], [], []
    for P, V, b, w in parts:
        P = np.asarray(P, dtype=np.float64)
        xs.append(P)
        vs.append(np.zeros_like(P) if V is None else np.broadcast_to(np.asarray(V, float), P.shape))
        bs.append(np.full(P.shape[0], b, dtype=np.int32))
        ms.append(np.full(P.shape[0], 0.0 if b == STATIC else w))
        rs.append(P - P.mean(axis=0) if b >= 0 else np.zeros_like(P))
    cat = lambda a: np.ascontiguousarray(np.concatenate(a).T, dtype=F32)
    return LRScene(name, float(r), float(dt), tuple(g), np.asarray(lo, F32), np.asarray(hi, F32), float(ground_y),
                   cat(xs), cat(vs), np.concatenate(bs), np.concatenate(ms).astype(F32), cat(rs))


def column_collapse(scale: float = 1.0, seed: int = 2, dt: float = 0.005) -> LRScene:
    """16,384 * scale granular particles of the column workload at rest on a
    static floor (centres at y = -r, spacing 2r) that reaches 0.75 m beyond
    the column on every side."""
    r = 0.25 / 21.0
    rng = np.random.default_rng(np.random.SeedSequence([seed, 11]))
    geom = make_geometry("column", with_walls=False)
    sand = fill_lattice(geom, r, int(16384 * scale), rng)
    c = geom.params["center"]
    reach = 0.25 + 0.75 * min(1.0, max(scale, 0.2) ** 0.5)
    floor = _lattice((c[0] - reach, -r, c[2] - reach), (c[0] + reach, -r, c[2] + reach), 2 * r)
    lo = (0.0, -4 * r, 0.0)
    hi = (2.0, 1.5, 2.0)
    return _assemble("column_collapse", r, dt, (0.0, -9.81, 0.0), lo, hi, 0.0,
                     [(floor, None, STATIC, 0.0), (sand, None, GRANULAR, 1.0)])


def impact(small: bool = False, seed: int = 6, dt: float = 0.005) -> LRScene:
    """A granular bed in an open box of static samples (floor and four walls,
    spacing 2r), a rigid ellipsoid thrown into it and a rigid cube dropped
    beside it.  The bodies are 2.5 times denser than the sand."""
    r = 0.01
    rng = np.random.default_rng(np.random.SeedSequence([seed, 12]))
    L = 0.4 if small else 0.8
    depth = 0.08 if small else 0.16
    H = depth + 0.1
    sp = 2 * r
    floor = _lattice((-r, -r, -r), (L + r, -r, L + r), sp)
    walls = []
    for a, pos in ((0, -r), (0, L + r), (2, -r), (2, L + r)):
        lo_w = [-r, r, -r]
        hi_w = [L + r, H, L + r]
        lo_w[a] = hi_w[a] = pos
        walls.append(_lattice(lo_w, hi_w, sp))
    boundary = np.unique(np.round(np.concatenate([floor] + walls), 9), axis=0)
    sand = _lattice((r, r, r), (L - r, depth, L - r), sp)
    sand = sand + rng.uniform(-0.1 * r, 0.1 * r, sand.shape)
    # ellipsoid (semi-axes a, b, b) on the lattice, thrown down and sideways
    a_ax, b_ax = (0.06, 0.04) if small else (0.12, 0.08)
    E = _lattice((-a_ax, -b_ax, -b_ax), (a_ax, b_ax, b_ax), sp)
    E = E - E.mean(axis=0)
    E = E[(E[:, 0] / a_ax) ** 2 + (E[:, 1] / b_ax) ** 2 + (E[:, 2] / b_ax) ** 2 <= 1.0]
    e_c = np.array([0.3 * L, depth + b_ax + 3 * r, 0.5 * L])
    cube_n = 4 if small else 6
    C = _lattice((0, 0, 0), ((cube_n - 1) * sp,) * 3, sp)
    C = C - C.mean(axis=0)
    c_c = np.array([0.75 * L, depth + 0.5 * cube_n * sp + 0.02, 0.5 * L])
    lo = (-3 * r, -3 * r, -3 * r)
    hi = (L + 3 * r, H + 0.3, L + 3 * r)
    return _assemble("impact_small" if small else "impact", r, dt, (0.0, -9.81, 0.0), lo, hi, 0.0,
                     [(boundary, None, STATIC, 0.0), (sand, None, GRANULAR, 1.0),
                      (E + e_c, (2.0, -2.5, 0.0), 0, 0.4), (C + c_c, (0.0, -1.0, 0.0), 1, 0.4)])


def drain_flow(scale: float = 1.0, seed: int = 3, dt: float = 0.0025) -> LRScene:
    """The drain workload's granular LR fill (65,536 * scale particles,
    jittered lattice, at rest) on static samples of its boundary: the four
    hopper planes from the orifice plate's throat up to the silo walls, the
    plate's corners around the orifice (radius 0.1), the silo walls above
    the hopper and below the plate, and a floor at y = 0.  Every static
    sample sits r behind the surface it represents, at spacing 2r.  The time
    step is the default 0.005 s limited by the CFL condition (Section 5.2):
    sand falling the 0.6 m below the plate reaches about 3.4 m/s, so a step
    of 0.0025 s moves it at most about r."""
    r = 0.0125
    rng = np.random.default_rng(np.random.SeedSequence([seed, 13]))
    geom = make_geometry("drain", with_walls=False)
    y0, th, R = geom.params["plate_y"], geom.params["throat"], geom.params["orifice"]
    sand = fill_lattice(geom, r, int(65536 * scale), rng)
    sp = 2 * r
    ta = math.tan(HOPPER_ANGLE)
    s_, c_ = math.sin(HOPPER_ANGLE), math.cos(HOPPER_ANGLE)
    y_top = y0 + (0.5 - th) * ta           # where the hopper meets the silo walls
    top = float(sand[:, 1].max()) + 4 * r
    parts = []
    # hopper planes: along the slope from the throat edge, across within the
    # frustum's half-width at that height; offset r along the outward normal
    t_max = (y_top - y0) / s_
    for ax in (0, 2):
        other = 2 - ax
        for sign in (1.0, -1.0):
            for t in np.arange(0.0, t_max + 1e-9, sp):
                y = y0 + s_ * t
                hw = th + (y - y0) / ta
                u = np.arange(0.5 - hw, 0.5 + hw + 1e-9, sp)
                P = np.zeros((u.size, 3))
                P[:, ax] = 0.5 + sign * (th + c_ * t) + sign * s_ * r
                P[:, 1] = y - c_ * r
                P[:, other] = u
                parts.append(P)
    # orifice plate: the corners of the throat square outside the hole
    g = np.arange(0.5 - th, 0.5 + th + 1e-9, sp)
    gx, gz = np.meshgrid(g, g, indexing="ij")
    keep = np.hypot(gx - 0.5, gz - 0.5) >= R + r
    parts.append(np.stack([gx[keep], np.full(keep.sum(), y0 - r), gz[keep]], axis=1))
    # silo walls above the hopper and below the plate, and the floor
    ys = np.concatenate([np.arange(-r, y0 + 1e-9, sp), np.arange(y_top - r, top + 1e-9, sp)])
    w = np.arange(0.0, 1.0 + 1e-9, sp)
    for ax in (0, 2):
        other = 2 - ax
        for pos in (-r, 1.0 + r):
            A, Y = np.meshgrid(w, ys, indexing="ij")
            P = np.zeros((A.size, 3))
            P[:, ax] = pos
            P[:, 1] = Y.ravel()
            P[:, other] = A.ravel()
            parts.append(P)
    F = _lattice((0.0, -r, 0.0), (1.0, -r, 1.0), sp)
    parts.append(F)
    boundary = np.unique(np.round(np.concatenate(parts), 9), axis=0)
    lo = (-4 * r, -4 * r, -4 * r)
    hi = (1.0 + 4 * r, 2.4 + 4 * r, 1.0 + 4 * r)
    return _assemble("drain_flow", r, dt, (0.0, -9.81, 0.0), lo, hi, 0.0,
                     [(boundary, None, STATIC, 0.0), (sand, None, GRANULAR, 1.0)])
