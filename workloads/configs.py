"""The five workloads the path is measured and parity-tested on.

Each function returns seeded :class:`~workloads.generators.Scene` objects; the
``scale`` argument shrinks particle counts for CPU-side tests while keeping the
geometry and the per-LR HR density.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .generators import Scene, build_scene

# name -> (geometry, n_lr, n_hr, r_lr, steps)
WORKLOADS = {
    "plain":  ("plain", 2048, 65536, 0.02, 10),
    "column": ("column", 16384, 500000, 0.25 / 21.0, 300),
    "drain":  ("drain", 65536, 4194304, 0.0125, 600),
    "diff":   ("heap", 16384, 1048576, 0.008, 40),
}
CONFIG_INDEX = {"plain": 1, "column": 2, "drain": 3, "batched": 4, "diff": 5}


def plain(seed=None) -> Scene:
    """2,048 LR (r = 0.02) on a jittered lattice in a unit box, 65,536 HR, 10 steps."""
    g, nl, nh, r, _ = WORKLOADS["plain"]
    return build_scene(g, nl, nh, seed if seed is not None else 1, r_lr=r, name="plain")


def column(seed=None, scale: float = 1.0) -> Scene:
    """16,384 LR in a 0.5 x 1.0 x 0.5 column, 500,000 HR (about 30 per LR)."""
    g, nl, nh, r, _ = WORKLOADS["column"]
    return build_scene(g, int(nl * scale), int(nh * scale), seed if seed is not None else 2,
                       r_lr=r, name="column")


def drain(seed=None, scale: float = 1.0) -> Scene:
    """65,536 LR (r = 0.0125) and 4,194,304 HR (r_HR = r/4) in a silo with a
    60 degree hopper and an orifice of radius 0.1."""
    g, nl, nh, r, _ = WORKLOADS["drain"]
    return build_scene(g, int(nl * scale), int(nh * scale), seed if seed is not None else 3,
                       r_lr=r, hr_radius_ratio=0.25, name="drain")


def diff(seed=None, n_lr: int = 16384, n_hr: int = 1048576) -> Scene:
    """Heap of 16,384 LR (r = 0.008) and 1,048,576 HR with a seeded target cloud
    (HR start positions plus N(0, 0.05^2) noise, paired by index)."""
    g, _, _, _, _ = WORKLOADS["diff"]
    r = 0.008 if n_lr == 16384 else None
    return build_scene(g, n_lr, n_hr, seed if seed is not None else 5, r_lr=r,
                       with_target=True, name="diff")


def batched(n_scenes: int = 64, seed: int = 4, hr_range=(50_000, 1_000_000),
            lr_per_hr: int = 32) -> List[Scene]:
    """Independent scenes, N_H log-uniform in ``hr_range``, N_L = N_H / 32,
    geometry cycling heap / column / drain; scene s uses SeedSequence([seed, s])."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    lo, hi = math.log(hr_range[0]), math.log(hr_range[1])
    geoms = ("heap", "column", "drain")
    out = []
    for s in range(n_scenes):
        nh = int(round(math.exp(rng.uniform(lo, hi))))
        nl = max(64, nh // lr_per_hr)
        out.append(build_scene(geoms[s % 3], nl, nh, np.random.SeedSequence([seed, s]),
                               name=f"batched{s}_{geoms[s % 3]}"))
    return out
