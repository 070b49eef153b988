"""Seeded synthetic inputs (geometry, LR trajectories, HR initial states)."""
from .generators import (Scene, build_scene, box_walls, wall, GRAVITY, DT_60, NO_CLIP)  # noqa: F401
from . import configs  # noqa: F401
