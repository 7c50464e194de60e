"""Seeded synthetic inputs shared by the oracle tests and the GPU path."""
from .scenes import (FrameKind, KINDS, CONFIG_KIND, make_frame, config_frame,
                     random_grid, batch_mix, poisson_arrivals, scene_planes)

__all__ = ["FrameKind", "KINDS", "CONFIG_KIND", "make_frame", "config_frame",
           "random_grid", "batch_mix", "poisson_arrivals", "scene_planes"]
