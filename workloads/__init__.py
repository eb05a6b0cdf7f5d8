"""Seeded synthetic inputs (water boxes and droplets) shared by the oracle tests
and the GPU path.  Geometry, topology and Maxwell velocities only: nothing in
this package evaluates the potential or advances the dynamics."""
from .water import (WaterSystem, tip3p_params, water_box, water_droplet,
                    droplet_batch, jitter_positions, maxwell_velocities,
                    KB_KCAL, ACC_CONV)

__all__ = ["WaterSystem", "tip3p_params", "water_box", "water_droplet",
           "droplet_batch", "jitter_positions", "maxwell_velocities",
           "KB_KCAL", "ACC_CONV"]
