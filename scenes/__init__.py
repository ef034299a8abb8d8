"""Seeded synthetic workloads shared by the oracle and the GPU library (inputs only)."""
from .meshgen import (GRAVITY, Scene, batch_scenes, beam_twist, block_rotate, config, cube_compress,
                      cube_jitter, kuhn_grid, permuted, renumbered,
                      serving_scenes)

__all__ = ["GRAVITY", "Scene", "batch_scenes", "beam_twist", "block_rotate", "config", "cube_compress",
           "cube_jitter", "kuhn_grid", "permuted",
           "renumbered", "serving_scenes"]
