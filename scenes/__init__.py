"""Seeded synthetic workloads shared by the oracle and the GPU library (inputs only)."""
from .meshgen import GRAVITY, Scene, beam_twist, config, cube_compress, cube_jitter, kuhn_grid

__all__ = ["GRAVITY", "Scene", "beam_twist", "config", "cube_compress", "cube_jitter", "kuhn_grid"]
