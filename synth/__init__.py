"""Seeded synthetic inputs shaped like the BAL bundle-adjustment problems.

This package draws random numbers and lays out scenes; it holds none of the
solver's arithmetic (no projection, no Jacobian, no retraction).  Both the
CPU oracle and the GPU library take their inputs from here.
"""
from .ba_scene import (Scene, make_scene, scene_config, SCENE_CONFIGS,  # noqa: F401
                       BetweenDraws, between_draws)
