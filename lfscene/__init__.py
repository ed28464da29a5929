"""Seeded synthetic light-field scenes, camera paths and encoding settings.

This package is the only code shared by the CPU oracle (``oracle/``) and the
GPU library (``paper_1902_09396_amd``).  It produces inputs only: images,
camera homographies and parameter dictionaries.  It holds none of the codec's
arithmetic (no colour transform, hierarchy, motion compensation, quantisation,
bit packing, decoding or blending).

The Stanford light-field archive scenes that the paper measures on (Evaluation
section) are not available here; the scenes below are procedural stand-ins
with the same grid shapes, 8-bit RGB samples and view-to-view disparities.
"""

from .scene import make_lf, make_scene_layers, perlin_fbm
from .cameras import (
    full_frame_st,
    pinhole_camera,
    camera_path_orbit,
    random_fixed_uv_cameras,
    random_pinhole_cameras,
    projective_warp,
)
from .configs import CONFIGS, get_config, make_views

__all__ = [
    "make_lf",
    "make_scene_layers",
    "perlin_fbm",
    "full_frame_st",
    "pinhole_camera",
    "camera_path_orbit",
    "random_fixed_uv_cameras",
    "random_pinhole_cameras",
    "projective_warp",
    "CONFIGS",
    "get_config",
    "make_views",
]
