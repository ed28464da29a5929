"""Workload shapes: light-field scenes, encoding settings and camera sets.

Encoding settings follow the parameters the paper names for its encoder
(tree height, block size, the two block thresholds and the search window;
Compressing HMLFC tree section) plus a per-level quantisation step and
quarter-pel motion vectors.
"""

from __future__ import annotations

import copy

import numpy as np

from .cameras import camera_path_orbit, random_fixed_uv_cameras, random_pinhole_cameras


def _enc(levels, block, step, win, t_ref=0, t_pred=0, subpel=True, zero_phase=False, no_mc=False):
    return {
        "levels": levels,
        "block": block,
        "step": [step] * levels if np.isscalar(step) else list(step),
        "win": [win] * levels if np.isscalar(win) else list(win),
        "t_ref": [t_ref] * levels if np.isscalar(t_ref) else list(t_ref),
        "t_pred": [t_pred] * levels if np.isscalar(t_pred) else list(t_pred),
        "subpel": bool(subpel),
        "zero_phase": bool(zero_phase),
        "no_mc": bool(no_mc),
    }


CONFIGS = {
    # 8x8 views of 64x64, three planes (flat background + two rectangles/discs),
    # disparity in [-2, 2] px, 2-level tree, 8x8 blocks, step 4.
    "tiny": {
        "lf": {"na": 8, "nb": 8, "h": 64, "w": 64, "seed": 11,
               "spec": {"planes": 2, "dmax": 2.0, "background": "flat", "period": 32.0}},
        "enc": _enc(levels=2, block=8, step=4, win=4),
        "views": {"kind": "fixed_uv", "n": 4, "wo": 64, "ho": 64, "seed": 12},
    },
    # 17x17 views of 512x512, six planes in front of a terrain, disparity in
    # [-4, 4] px, 4-level tree, 16x16 blocks, step 4, 120-frame orbit path.
    "path512": {
        "lf": {"na": 17, "nb": 17, "h": 512, "w": 512, "seed": 21,
               "spec": {"planes": 6, "dmax": 4.0, "background": "terrain", "period": 64.0}},
        "enc": _enc(levels=4, block=16, step=4, win=8),
        "views": {"kind": "orbit", "n": 120, "wo": 512, "ho": 512},
    },
    # 32x32 views of 1024x1024, 16 shaded layers, disparity in [-8, 8] px,
    # 5-level tree, batches of 32 random 1920x1080 cameras.
    "batch1080": {
        "lf": {"na": 32, "nb": 32, "h": 1024, "w": 1024, "seed": 31,
               "spec": {"planes": 16, "dmax": 8.0, "background": "flat", "shading": True,
                        "period": 48.0}},
        "enc": _enc(levels=5, block=16, step=4, win=8),
        "views": {"kind": "random_pinhole", "n": 32, "wo": 1920, "ho": 1080, "seed": 32},
    },
    # Differentiation workload: the 17x17x512^2 light field, 16 orbit views.
    "grad512": {
        "lf": {"na": 17, "nb": 17, "h": 512, "w": 512, "seed": 21,
               "spec": {"planes": 6, "dmax": 4.0, "background": "terrain", "period": 64.0}},
        "enc": _enc(levels=4, block=16, step=4, win=8),
        "views": {"kind": "orbit", "n": 16, "wo": 512, "ho": 512},
    },
    # Serving light fields (the other two resident ones are path512 and batch1080).
    "serve256": {
        "lf": {"na": 9, "nb": 9, "h": 256, "w": 256, "seed": 51,
               "spec": {"planes": 4, "dmax": 4.0, "background": "flat", "period": 24.0}},
        "enc": _enc(levels=3, block=16, step=4, win=8),
        "views": {"kind": "random_pinhole", "n": 8, "wo": 256, "ho": 256, "seed": 52},
    },
    "serve1024": {
        "lf": {"na": 17, "nb": 17, "h": 1024, "w": 1024, "seed": 53,
               "spec": {"planes": 8, "dmax": 6.0, "background": "terrain", "period": 48.0}},
        "enc": _enc(levels=4, block=16, step=4, win=8),
        "views": {"kind": "random_pinhole", "n": 8, "wo": 1024, "ho": 1024, "seed": 54},
    },
}


def get_config(name: str, **overrides) -> dict:
    cfg = copy.deepcopy(CONFIGS[name])
    for k, v in overrides.items():
        if k in cfg["enc"]:
            L = cfg["enc"]["levels"]
            per_level = k in ("step", "win", "t_ref", "t_pred")
            cfg["enc"][k] = [v] * L if (per_level and np.isscalar(v)) else v
        else:
            cfg[k] = v
    return cfg


def make_views(cfg: dict) -> np.ndarray:
    """Camera array float32[V][18] for a config's view set."""
    lf, vw = cfg["lf"], cfg["views"]
    na, nb, w, h = lf["na"], lf["nb"], lf["w"], lf["h"]
    kind = vw["kind"]
    if kind == "fixed_uv":
        return random_fixed_uv_cameras(vw["n"], na, nb, w, h, vw["wo"], vw["ho"], vw["seed"])
    if kind == "orbit":
        radius = min(6.0, (na - 1) / 2.0 - 0.5)
        return camera_path_orbit(vw["n"], na, nb, w, h, vw["wo"], vw["ho"], radius=radius)
    if kind == "random_pinhole":
        return random_pinhole_cameras(vw["n"], na, nb, w, h, vw["wo"], vw["ho"], vw["seed"])
    raise ValueError(kind)
