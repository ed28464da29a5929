"""Novel-view cameras for a two-plane light field, as pairs of 3x3 homographies.

A camera is ``float32[18]``: the row-major homography ``h_uv`` followed by
``h_st``.  Output pixel ``(i, j)`` (column, row) is sent through each one at
its centre ``(i + 1/2, j + 1/2, 1)``; dividing by the third component gives
the ray's crossing of the uv plane (view grid units: ``u`` = view column,
``v`` = view row) and of the st plane (pixel units of the captured views).

The pinhole model is a camera at eye ``(eu, ev, ez)`` looking along +z,
parallel to both planes: the uv plane sits at z = 0 and the st plane at
z = 1, and ``rho`` is the size of one st pixel in uv units.  The ray through
the eye and the st point ``(rho*s, rho*t, 1)`` meets z = 0 at
``u = (eu - ez*rho*s) / (1 - ez)`` (and likewise for v), so ``h_uv`` is the
affine map ``A`` composed with ``h_st``.
"""

from __future__ import annotations

import numpy as np


def full_frame_st(w: int, h: int, wo: int, ho: int, zoom: float = 1.0,
                  off_x: float = 0.0, off_y: float = 0.0) -> np.ndarray:
    """st homography of a window of the captured image, scaled to wo x ho.

    With ``zoom = 1`` and no offset, output pixel centres land on
    ``s = (i + 1/2) * w / wo - 1/2``: the whole captured frame.
    """
    sx = zoom * w / wo
    sy = zoom * h / ho
    return np.array([[sx, 0.0, off_x - 0.5], [0.0, sy, off_y - 0.5], [0.0, 0.0, 1.0]])


def pinhole_camera(eu: float, ev: float, ez: float, rho: float, h_st: np.ndarray) -> np.ndarray:
    """Camera (float32[18]) for a pinhole at (eu, ev, ez) with the given st window."""
    k = 1.0 / (1.0 - ez)
    A = np.array([[-ez * rho * k, 0.0, eu * k], [0.0, -ez * rho * k, ev * k], [0.0, 0.0, 1.0]])
    h_uv = A @ h_st
    return np.concatenate([h_uv.reshape(-1), h_st.reshape(-1)]).astype(np.float32)


def fixed_uv_camera(u: float, v: float, h_st: np.ndarray) -> np.ndarray:
    """Camera whose rays all cross the uv plane at (u, v) (eye on the uv plane, ez = 0)."""
    h_uv = np.array([[0.0, 0.0, u], [0.0, 0.0, v], [0.0, 0.0, 1.0]])
    return np.concatenate([h_uv.reshape(-1), h_st.reshape(-1)]).astype(np.float32)


def random_fixed_uv_cameras(n: int, na: int, nb: int, w: int, h: int, wo: int, ho: int,
                            seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    st = full_frame_st(w, h, wo, ho)
    cams = [fixed_uv_camera(rng.uniform(0, na - 1), rng.uniform(0, nb - 1), st) for _ in range(n)]
    return np.stack(cams)


def camera_path_orbit(frames: int, na: int, nb: int, w: int, h: int, wo: int, ho: int,
                      radius: float = 6.0, rho: float = 1.0 / 64.0) -> np.ndarray:
    """Circular eye path around the grid centre with a gently varying depth.

    eu = c + r*cos(2 pi k / F), ev = c + r*sin(2 pi k / F),
    ez = -0.5 + 0.25*sin(4 pi k / F), full-frame st window.
    """
    st = full_frame_st(w, h, wo, ho)
    cu, cv = (na - 1) / 2.0, (nb - 1) / 2.0
    cams = []
    for k in range(frames):
        ang = 2.0 * np.pi * k / frames
        eu = cu + radius * np.cos(ang)
        ev = cv + radius * np.sin(ang)
        ez = -0.5 + 0.25 * np.sin(2.0 * ang)
        cams.append(pinhole_camera(eu, ev, ez, rho, st))
    return np.stack(cams)


def random_pinhole_cameras(n: int, na: int, nb: int, w: int, h: int, wo: int, ho: int,
                           seed: int, ez_range=(-1.0, 0.5), zoom_range=(0.5, 1.0),
                           rho: float | None = None) -> np.ndarray:
    """Uniformly random eyes over the grid with random zoomed st windows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if rho is None:
        rho = 1.0 / max(w / max(na - 1, 1), 1.0)
    cams = []
    for _ in range(n):
        eu = rng.uniform(0, na - 1)
        ev = rng.uniform(0, nb - 1)
        ez = rng.uniform(*ez_range)
        zoom = rng.uniform(*zoom_range)
        # Keep the output aspect: the window spans zoom * w columns.
        win_w = zoom * w
        win_h = win_w * ho / wo
        win_h = min(win_h, h)
        ox = rng.uniform(0, max(w - win_w, 0))
        oy = rng.uniform(0, max(h - win_h, 0))
        st = np.array([[win_w / wo, 0.0, ox - 0.5], [0.0, win_h / ho, oy - 0.5], [0.0, 0.0, 1.0]])
        cams.append(pinhole_camera(eu, ev, ez, rho, st))
    return np.stack(cams)


def projective_warp(cams: np.ndarray, px: float, py: float) -> np.ndarray:
    """Compose every camera with the pixel-plane homography ``[[1,0,0],[0,1,0],[px,py,1]]``.

    Both homographies get a non-trivial third row (a tilted image plane), so
    rays go through the divisions of the projective path.  Keep
    ``1 + px*i + py*j`` positive over the output image.
    """
    P = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [px, py, 1.0]])
    out = []
    for c in np.asarray(cams, dtype=np.float64).reshape(-1, 18):
        h_uv = c[:9].reshape(3, 3) @ P
        h_st = c[9:].reshape(3, 3) @ P
        out.append(np.concatenate([h_uv.reshape(-1), h_st.reshape(-1)]))
    return np.stack(out).astype(np.float32)
