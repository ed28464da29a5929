"""Procedural two-plane light fields built from textured layers.

A light field is returned as ``uint8[Nb][Na][H][W][3]``: ``b`` is the view row
(v), ``a`` the view column (u), then the image row (t, ``y``), the image
column (s, ``x``) and RGB.  This is the 4D grid of 2D views described in the
paper's Light Field Rendering background section.

View ``(b, a)`` shows, at pixel ``(x, y)``, the front-most layer whose support
contains the source point ``(x - d*(a - ac), y - d*(b - bc))``, where
``(ac, bc)`` is the grid centre and ``d`` the layer's disparity in pixels
between adjacent views.  Layers are composited back to front in order of
increasing disparity; a full-frame background (flat or terrain) sits behind
them.  Textures are Perlin gradient-noise fBm (Perlin, "Improving Noise",
SIGGRAPH 2002), rendered once on an integer lattice with a margin and sampled
bilinearly at the sub-pixel source positions.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _perm_table(rng: np.random.Generator) -> np.ndarray:
    p = rng.permutation(256).astype(np.int64)
    return np.concatenate([p, p])


def _grad2(h, x, y):
    # Eight gradient directions: (+-1,+-1), (+-1,0), (0,+-1).
    h = h & 7
    gx = np.where(h < 4, np.where(h & 1, -1.0, 1.0), np.where(h < 6, np.where(h & 1, -1.0, 1.0), 0.0))
    gy = np.where(h < 4, np.where(h & 2, -1.0, 1.0), np.where(h < 6, 0.0, np.where(h & 1, -1.0, 1.0)))
    return gx * x + gy * y


def perlin2(x: np.ndarray, y: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """2D improved Perlin gradient noise at real coordinates, values in about [-1, 1]."""
    xi = np.floor(x)
    yi = np.floor(y)
    xf = x - xi
    yf = y - yi
    X = xi.astype(np.int64) & 255
    Y = yi.astype(np.int64) & 255
    u = _fade(xf)
    v = _fade(yf)
    aa = perm[perm[X] + Y]
    ab = perm[perm[X] + Y + 1]
    ba = perm[perm[X + 1] + Y]
    bb = perm[perm[X + 1] + Y + 1]
    n00 = _grad2(aa, xf, yf)
    n10 = _grad2(ba, xf - 1.0, yf)
    n01 = _grad2(ab, xf, yf - 1.0)
    n11 = _grad2(bb, xf - 1.0, yf - 1.0)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return nx0 + v * (nx1 - nx0)


def perlin_fbm(h: int, w: int, rng: np.random.Generator, period: float = 32.0,
               octaves: int = 4, origin=(0.0, 0.0)) -> np.ndarray:
    """fBm of ``octaves`` Perlin octaves on an ``h x w`` integer lattice, float64 in ~[-1, 1]."""
    perm = _perm_table(rng)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    xs = xs + origin[0] + rng.uniform(0, 256)
    ys = ys + origin[1] + rng.uniform(0, 256)
    out = np.zeros((h, w))
    amp, freq, norm = 1.0, 1.0 / period, 0.0
    for _ in range(octaves):
        out += amp * perlin2(xs * freq, ys * freq, perm)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return out / norm * 1.6


def _texture(h: int, w: int, rng: np.random.Generator, period: float) -> np.ndarray:
    """RGB texture in [16, 240] (float32, shape [h][w][3]); one fBm field per channel."""
    base = rng.uniform(0.25, 0.75, size=3)
    chans = []
    for c in range(3):
        f = perlin_fbm(h, w, rng, period=period)
        chans.append(np.clip(base[c] + 0.5 * f, 0.0, 1.0))
    t = np.stack(chans, axis=-1)
    return (16.0 + 224.0 * t).astype(np.float32)


def make_scene_layers(spec: dict, h: int, w: int, na: int, nb: int, seed: int) -> dict:
    """Draw the layer list of a scene from ``spec`` with a seeded PCG64 generator.

    ``spec`` keys: ``planes`` (number of foreground layers), ``dmax`` (max |d|
    in pixels between adjacent views), ``background`` ('flat' or 'terrain'),
    ``shading`` (bool: Lambertian albedo*(0.2+0.8*max(0,n.l)) per layer),
    ``period`` (texture base period in pixels).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dmax = float(spec["dmax"])
    ac, bc = (na - 1) / 2.0, (nb - 1) / 2.0
    margin = int(np.ceil(dmax * max(ac, bc, 1.0))) + 4
    th, tw = h + 2 * margin, w + 2 * margin
    period = float(spec.get("period", 32.0))
    layers = []
    bg_kind = spec.get("background", "flat")
    bg = {"kind": bg_kind, "tex": _texture(th, tw, rng, period), "d": 0.0}
    if bg_kind == "terrain":
        # Smooth disparity field d(x, y) = dmax * noise(x / 256, y / 256), in target space.
        bg["dfield"] = (dmax * np.clip(perlin_fbm(h, w, rng, period=256.0, octaves=2), -1, 1)).astype(np.float32)
    else:
        bg["d"] = float(rng.uniform(-dmax, dmax))
    for _ in range(int(spec["planes"])):
        kind = "disc" if rng.uniform() < 0.4 else "rect"
        d = float(rng.uniform(-dmax, dmax))
        cx, cy = rng.uniform(0.1 * w, 0.9 * w), rng.uniform(0.1 * h, 0.9 * h)
        if kind == "rect":
            hw_, hh_ = rng.uniform(0.08 * w, 0.3 * w), rng.uniform(0.08 * h, 0.3 * h)
            geom = (cx - hw_, cy - hh_, cx + hw_, cy + hh_)
        else:
            geom = (cx, cy, rng.uniform(0.06, 0.25) * min(w, h))
        tex = _texture(th, tw, rng, period * rng.uniform(0.5, 1.5))
        if spec.get("shading", False):
            nvec = rng.normal(size=3)
            nvec[2] = abs(nvec[2]) + 0.5
            nvec /= np.linalg.norm(nvec)
            lvec = np.array([0.3, -0.4, 0.866])
            shade = 0.2 + 0.8 * max(0.0, float(nvec @ lvec))
            tex = (16.0 + (tex - 16.0) * shade).astype(np.float32)
        layers.append({"kind": kind, "d": d, "geom": geom, "tex": tex})
    layers.sort(key=lambda L: L["d"])
    return {"margin": margin, "bg": bg, "layers": layers, "ac": ac, "bc": bc}


def _shift_sample(tex: np.ndarray, margin: int, h: int, w: int, sx: float, sy: float) -> np.ndarray:
    """Bilinear sample of ``tex`` at (x - sx, y - sy) for the h x w target grid (constant shift)."""
    fx0 = np.floor(-sx)
    fy0 = np.floor(-sy)
    fx = np.float32(-sx - fx0)
    fy = np.float32(-sy - fy0)
    x0 = margin + int(fx0)
    y0 = margin + int(fy0)
    t00 = tex[y0:y0 + h, x0:x0 + w]
    t01 = tex[y0:y0 + h, x0 + 1:x0 + 1 + w]
    t10 = tex[y0 + 1:y0 + 1 + h, x0:x0 + w]
    t11 = tex[y0 + 1:y0 + 1 + h, x0 + 1:x0 + 1 + w]
    top = t00 + fx * (t01 - t00)
    bot = t10 + fx * (t11 - t10)
    return top + fy * (bot - top)


def _shift_window(tex: np.ndarray, margin: int, bx0: int, by0: int, ww: int, hh: int, sx: float,
                  sy: float) -> np.ndarray:
    """Rows by0 .. by0 + hh - 1, columns bx0 .. bx0 + ww - 1 of ``_shift_sample`` (same arithmetic per pixel)."""
    fx0 = np.floor(-sx)
    fy0 = np.floor(-sy)
    fx = np.float32(-sx - fx0)
    fy = np.float32(-sy - fy0)
    x0 = margin + int(fx0) + bx0
    y0 = margin + int(fy0) + by0
    t00 = tex[y0:y0 + hh, x0:x0 + ww]
    t01 = tex[y0:y0 + hh, x0 + 1:x0 + 1 + ww]
    t10 = tex[y0 + 1:y0 + 1 + hh, x0:x0 + ww]
    t11 = tex[y0 + 1:y0 + 1 + hh, x0 + 1:x0 + 1 + ww]
    top = t00 + fx * (t01 - t00)
    bot = t10 + fx * (t11 - t10)
    return top + fy * (bot - top)


def _gather_sample(tex: np.ndarray, margin: int, srcx: np.ndarray, srcy: np.ndarray) -> np.ndarray:
    th, tw = tex.shape[:2]
    X = np.clip(srcx + margin, 0, tw - 1.001)
    Y = np.clip(srcy + margin, 0, th - 1.001)
    x0 = np.floor(X).astype(np.int64)
    y0 = np.floor(Y).astype(np.int64)
    fx = (X - x0)[..., None].astype(np.float32)
    fy = (Y - y0)[..., None].astype(np.float32)
    t00 = tex[y0, x0]
    t01 = tex[y0, x0 + 1]
    t10 = tex[y0 + 1, x0]
    t11 = tex[y0 + 1, x0 + 1]
    top = t00 + fx * (t01 - t00)
    bot = t10 + fx * (t11 - t10)
    return top + fy * (bot - top)


def render_view(scene: dict, b: int, a: int, h: int, w: int) -> np.ndarray:
    """One view (b, a) of the scene as float32 [h][w][3] in [16, 240]."""
    ox, oy = a - scene["ac"], b - scene["bc"]
    m = scene["margin"]
    bg = scene["bg"]
    if bg["kind"] == "terrain":
        ys, xs = np.mgrid[0:h, 0:w].astype(np.float32)
        d = bg["dfield"]
        img = _gather_sample(bg["tex"], m, xs - d * ox, ys - d * oy)
    else:
        img = _shift_sample(bg["tex"], m, h, w, bg["d"] * ox, bg["d"] * oy)
    for L in scene["layers"]:
        sx, sy = L["d"] * ox, L["d"] * oy
        # pixels outside the layer's bounding box (one pixel of slack) are not
        # covered; inside it the mask and samples are evaluated per pixel
        if L["kind"] == "rect":
            gx0, gy0, gx1, gy1 = L["geom"]
        else:
            cx, cy, r = L["geom"]
            gx0, gy0, gx1, gy1 = cx - r, cy - r, cx + r, cy + r
        bx0, bx1 = max(0, int(np.floor(gx0 + sx)) - 1), min(w, int(np.ceil(gx1 + sx)) + 2)
        by0, by1 = max(0, int(np.floor(gy0 + sy)) - 1), min(h, int(np.ceil(gy1 + sy)) + 2)
        if bx0 >= bx1 or by0 >= by1:
            continue
        xs = np.arange(bx0, bx1, dtype=np.float64)[None, :]
        ys = np.arange(by0, by1, dtype=np.float64)[:, None]
        if L["kind"] == "rect":
            mask = (((xs - sx) >= gx0) & ((xs - sx) < gx1)) & (((ys - sy) >= gy0) & ((ys - sy) < gy1))
        else:
            mask = ((xs - sx - cx) ** 2 + (ys - sy - cy) ** 2) < r * r
        if not mask.any():
            continue
        layer_img = _shift_window(L["tex"], m, bx0, by0, bx1 - bx0, by1 - by0, sx, sy)
        np.copyto(img[by0:by1, bx0:bx1], layer_img, where=mask[..., None])
    return img


def make_lf(na: int, nb: int, h: int, w: int, spec: dict, seed: int, progress=None) -> np.ndarray:
    """Seeded light field ``uint8[nb][na][h][w][3]``; colour quantised as floor(c + 1/2).

    ``progress(done, total)``, if given, is called after every tenth of the views."""
    scene = make_scene_layers(spec, h, w, na, nb, seed)
    out = np.empty((nb, na, h, w, 3), dtype=np.uint8)
    total = nb * na

    def one(idx):
        b, a = divmod(idx, na)
        img = render_view(scene, b, a, h, w)
        out[b, a] = np.clip(np.floor(img + 0.5), 0, 255).astype(np.uint8)

    # Views are independent; numpy releases the GIL inside its kernels.
    workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for k, _ in enumerate(ex.map(one, range(total))):
            if progress is not None and (k + 1) % max(1, total // 10) == 0:
                progress(k + 1, total)
    return out
