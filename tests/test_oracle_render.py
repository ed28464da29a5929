"""Pins of the oracle's two-plane renderer and footprint accounting.

Light Field Rendering (Prior Work): a new view interpolates captured rays
indexed by their crossings (u, v) and (s, t) of the two planes.  The oracle
must agree with SciPy's multilinear interpolation (``map_coordinates``,
order 1, edge-clamped) on the decoded 4D array, return stored samples
exactly at integer coordinates, render a constant light field as that
constant, and give the same image from random-access decoding as from the
fully decoded array.
"""

import numpy as np
import pytest
from scipy import ndimage

import lfscene
import oracle


def _coords(cams, wo, ho):
    out = np.empty((cams.shape[0], ho, wo, 4), dtype=np.float32)
    for v in range(cams.shape[0]):
        for j in range(ho):
            for i in range(wo):
                out[v, j, i] = oracle.ray_coords(cams[v], wo, ho, i, j)
    return out


def test_ray_coords_full_frame_integer():
    st = lfscene.full_frame_st(64, 64, 64, 64)
    cam = lfscene.cameras.fixed_uv_camera(2.25, 5.5, st)
    for i, j in [(0, 0), (17, 40), (63, 63)]:
        q = oracle.ray_coords(cam, 64, 64, i, j)
        assert q.tolist() == [2.25, 5.5, float(i), float(j)]


@pytest.mark.parametrize("which", ["fixed", "ez"])
def test_render_matches_scipy_multilinear(tiny_oracle, tiny_cams, tiny_cams_ez, which):
    cams = tiny_cams if which == "fixed" else tiny_cams_ez
    o = tiny_oracle
    full = o.decode_full().astype(np.float64) / 255.0
    wo = ho = 24  # a sub-sampled output grid keeps the python coordinate loop short
    cams = cams.copy()
    # rescale the st homography to the smaller output (same window)
    for v in range(cams.shape[0]):
        cams[v, 9:18] = (cams[v, 9:18].reshape(3, 3) @ np.diag([64 / wo, 64 / ho, 1.0])).reshape(-1)
        cams[v, 0:9] = (cams[v, 0:9].reshape(3, 3) @ np.diag([64 / wo, 64 / ho, 1.0])).reshape(-1)
    got = o.render(cams, wo, ho)
    q = _coords(cams, wo, ho).astype(np.float64)  # [V][ho][wo][u, v, s, t]
    for c in range(3):
        vol = full[..., c]  # [b][a][y][x]
        pts = np.stack([q[..., 1].ravel(), q[..., 0].ravel(), q[..., 3].ravel(), q[..., 2].ravel()])
        ref = ndimage.map_coordinates(vol, pts, order=1, mode="nearest").reshape(cams.shape[0], ho, wo)
        assert np.abs(got[:, c] - ref).max() <= 1e-6


def test_render_integer_rays_return_samples(tiny_oracle):
    o = tiny_oracle
    full = o.decode_full()
    st = lfscene.full_frame_st(64, 64, 64, 64)
    cams = np.stack([lfscene.cameras.fixed_uv_camera(u, v, st) for u, v in [(0, 0), (3, 5), (7, 7), (6, 1)]])
    got = o.render(cams, 64, 64)
    for k, (u, v) in enumerate([(0, 0), (3, 5), (7, 7), (6, 1)]):
        expect = np.moveaxis(full[v, u], -1, 0) / 255.0
        # fraction 0 gives the lower sample exactly; on the last row/column/view the
        # fraction is 1 and p + 1*(q - p) may differ from q in the last bit
        assert np.abs(got[k] - expect).max() <= 2.0 ** -52
        if u < 7 and v < 7:
            assert np.array_equal(got[k][:, :63, :63], expect[:, :63, :63])


def test_render_constant_lf():
    lf = np.empty((4, 4, 16, 16, 3), dtype=np.uint8)
    lf[...] = (200, 17, 99)
    enc = lfscene.get_config("tiny")["enc"]
    enc.update(block=8)
    o = oracle.OracleLF(oracle.encode(lf, enc))
    cams = lfscene.random_pinhole_cameras(3, 4, 4, 16, 16, 20, 12, seed=3, rho=0.25)
    got = o.render(cams, 20, 12)
    for c, val in enumerate((200, 17, 99)):
        assert np.allclose(got[:, c], val / 255.0, atol=1e-12, rtol=0)


def test_random_access_render_equals_dense(tiny_oracle, tiny_cams, tiny_cams_ez):
    o = tiny_oracle
    full = o.decode_full()
    for cams in (tiny_cams, tiny_cams_ez):
        assert np.array_equal(o.render(cams, 64, 64), oracle.render_dense(full, cams, 64, 64))


def test_footprint_exact_reference_only():
    # A 1x1 view grid has no predictive nodes: the footprint is the output plus the
    # reference blocks and root blocks the rays touch, all closed-form.
    rng = np.random.default_rng(1)
    lf = rng.integers(0, 256, size=(1, 1, 32, 32, 3)).astype(np.uint8)
    enc = lfscene.get_config("tiny")["enc"]
    enc.update(block=8)  # levels 2: grids 1 -> 1 -> 1
    o = oracle.OracleLF(oracle.encode(lf, enc))
    st = lfscene.full_frame_st(32, 32, 8, 8, zoom=0.25, off_x=8.0, off_y=0.0)
    cam = lfscene.cameras.fixed_uv_camera(0, 0, st)
    # s in [8, 15] and t in [0, 7] (+1 upper neighbour: x up to 16, y up to 8)
    # -> blocks (row 0, col 1), (0, 2), (1, 1), (1, 2)
    fb = o.footprint_bytes(cam[None], 8, 8)
    blocks = 4
    expect = 12 * 64 + 3 * 2 * blocks * 2 * 64 + 3 * blocks * 2 * 64
    assert fb[0] == expect


def test_render_rays_equals_render_every_ray(tiny_oracle, tiny_cams, tiny_cams_ez):
    # the selected-ray renderer (the full-size checker) gives, ray for ray, the
    # value of the whole-image renderer pinned above
    o = tiny_oracle
    for cams in (tiny_cams, tiny_cams_ez):
        full = o.render(cams, 64, 64)
        v, j, i = np.meshgrid(np.arange(cams.shape[0]), np.arange(64), np.arange(64), indexing="ij")
        rays = np.stack([v.ravel(), i.ravel(), j.ravel()], 1).astype(np.int32)
        got = o.render_rays(cams, 64, 64, rays)
        assert np.array_equal(got, np.moveaxis(full, 1, -1).reshape(-1, 3))


# ---------------------------------------------------------------------------
# Footprint of predictive blocks, closed form (the per-view algorithmic bytes:
# 12 B per ray; per distinct predictive block its 8-byte table entry, its
# payload words and its share of the motion-vector stream; 2 B per pixel of
# every distinct reference block read directly or through a non-zero-weight
# prediction tap, and of every distinct root block).  The stream is built by
# hand so that every motion vector is chosen by the test.

from streamkit import Craft  # noqa: E402


def _craft_2x2():
    # 2x2 views of 8x8, one SRV level (root 1x1), 4x4 blocks (2x2 per image),
    # step 2, window 4 (motion values 0..32: 6-bit plain fields)
    k = Craft(na=2, nb=2, w=8, h=8, levels=1, block=4, step=[2], win=[4])
    rng = np.random.default_rng(5)
    k.root[:] = rng.integers(-40, 40, size=k.root.shape)
    for c in range(3):
        for blk in range(4):
            k.set_block(c, 0, 0, 0, blk, rng.integers(-6, 6, 16))  # reference: 4 bits
    mv = {  # (channel, B, A): (mx, my, sigma) of block 0, in quarter pixels
        (0, 0, 1): (8, 0, 1),      # whole-pixel: taps at x + 2 -> columns 3, 4
        (0, 1, 0): (5, -3, 1),     # fractional: taps x0, x0 + 1 and y0, y0 + 1
        (0, 1, 1): (0, 0, 0),      # no prediction: no taps
        (1, 0, 1): (-16, 6, 1),    # across the left border (clamped) and half-pel in y
        (1, 1, 0): (0, 0, -1),
        (1, 1, 1): (16, 16, 1),    # lands wholly in block 3
        (2, 0, 1): (0, 0, 1), (2, 1, 0): (0, 0, 1), (2, 1, 1): (0, 0, 1),
    }
    for (c, B, A), (mx, my, sg) in mv.items():
        k.set_mv(c, 0, B, A, 0, mx, my, sg)
        if (c, B, A) == (0, 1, 1):
            continue  # insignificant block: no payload
        hi = 32 if (c, B, A) == (2, 0, 1) else 8  # 5-bit or 3-bit fields
        q = rng.integers(0, hi, 16)
        q[0], q[1] = 0, hi - 1
        k.set_block(c, 0, B, A, 0, q)
    return k


def test_streamkit_decode_matches_oracle():
    # the hand-built stream means what the kit says it means: the oracle's
    # full decode equals the kit's own reading of its content
    k = _craft_2x2()
    o = oracle.OracleLF(k.build())
    assert np.array_equal(o.decode_full_ycocg(), k.decode_ycocg())


def test_footprint_predictive_closed_form():
    k = _craft_2x2()
    o = oracle.OracleLF(k.build())
    # every ray: (u, v) = (0.5, 0.5) -> all four views; (s, t) = (1.5, 2.5)
    # -> x in {1, 2}, y in {2, 3}: block 0 of every image
    cam = np.array([0, 0, 0.5, 0, 0, 0.5, 0, 0, 1, 0, 0, 1.5, 0, 0, 2.5, 0, 0, 1], dtype=np.float32)
    rays = 2 * 2
    out = 12 * rays
    root = 3 * 2 * 16                     # block 0 of the root, three channels
    # reference blocks per channel: block 0 read directly, plus the tap blocks
    #   c0: (0,1) mv (8, 0) -> x+2 in {3, 4}: blocks 0, 1; (1,0) mv (5, -3):
    #       X = 4x + 5 -> x0 in {2, 3}, taps {2, 3, 4}; Y = 4y - 3 -> rows 1..3: blocks 0, 1
    #   c1: (0,1) mv (-16, 6): columns clamp to 0, Y = 4y + 6 -> rows 3..5: blocks 0, 2;
    #       (1,0) mv 0: block 0; (1,1) mv (16, 16): block 3
    #   c2: block 0
    refs = 2 * 16 * (2 + 3 + 1)
    # predictive blocks: 3 nodes x 3 channels, block 0; 12 records per (channel,
    # level), 24 six-bit motion values and 12 two-bit phase codes
    share = (24 * 6 + 12 * 2) / (8 * 12)
    table = 9 * (8 + share)
    payload = 4 * (7 * 2 + 3)  # seven 3-bit blocks of 16 values (2 words), one 5-bit (3 words)
    assert o.footprint_bytes(cam[None], 2, 2)[0] == out + root + refs + table + payload


def test_footprint_predictive_block_straddle():
    # (s, t) = (3.5, 0.5): x in {3, 4} -> blocks 0 and 1 of every image, y in {0, 1}
    k = _craft_2x2()
    o = oracle.OracleLF(k.build())
    cam = np.array([0, 0, 0.5, 0, 0, 0.5, 0, 0, 1, 0, 0, 3.5, 0, 0, 0.5, 0, 0, 1], dtype=np.float32)
    root = 3 * 2 * 16 * 2
    # block 1 of the predictive nodes carries the default record (0, 0, +1): its
    # taps stay in block 1; block 0 records as above but with y in {0, 1}, x in {3, 4}:
    #   c0 (0,1): x+2 in {5, 6}: block 1; (1,0): X = 4x + 5 -> taps 4..5, Y = 4y - 3 ->
    #       rows clamp to 0..1: block 1
    #   c1 (0,1): column 0, Y = 4y + 6 -> rows 1..2: block 0; (1,1): x+4 in {7, 8 -> 7},
    #       y+4 in {4, 5}: block 3
    refs = 2 * 16 * (2 + 3 + 2)  # c0 {0, 1}, c1 {0, 1, 3}, c2 {0, 1}
    share = (24 * 6 + 12 * 2) / (8 * 12)
    table = 18 * (8 + share)  # blocks 0 and 1 of 3 nodes x 3 channels; block 1 is insignificant
    payload = 4 * (7 * 2 + 3)
    assert o.footprint_bytes(cam[None], 2, 2)[0] == 12 * 4 + root + refs + table + payload
