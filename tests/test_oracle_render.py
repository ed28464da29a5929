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
