"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Integer sample reconstruction must be bit-exact; FP32 rendering within 1e-5
absolute on the [0, 1] scale; ray coordinates bit-exact (both sides evaluate
them in binary32 without contraction, so every floor/fraction decision is
taken identically); footprint bytes equal.
"""

import numpy as np
import pytest

import lfscene
import oracle
from conftest import stream_for

pytestmark = pytest.mark.gpu

RENDER_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def lfmod():
    from paper_1902_09396_amd import lf

    return lf


def _cams_dev(torch, cams):
    return torch.from_numpy(np.ascontiguousarray(cams, dtype=np.float32)).cuda()


def _all_coords(o):
    b, a, y, x = np.meshgrid(np.arange(o.nb), np.arange(o.na), np.arange(o.h), np.arange(o.w), indexing="ij")
    return np.stack([b.ravel(), a.ravel(), y.ravel(), x.ravel()], 1).astype(np.int32)


def test_decode_tiny_every_pixel(torch_mod, lfmod, tiny_stream, tiny_oracle):
    torch = torch_mod
    L = lfmod.LightField(tiny_stream)
    coords = _all_coords(tiny_oracle)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    expect = tiny_oracle.decode_full().reshape(-1, 3)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("variant", ["step1", "step8_thr", "nomc", "zero_phase"])
def test_decode_tiny_variants(torch_mod, lfmod, tiny_lf, variant):
    torch = torch_mod
    over = {"step1": dict(step=1), "step8_thr": dict(step=8, t_ref=200, t_pred=400),
            "nomc": dict(no_mc=True), "zero_phase": dict(zero_phase=True)}[variant]
    s = stream_for("tiny", tiny_lf, **over)
    o = oracle.OracleLF(s)
    L = lfmod.LightField(s)
    coords = _all_coords(o)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_full().reshape(-1, 3))


def test_decode_mid_random_and_tiles(torch_mod, lfmod, mid_stream, mid_oracle):
    torch = torch_mod
    o = mid_oracle
    L = lfmod.LightField(mid_stream)
    rng = np.random.default_rng(11)
    n = 300000
    rand = np.stack([rng.integers(0, o.nb, n), rng.integers(0, o.na, n), rng.integers(0, o.h, n),
                     rng.integers(0, o.w, n)], 1).astype(np.int32)
    # tile-structured: whole 16x16 blocks of a few views, including the last block row/column
    tiles = []
    for (b, a) in [(0, 0), (16, 16), (7, 12), (3, 1)]:
        for by0, bx0 in [(0, 0), (112, 112), (48, 96)]:
            yy, xx = np.mgrid[by0:by0 + 16, bx0:bx0 + 16]
            tiles.append(np.stack([np.full(256, b), np.full(256, a), yy.ravel(), xx.ravel()], 1))
    coords = np.concatenate([rand] + tiles).astype(np.int32)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(coords))


def test_decode_clamps_and_empty(torch_mod, lfmod, tiny_stream, tiny_oracle):
    torch = torch_mod
    L = lfmod.LightField(tiny_stream)
    coords = np.array([[-1, -5, -3, -2], [8, 9, 64, 100], [3, 100, 10, -7]], dtype=np.int32)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    clamped = np.stack([np.clip(coords[:, 0], 0, 7), np.clip(coords[:, 1], 0, 7), np.clip(coords[:, 2], 0, 63),
                        np.clip(coords[:, 3], 0, 63)], 1)
    assert np.array_equal(got, tiny_oracle.decode_at(clamped))
    empty = L.decode_pixels(torch.zeros((0, 4), dtype=torch.int32, device="cuda"))
    assert empty.shape == (0, 3)


def test_ray_coords_bit_exact(torch_mod, lfmod, tiny_cams, tiny_cams_ez):
    torch = torch_mod
    cams = np.concatenate([tiny_cams, tiny_cams_ez, lfscene.make_views(lfscene.get_config("path512"))[:3]])
    wo, ho = 37, 29
    got = lfmod.ray_coords(_cams_dev(torch, cams), wo, ho).cpu().numpy()
    for v in range(cams.shape[0]):
        for (i, j) in [(0, 0), (36, 28), (5, 17), (20, 3), (36, 0)]:
            assert np.array_equal(got[v, j, i], oracle.ray_coords(cams[v], wo, ho, i, j)), (v, i, j)


@pytest.mark.parametrize("which", ["fixed", "ez"])
def test_render_tiny(torch_mod, lfmod, tiny_stream, tiny_oracle, tiny_cams, tiny_cams_ez, which):
    torch = torch_mod
    cams = tiny_cams if which == "fixed" else tiny_cams_ez
    L = lfmod.LightField(tiny_stream)
    got = L.render_views(_cams_dev(torch, cams), 64, 64).cpu().numpy().astype(np.float64)
    expect = tiny_oracle.render(cams, 64, 64)
    assert np.abs(got - expect).max() <= RENDER_TOL


def test_render_ragged_sizes(torch_mod, lfmod, tiny_stream, tiny_oracle, tiny_cams_ez):
    torch = torch_mod
    L = lfmod.LightField(tiny_stream)
    for wo, ho in [(1, 1), (13, 7), (70, 33)]:
        got = L.render_views(_cams_dev(torch, tiny_cams_ez[:2]), wo, ho).cpu().numpy().astype(np.float64)
        expect = tiny_oracle.render(tiny_cams_ez[:2], wo, ho)
        assert np.abs(got - expect).max() <= RENDER_TOL, (wo, ho)


def test_render_mid_orbit(torch_mod, lfmod, mid_stream, mid_oracle):
    torch = torch_mod
    cams = lfscene.camera_path_orbit(120, 17, 17, 128, 128, 128, 128, radius=6.0)[::29]
    L = lfmod.LightField(mid_stream)
    got = L.render_views(_cams_dev(torch, cams), 128, 128).cpu().numpy().astype(np.float64)
    expect = mid_oracle.render(cams, 128, 128)
    assert np.abs(got - expect).max() <= RENDER_TOL


def test_tiled_equals_per_ray(torch_mod, lfmod, mid_stream, tiny_stream, tiny_cams_ez):
    torch = torch_mod
    M = lfmod.LightField(mid_stream)
    cams = _cams_dev(torch, lfscene.camera_path_orbit(6, 17, 17, 128, 128, 100, 70))
    a = M.render_views(cams, 100, 70).cpu().numpy()
    b = M.render_views(cams, 100, 70, per_ray=True).cpu().numpy()
    assert np.array_equal(a, b)
    # zoomed-out wide cameras: footprints exceed the staging budget and take the per-ray branch
    T = lfmod.LightField(tiny_stream)
    wide = lfscene.random_pinhole_cameras(3, 8, 8, 64, 64, 40, 40, seed=5, ez_range=(-8.0, -6.0),
                                          zoom_range=(4.0, 6.0), rho=1.0)
    a = T.render_views(_cams_dev(torch, wide), 40, 40).cpu().numpy()
    b = T.render_views(_cams_dev(torch, wide), 40, 40, per_ray=True).cpu().numpy()
    assert np.array_equal(a, b)


def test_tail_split_equals_per_ray(torch_mod, lfmod, mid_stream):
    """A launch with more (chunk, tile) items than one round of resident
    workgroups and a ragged remainder: the remainder items are cut into runs
    of views, the last chunk is short, and every pixel still equals the
    per-ray kernel's."""
    torch = torch_mod
    M = lfmod.LightField(mid_stream)
    nv, wo, ho = 60, 400, 200
    vpg, vpc = lfmod.render_config(nv, wo, ho)
    tiles = ((wo + 31) // 32) * ((ho + 7) // 8)
    n_work = tiles * ((nv + vpc - 1) // vpc)
    assert n_work > 3 * 256 and n_work % (3 * 256) != 0 and nv % vpc != 0
    cams = _cams_dev(torch, lfscene.camera_path_orbit(nv, 17, 17, 128, 128, wo, ho))
    a = M.render_views(cams, wo, ho).cpu().numpy()
    b = M.render_views(cams, wo, ho, per_ray=True).cpu().numpy()
    assert np.array_equal(a, b)


def test_render_projective_cameras(torch_mod, lfmod, tiny_stream, tiny_oracle, tiny_cams_ez, mid_stream):
    """Cameras with a tilted image plane: the footprint boxes come from every
    pixel of a tile instead of its four corners."""
    torch = torch_mod
    cams = lfscene.projective_warp(tiny_cams_ez, 2e-3, -3e-3)
    assert np.all(cams[:, 8] == 1.0) and np.any(cams[:, 6] != 0.0)
    L = lfmod.LightField(tiny_stream)
    got = L.render_views(_cams_dev(torch, cams), 64, 64).cpu().numpy().astype(np.float64)
    expect = tiny_oracle.render(cams, 64, 64)
    assert np.abs(got - expect).max() <= RENDER_TOL
    # mixed group: affine and projective views in one launch, tiled = per-ray
    M = lfmod.LightField(mid_stream)
    orbit = lfscene.camera_path_orbit(8, 17, 17, 128, 128, 100, 70)
    mixed = orbit.copy()
    mixed[1::2] = lfscene.projective_warp(orbit[1::2], 1e-3, 2e-3)
    a = M.render_views(_cams_dev(torch, mixed), 100, 70).cpu().numpy()
    b = M.render_views(_cams_dev(torch, mixed), 100, 70, per_ray=True).cpu().numpy()
    assert np.array_equal(a, b)


def test_load_rejects_large_reference_values(torch_mod, lfmod, tiny_stream):
    """A reference SRV beyond +-2047 (impossible for 8-bit content) is a format error."""
    table_off = int(np.frombuffer(tiny_stream[128:136].tobytes(), np.uint64)[0])
    bad = tiny_stream.copy()
    # BFS node 0 is the (0, 0) reference node of level H-1; raise the minimum of
    # its first significant block of channel 0
    for e in range(64):
        o = table_off + 8 * e
        if bad[o + 6] != 0xFF:
            bad[o + 4:o + 6] = np.frombuffer(np.int16(2000).tobytes(), np.uint8)
            break
    else:
        pytest.skip("no significant reference block in node 0")
    with pytest.raises(lfmod.LFError) as e:
        lfmod.LightField(bad)
    assert e.value.status == lfmod.LF_EFORMAT
    lfmod.LightField(tiny_stream)  # the unmodified stream still loads


def test_cached_groups_equal_per_ray(torch_mod, lfmod, mid_stream):
    """Long view sequences: a workgroup renders a chunk of views in several
    groups and keeps decoded leaf views and ancestors between them.  The
    staged renderer must match the unstaged per-ray kernel bit for bit when
    entries are kept, evicted, and invalidated (footprint box changes)."""
    torch = torch_mod
    M = lfmod.LightField(mid_stream)
    orbit = lfscene.camera_path_orbit(48, 17, 17, 128, 128, 128, 96, radius=6.0)
    back = orbit[::-1].copy()
    mixed = np.empty_like(orbit)
    mixed[0::2], mixed[1::2] = orbit[0::2], back[0::2]  # jumps back and forth across the grid
    zoom = lfscene.random_pinhole_cameras(40, 17, 17, 128, 128, 128, 96, seed=21, rho=1.0 / 16.0)
    for cams in (orbit, mixed, zoom):
        c = _cams_dev(torch, cams)
        a = M.render_views(c, 128, 96).cpu().numpy()
        b = M.render_views(c, 128, 96, per_ray=True).cpu().numpy()
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(1, 5, 64, 32, 3, 8), (7, 3, 48, 40, 2, 4), (2, 2, 32, 32, 1, 16),
                                   (9, 1, 16, 64, 4, 16), (5, 4, 64, 64, 2, 2), (4, 5, 96, 64, 2, 32),
                                   (3, 3, 128, 64, 2, 64)])
def test_thin_and_ragged_grids(torch_mod, lfmod, shape):
    """Single-row and single-column grids, odd grid sizes, one-level trees and
    every block size the loader accepts for the tile renderer and below it
    (2x2 blocks render per ray; 32x32 and 64x64 on the tile path): decode
    bit-exact, render <= 1e-5, staged = per-ray."""
    torch = torch_mod
    na, nb, w, h, levels, block = shape
    lf = np.ascontiguousarray(lfscene.make_lf(na, nb, h, w, lfscene.get_config("tiny")["lf"]["spec"], 7))
    cfg = lfscene.get_config("tiny", levels=levels, block=block, step=4, win=4, t_ref=0, t_pred=0)
    s = oracle.encode(lf, cfg["enc"])
    o = oracle.OracleLF(s)
    L = lfmod.LightField(s)
    coords = _all_coords(o)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_full().reshape(-1, 3))
    cams = lfscene.random_pinhole_cameras(5, na, nb, w, h, 45, 27, seed=3, rho=1.0 / 8.0)
    c = _cams_dev(torch, cams)
    img = L.render_views(c, 45, 27).cpu().numpy()
    assert np.abs(img.astype(np.float64) - o.render(cams, 45, 27)).max() <= RENDER_TOL
    assert np.array_equal(img, L.render_views(c, 45, 27, per_ray=True).cpu().numpy())


def test_render_deterministic(torch_mod, lfmod, mid_stream):
    torch = torch_mod
    cams = _cams_dev(torch, lfscene.camera_path_orbit(8, 17, 17, 128, 128, 96, 80))
    L = lfmod.LightField(mid_stream)
    a = L.render_views(cams, 96, 80).cpu().numpy()
    b = L.render_views(cams, 96, 80).cpu().numpy()
    assert np.array_equal(a, b)


def test_footprint_bytes_match_oracle(torch_mod, lfmod, tiny_stream, tiny_oracle, tiny_cams, tiny_cams_ez,
                                      mid_stream, mid_oracle):
    torch = torch_mod
    L = lfmod.LightField(tiny_stream)
    cams = np.concatenate([tiny_cams, tiny_cams_ez])
    got = L.footprint_bytes(_cams_dev(torch, cams), 64, 64)
    expect = tiny_oracle.footprint_bytes(cams, 64, 64)
    assert np.allclose(got, expect, rtol=1e-12, atol=0)
    M = lfmod.LightField(mid_stream)
    cams = lfscene.camera_path_orbit(120, 17, 17, 128, 128, 128, 128)[::40]
    assert np.allclose(M.footprint_bytes(_cams_dev(torch, cams), 128, 128),
                       mid_oracle.footprint_bytes(cams, 128, 128), rtol=1e-12, atol=0)
