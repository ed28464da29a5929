"""The 4:2:0 chroma variant (Compressing HMLFC tree: the chroma channels are
sub-sampled) on the GPU against the oracle: the GPU encoder's streams equal
the oracle encoder's byte for byte; random-access decoding (leaf views and
every level of the progressive decode) is bit-exact, and rendering is within
1e-5, the tile renderer (leaf samples reconstructed from the luma walk and
the up-sampled chroma walks) equal to the per-ray kernel pixel for pixel.
Calls built on one plane geometry for all channels reject 4:2:0 handles."""

import ctypes as C

import numpy as np
import pytest

import lfscene
import oracle
from conftest import crop_lf

pytestmark = pytest.mark.gpu


def _enc(name="tiny", **over):
    e = lfscene.get_config(name)["enc"]
    e["chroma420"] = True
    for k, v in over.items():
        e[k] = [v] * e["levels"] if k in ("step", "win", "t_ref", "t_pred") and np.isscalar(v) else v
    return e


@pytest.fixture(scope="module")
def tiny420(tiny_lf):
    return oracle.encode(tiny_lf, _enc())


@pytest.fixture(scope="module")
def mid420(mid_lf):
    return oracle.encode(mid_lf, _enc("path512"))


@pytest.mark.parametrize("over", [{}, {"step": 1}, {"zero_phase": True}, {"no_mc": True},
                                  {"step": 8, "t_ref": 200, "t_pred": 400}, {"block": 4}, {"block": 2}])
def test_encoder_420_tiny(tiny_lf, over):
    from paper_1902_09396_amd import lf

    e = _enc(**over)
    assert np.array_equal(lf.encode(tiny_lf, e), oracle.encode(tiny_lf, e)), over


def test_encoder_420_odd_and_mid(mid_lf):
    from paper_1902_09396_amd import lf

    x = crop_lf("tiny", 7, 5, 32, 48)
    e = _enc(levels=3, block=4, step=[3, 2, 5], win=[2, 1, 3], t_ref=[10, 0, 0], t_pred=[30, 5, 0])
    assert np.array_equal(lf.encode(x, e), oracle.encode(x, e))
    e = _enc("path512")
    assert np.array_equal(lf.encode(mid_lf, e), oracle.encode(mid_lf, e))


def test_decode_420_every_pixel_and_levels(tiny420):
    import torch

    from paper_1902_09396_amd import lf

    o = oracle.OracleLF(tiny420)
    L = lf.LightField(tiny420)
    assert L.info["chroma420"] == 1
    coords = np.array([(b, a, y, x) for b in range(8) for a in range(8) for y in range(64) for x in range(64)],
                      dtype=np.int32)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(coords))
    assert np.array_equal(got.reshape(8, 8, 64, 64, 3), o.decode_full())
    for level in range(1, 3):
        n = 8 >> level if level < 3 else 1
        nodes = np.array([(B, A, y, x) for B in range(n) for A in range(n) for y in range(0, 64, 3)
                          for x in range(64)], dtype=np.int32)
        got = L.decode_nodes(level, torch.from_numpy(nodes).cuda()).cpu().numpy()
        assert np.array_equal(got, o.decode_node(level, nodes)), level
    # clamped requests are counted
    bad = np.array([[9, 0, 0, 0], [0, 0, 64, -1], [1, 1, 1, 1]], dtype=np.int32)
    got = L.decode_pixels(torch.from_numpy(bad).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(np.clip(bad, 0, [7, 7, 63, 63])))
    assert L.clamped_coords() == 2


def test_render_420(tiny420, tiny_cams, tiny_cams_ez):
    import torch

    from paper_1902_09396_amd import lf

    o = oracle.OracleLF(tiny420)
    L = lf.LightField(tiny420)
    for cams in (tiny_cams, tiny_cams_ez):
        cd = torch.from_numpy(np.ascontiguousarray(cams)).cuda()
        img = L.render_views(cd, 64, 48)
        assert torch.equal(img, L.render_views(cd, 64, 48, per_ray=True))
        assert np.abs(img.cpu().numpy() - o.render(cams, 64, 48)).max() <= 1e-5
        lod = L.render_views_lod(1, cd, 40, 24).cpu().numpy()
        assert np.abs(lod - o.render_lod(1, cams, 40, 24)).max() <= 1e-5


@pytest.mark.parametrize("block", [4, 16])
def test_render_420_tile_blocks(tiny_lf, block):
    """Tile renderer on 4:2:0 streams with 4x4 blocks (the small-block
    instance) and 16x16 blocks: equal to the per-ray kernel, within 1e-5 of
    the oracle."""
    import torch

    from paper_1902_09396_amd import lf

    s = oracle.encode(tiny_lf, _enc(block=block))
    o = oracle.OracleLF(s)
    L = lf.LightField(s)
    cams = lfscene.make_views(lfscene.get_config("tiny"))
    cd = torch.from_numpy(np.ascontiguousarray(cams)).cuda()
    img = L.render_views(cd, 72, 40)
    assert torch.equal(img, L.render_views(cd, 72, 40, per_ray=True))
    assert np.abs(img.cpu().numpy() - o.render(cams, 72, 40)).max() <= 1e-5


def test_render_420_beyond_budget(tiny420):
    """Zoomed-out wide cameras whose tile footprints exceed the tile
    renderer's LDS budget even for one view: those tiles are left to the
    4:2:0 per-ray pass.  Equal to the per-ray kernel, within 1e-5 of the
    oracle."""
    import torch

    from paper_1902_09396_amd import lf

    L = lf.LightField(tiny420)
    wide = lfscene.random_pinhole_cameras(3, 8, 8, 64, 64, 40, 40, seed=5, ez_range=(-8.0, -6.0),
                                          zoom_range=(4.0, 6.0), rho=1.0)
    cd = torch.from_numpy(np.ascontiguousarray(wide)).cuda()
    img = L.render_views(cd, 40, 40)
    assert torch.equal(img, L.render_views(cd, 40, 40, per_ray=True))
    assert np.abs(img.cpu().numpy() - oracle.OracleLF(tiny420).render(wide, 40, 40)).max() <= 1e-5


def test_render_420_tiled_orbit(mid420):
    """A 60-view orbit over the 17x17 grid in 4:2:0 through the tile
    renderer: more (chunk, tile) items than one round of resident
    workgroups with a ragged remainder (tail runs, a short last chunk),
    groups of views sharing the cached leaf samples.  Every pixel equals the
    per-ray kernel's; sampled rays are within 1e-5 of the oracle."""
    import torch

    from paper_1902_09396_amd import lf

    L = lf.LightField(mid420)
    nv, wo, ho = 60, 400, 200
    cams = lfscene.camera_path_orbit(nv, 17, 17, 128, 128, wo, ho)
    cd = torch.from_numpy(np.ascontiguousarray(cams)).cuda()
    img = L.render_views(cd, wo, ho)
    assert torch.equal(img, L.render_views(cd, wo, ho, per_ray=True))
    rng = np.random.default_rng(21)
    rays = np.stack([rng.integers(0, nv, 4000), rng.integers(0, wo, 4000), rng.integers(0, ho, 4000)], 1)
    expect = oracle.OracleLF(mid420).render_rays(cams, wo, ho, rays)
    got = img.cpu().numpy()[rays[:, 0], :, rays[:, 2], rays[:, 1]]
    assert np.abs(got - expect).max() <= 1e-5


def test_render_420_mid(mid_lf, mid420):
    import torch

    from paper_1902_09396_amd import lf

    s = mid420
    o = oracle.OracleLF(s)
    L = lf.LightField(s)
    cams = lfscene.random_pinhole_cameras(3, 17, 17, 128, 128, 96, 64, seed=9, rho=1.0 / 16.0)
    cd = torch.from_numpy(cams).cuda()
    img = L.render_views(cd, 96, 64)
    assert torch.equal(img, L.render_views(cd, 96, 64, per_ray=True))
    img = img.cpu().numpy()
    assert np.abs(img - o.render(cams, 96, 64)).max() <= 1e-5
    rng = np.random.default_rng(4)
    coords = np.stack([rng.integers(0, 17, 200000), rng.integers(0, 17, 200000), rng.integers(0, 128, 200000),
                       rng.integers(0, 128, 200000)], 1).astype(np.int32)
    assert np.array_equal(L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy(), o.decode_at(coords))


def test_420_rejected_where_channels_share_one_geometry(tiny420, tiny_cams):
    import torch

    from paper_1902_09396_amd import lf
    from paper_1902_09396_amd.serve import Server

    L = lf.LightField(tiny420)
    cams = torch.from_numpy(np.ascontiguousarray(tiny_cams)).cuda()
    for call in (lambda: L.export_params(), lambda: L.footprint_bytes(cams, 64, 64),
                 lambda: Server([L], pool_bytes=1 << 20), lambda: lf.LightField(tiny420, sparse_refs=True)):
        with pytest.raises(lf.LFError) as e:
            call()
        assert e.value.status == lf.LF_EINVAL
    need = C.c_int64()
    assert lf.lib().lf_backward_workspace(L.handle, 1, 64, 64, C.byref(need)) == lf.LF_EINVAL
