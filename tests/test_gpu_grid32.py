"""Parity on the 32x32-view, 5-level configuration: the same grid, tree
height, shaded layers and disparity range as the 32x32x1024^2 light field,
with 128x128 views so the oracle encodes it in seconds; batches of 1920x1080
random pinhole cameras (magnified st windows, eye heights -1 .. 0.5).  The
oracle checks sampled outputs one by one: 2*10^5 decoded samples (bit-exact)
and 20000 random rays plus whole rows of each view (<= 1e-5)."""

import copy

import numpy as np
import pytest

import lfscene
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grid32():
    import torch

    from paper_1902_09396_amd import lf

    cfg = copy.deepcopy(lfscene.get_config("batch1080"))
    L = cfg["lf"]
    L["h"] = L["w"] = 128
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    stream = oracle.encode(light, cfg["enc"])
    o = oracle.OracleLF(stream)
    field = lf.LightField(stream, device="cuda:0")
    cams = lfscene.random_pinhole_cameras(8, 32, 32, 128, 128, 1920, 1080, seed=32)
    return torch, o, field, cams


def test_grid32_decode_samples(grid32):
    torch, o, field, cams = grid32
    assert field.info["levels"] == 5
    rng = np.random.default_rng(31)
    n = 200_000
    coords = np.stack([rng.integers(0, 32, n), rng.integers(0, 32, n), rng.integers(0, 128, n),
                       rng.integers(0, 128, n)], 1).astype(np.int32)
    got = field.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(coords))


def test_grid32_render_1080p(grid32):
    torch, o, field, cams = grid32
    V, wo, ho = cams.shape[0], 1920, 1080
    dev = torch.from_numpy(cams).cuda()
    img = field.render_views(dev, wo, ho).cpu().numpy()
    rng = np.random.default_rng(33)
    n = 20000
    rays = np.stack([rng.integers(0, V, n), rng.integers(0, wo, n), rng.integers(0, ho, n)], 1)
    for v, j in [(0, 0), (3, 539), (7, 1079)]:
        rows = np.stack([np.full(wo, v), np.arange(wo), np.full(wo, j)], 1)
        rays = np.concatenate([rays, rows])
    rays = rays.astype(np.int32)
    expect = o.render_rays(cams, wo, ho, rays)
    got = img[rays[:, 0], :, rays[:, 2], rays[:, 1]].astype(np.float64)
    assert np.abs(got - expect).max() <= 1e-5
    # the staged renderer equals the per-ray kernel on every pixel of two views
    a = field.render_views(dev[:2], wo, ho).cpu().numpy()
    b = field.render_views(dev[:2], wo, ho, per_ray=True).cpu().numpy()
    assert np.array_equal(a, b)
