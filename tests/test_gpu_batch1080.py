"""Full-size parity on the 32x32x1024^2 configuration: 16 shaded layers with
occlusion edges, disparity -8 .. 8 px, a 5-level tree, 16x16 blocks, step 4,
quarter-pel vectors, rendered as one batch of 32 random 1920x1080 pinhole
cameras (eye heights -1 .. 0.5, st windows zoomed 0.5 .. 1) in the launch
configuration the benchmark times.  The stream comes from the GPU encoder
(parity is on decoding a given stream; that encoder equals the oracle's byte
for byte, test_gpu_encoder).  The oracle checks sampled outputs one by one:
10^5 random decoded samples bit-exact, and on 4 of the 32 views 20000 random
rays plus two whole rows each within 1e-5.  The tile renderer also equals the
one-thread-per-ray kernel bit for bit on those views."""

import numpy as np
import pytest

import lfscene
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch

    from paper_1902_09396_amd import lf

    cfg = lfscene.get_config("batch1080")
    L = cfg["lf"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    stream = lf.encode(light, cfg["enc"])
    del light
    field = lf.LightField(stream, device="cuda:0")
    o = oracle.OracleLF(stream)
    cams = lfscene.make_views(cfg)
    return torch, cfg, o, field, cams


def test_batch1080_decode_samples(big):
    torch, cfg, o, field, cams = big
    L = cfg["lf"]
    rng = np.random.default_rng(31)
    n = 100_000
    coords = np.stack([rng.integers(0, L["nb"], n), rng.integers(0, L["na"], n), rng.integers(0, L["h"], n),
                       rng.integers(0, L["w"], n)], 1).astype(np.int32)
    got = field.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(coords))


def test_batch1080_render_batch(big):
    torch, cfg, o, field, cams = big
    wo, ho = cfg["views"]["wo"], cfg["views"]["ho"]
    assert cams.shape[0] == 32
    out = field.render_views(torch.from_numpy(cams).cuda(), wo, ho)
    rng = np.random.default_rng(32)
    for v in (0, 9, 22, 31):
        img = out[v].cpu().numpy()
        n = 20000
        rays = np.stack([np.full(n, v), rng.integers(0, wo, n), rng.integers(0, ho, n)], 1)
        rows = [int(rng.integers(0, ho)), 0]
        rays = np.concatenate([rays] + [np.stack([np.full(wo, v), np.arange(wo), np.full(wo, j)], 1) for j in rows])
        rays = rays.astype(np.int32)
        exp = o.render_rays(cams, wo, ho, rays)
        assert np.abs(img[:, rays[:, 2], rays[:, 1]].T - exp).max() <= 1e-5, v
        one = torch.from_numpy(cams[v:v + 1].copy()).cuda()
        per_ray = field.render_views(one, wo, ho, per_ray=True)[0].cpu().numpy()
        assert np.array_equal(per_ray, img), v
