"""Serving loop: each result is the same alone and in the mix and matches
the oracle's render, memory admission queues what does not fit, oversize
requests are rejected, and graph replays give the same pixels as plain
launches.  Mixed requests up to 200x150 on the 8x8x64^2 and 17x17x128^2
fields, and the serving workload's resolutions (256^2, 512^2, 1920x1080,
2048^2) on full-size 9x9x256^2 and 17x17x512^2 fields."""

import numpy as np
import pytest

import lfscene
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fields(tiny_stream, mid_stream):
    from paper_1902_09396_amd import lf

    return [lf.LightField(tiny_stream), lf.LightField(mid_stream)]


@pytest.fixture(scope="module")
def oracles(tiny_oracle, mid_oracle):
    return [tiny_oracle, mid_oracle]


def _requests(n, seed=9):
    rng = np.random.default_rng(seed)
    sizes = [(64, 64), (100, 70), (128, 128), (33, 17), (200, 150)]
    reqs = []
    for k in range(n):
        field = int(rng.integers(0, 2))
        na, w = (8, 64) if field == 0 else (17, 128)
        wo, ho = sizes[int(rng.integers(0, len(sizes)))]
        cam = lfscene.random_pinhole_cameras(1, na, na, w, w, wo, ho, seed=int(rng.integers(1 << 30)),
                                             rho=1.0 / (4.0 if field == 0 else 16.0))[0]
        reqs.append((field, cam, wo, ho))
    return reqs


def _alone(torch, fields, reqs):
    outs = []
    for field, cam, wo, ho in reqs:
        c = torch.from_numpy(cam[None].copy()).cuda()
        outs.append(fields[field].render_views(c, wo, ho)[0].cpu().numpy())
    return outs


@pytest.mark.parametrize("use_graphs", [True, False])
def test_results_same_alone_and_in_mix(fields, oracles, use_graphs):
    import torch

    from paper_1902_09396_amd.serve import Server

    reqs = _requests(40)
    ref = _alone(torch, fields, reqs)
    # small launches and chunks force every request to span several launches and streams
    srv = Server(fields, pool_bytes=64 << 20, max_slots=8, max_tiles=24, chunk_tiles=3, n_streams=2,
                 use_graphs=use_graphs, grid=64)
    ids = [srv.submit(f, cam, wo, ho) for (f, cam, wo, ho) in reqs]
    for k, rid in enumerate(ids):
        out, lat = srv.wait(rid, reqs[k][2], reqs[k][3])
        got = out.cpu().numpy()
        assert np.abs(got - ref[k]).max() <= 1e-5
        assert np.array_equal(got, ref[k])  # same tile routine: expected bit for bit
        f, cam, wo, ho = reqs[k]
        assert np.abs(got - oracles[f].render(cam[None], wo, ho)[0]).max() <= 1e-5
        assert lat > 0
        srv.release(rid)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["launches"] > 10
    srv.close()


def test_memory_admission_queues_and_rejects(fields):
    import torch

    from paper_1902_09396_amd import lf
    from paper_1902_09396_amd.serve import Server

    reqs = [(1, r[1], 128, 128) for r in _requests(12, seed=3) if r[0] == 1][:6]
    reqs += [(0, r[1], 64, 64) for r in _requests(12, seed=4) if r[0] == 0][:6]
    ref = _alone(torch, fields, reqs)
    one = 3 * 128 * 128 * 4
    srv = Server(fields, pool_bytes=2 * one + 4096, max_slots=16, max_tiles=64, chunk_tiles=16)
    ids = [srv.submit(f, cam, wo, ho) for (f, cam, wo, ho) in reqs]
    # outputs are released only after reading them: at most two 128^2 results fit at once
    for k, rid in enumerate(ids):
        out, _ = srv.wait(rid, reqs[k][2], reqs[k][3])
        assert np.array_equal(out.cpu().numpy(), ref[k])
        srv.release(rid)
    with pytest.raises(lf.LFError) as e:
        srv.submit(1, reqs[0][1], 512, 512)
    assert e.value.status == lf.LF_ENOMEM
    srv.close()


def test_replay_and_baseline_schedule(fields):
    from paper_1902_09396_amd.serve import Server, baseline

    reqs = _requests(60, seed=5)
    field = np.array([r[0] for r in reqs])
    cams = np.stack([r[1] for r in reqs])
    wh = np.array([[r[2], r[3]] for r in reqs])
    arrival = np.cumsum(np.random.default_rng(6).exponential(1.0 / 2000.0, size=len(reqs)))
    srv = Server(fields, pool_bytes=64 << 20)
    lat, mk = srv.replay(field, cams, wh, arrival)
    assert np.all(lat > 0) and mk > 0
    srv.close()
    lat_b, mk_b = baseline(fields, field, cams, wh, arrival)
    assert np.all(lat_b > 0) and mk_b > 0


@pytest.fixture(scope="module")
def full_fields():
    """The serving workload's 9x9x256^2 and 17x17x512^2 fields, GPU-encoded."""
    from paper_1902_09396_amd import lf

    out = []
    for name in ("serve256", "path512"):
        cfg = lfscene.get_config(name)
        L = cfg["lf"]
        light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
        stream = lf.encode(light, cfg["enc"])
        out.append((lf.LightField(stream), oracle.OracleLF(stream), (L["na"], L["nb"], L["w"], L["h"])))
    return out


def test_serving_resolutions_match_oracle(full_fields):
    """1920x1080 and 2048^2 requests (minified and magnified st windows, eye
    heights -1 .. 0.5) beside 256^2 and 512^2 ones, all admitted together:
    each served output equals its own lf_render_views bit for bit and the
    oracle within 1e-5 on 20000 random rays and two whole rows."""
    import torch

    from paper_1902_09396_amd.serve import Server

    rng = np.random.default_rng(55)
    sizes = [(1920, 1080), (2048, 2048), (256, 256), (512, 512), (2048, 2048), (1920, 1080)]
    reqs = []
    for k, (wo, ho) in enumerate(sizes):
        f = k % 2
        na, nb, w, h = full_fields[f][2]
        cam = lfscene.random_pinhole_cameras(1, na, nb, w, h, wo, ho, seed=int(rng.integers(1 << 30)))[0]
        reqs.append((f, cam, wo, ho))
    pool = sum(3 * wo * ho * 4 for _, _, wo, ho in reqs) + (1 << 20)
    srv = Server([ff[0] for ff in full_fields], pool_bytes=pool, max_slots=8, max_tiles=4096, chunk_tiles=256,
                 n_streams=2)
    ids = [srv.submit(f, cam, wo, ho) for (f, cam, wo, ho) in reqs]
    for k, rid in enumerate(ids):
        f, cam, wo, ho = reqs[k]
        out, lat = srv.wait(rid, wo, ho)
        got = out.cpu().numpy()
        srv.release(rid)
        alone = full_fields[f][0].render_views(torch.from_numpy(cam[None].copy()).cuda(), wo, ho)[0].cpu().numpy()
        assert np.array_equal(got, alone), (k, wo, ho)
        n = 20000
        rays = np.stack([np.zeros(n, np.int64), rng.integers(0, wo, n), rng.integers(0, ho, n)], 1)
        rows = [int(rng.integers(0, ho)), ho - 1]
        rays = np.concatenate([rays] + [np.stack([np.zeros(wo, np.int64), np.arange(wo), np.full(wo, j)], 1)
                                        for j in rows]).astype(np.int32)
        exp = full_fields[f][1].render_rays(cam[None], wo, ho, rays)
        assert np.abs(got[:, rays[:, 2], rays[:, 1]].T - exp).max() <= 1e-5, (k, wo, ho)
        assert lat > 0
    assert srv.stats()["completed"] == len(reqs)
    srv.close()
