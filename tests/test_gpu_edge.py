"""Degenerate calls: zero views render nothing and succeed on every render
entry point (dense and sparse handles); sizes below one and unknown levels
are rejected before anything is enqueued."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_zero_views_and_bad_sizes(tiny_stream, tiny_cams):
    import torch

    from paper_1902_09396_amd import lf

    for sparse in (False, True):
        L = lf.LightField(tiny_stream, sparse_refs=sparse)
        none = torch.zeros((0, 18), dtype=torch.float32, device="cuda")
        assert L.render_views(none, 64, 48).shape == (0, 3, 48, 64)
        assert L.render_views(none, 64, 48, per_ray=True).shape == (0, 3, 48, 64)
        assert L.render_views_lod(1, none, 64, 48).shape == (0, 3, 48, 64)
        res, sh = L.export_params()
        assert L.render_relaxed(res, sh, none, 64, 48).shape == (0, 3, 48, 64)
        cams = torch.from_numpy(np.ascontiguousarray(tiny_cams[:1], dtype=np.float32)).cuda()
        for w, h in ((0, 48), (64, 0)):
            with pytest.raises(lf.LFError) as e:
                L.render_views(cams, w, h)
            assert e.value.status == lf.LF_EINVAL
        with pytest.raises(lf.LFError) as e:
            L.render_views_lod(L.info["levels"] + 1, cams, 64, 48)
        assert e.value.status == lf.LF_EINVAL
        L.close()


def _craft_2x2():
    from streamkit import Craft

    k = Craft(na=2, nb=2, w=16, h=8, levels=1, block=4, step=[4], win=[2])
    rng = np.random.default_rng(5)
    k.root[0] = rng.integers(0, 256, (1, 1, 8, 16))
    k.root[1:] = rng.integers(-100, 100, (2, 1, 1, 8, 16))
    for blk in range(k.nblk):
        k.set_block(0, 0, 0, 0, blk, rng.integers(-20, 20, 16))  # the reference
        for B, A in ((0, 1), (1, 0), (1, 1)):
            k.set_block(0, 0, B, A, blk, rng.integers(-20, 20, 16))
            k.set_mv(0, 0, B, A, blk, int(rng.integers(-8, 9)), int(rng.integers(-8, 9)), 1)
    return k


def _int32_path_matches_oracle(s):
    """A sparse handle renders and decodes through the int32 per-sample walk."""
    import torch

    import oracle
    from paper_1902_09396_amd import lf

    L = lf.LightField(s, sparse_refs=True)
    o = oracle.OracleLF(s)
    coords = np.array([(b, a, y, x) for b in range(2) for a in range(2) for y in range(8) for x in range(16)],
                      dtype=np.int32)
    got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
    assert np.array_equal(got, o.decode_at(coords))
    import lfscene

    cams = lfscene.random_pinhole_cameras(3, 2, 2, 16, 8, 24, 16, seed=4, rho=0.25)
    img = L.render_views(torch.from_numpy(cams).cuda(), 24, 16).cpu().numpy()
    assert np.abs(img - o.render(cams, 24, 16)).max() <= 1e-5
    L.close()


def test_load_rejects_samples_beyond_the_packed_range():
    """Decoded Y, Co or Cg beyond +-8191 (8-bit content stays within
    255 + step / 2) would wrap the tile renderer's 16-bit lanes: a dense load
    is a format error.  The stream itself is valid, and the int32 path that
    a sparse handle uses decodes and renders it as the oracle does."""
    from paper_1902_09396_amd import lf

    k = _craft_2x2()
    lf.LightField(k.build()).close()  # in range: loads
    k.set_block(0, 0, 1, 1, 3, np.full(16, 2100))  # residual 8400 on one block of view (1, 1)
    s = k.build()
    with pytest.raises(lf.LFError) as e:
        lf.LightField(s)
    assert e.value.status == lf.LF_EFORMAT and "sample" in str(e.value)
    _int32_path_matches_oracle(s)


def test_load_rejects_motion_vectors_beyond_12_bits():
    """The tile renderer's descriptors hold vector components in 12 signed
    bits; a stream may code a wider one (its sequence range exceeds 8W).  A
    dense load rejects it; the int32 path takes it as the oracle does."""
    from paper_1902_09396_amd import lf

    k = _craft_2x2()
    k.mv_bits[(0, 0)] = 13
    k.set_mv(0, 0, 1, 0, 2, 3000, -5, 1)  # far outside the plane: clamped taps
    s = k.build()
    with pytest.raises(lf.LFError) as e:
        lf.LightField(s)
    assert e.value.status == lf.LF_EFORMAT and "motion vector" in str(e.value)
    _int32_path_matches_oracle(s)
    k.set_mv(0, 0, 1, 0, 2, 2047, -8, -1)  # the widest accepted component (my + 4W must be >= 0)
    s = k.build()
    L = lf.LightField(s)
    import torch

    import oracle

    coords = np.array([(1, 0, y, x) for y in range(8) for x in range(16)], dtype=np.int32)
    assert np.array_equal(L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy(),
                          oracle.OracleLF(s).decode_at(coords))


def test_decode_clamps_are_counted(tiny_stream, tiny_oracle):
    """Coordinates outside the grid are clamped (the result is the clamped
    sample's) and every clamped request is counted in lf_info."""
    import torch

    from paper_1902_09396_amd import lf

    for sparse in (False, True):
        L = lf.LightField(tiny_stream, sparse_refs=sparse)
        assert L.clamped_coords() == 0
        rng = np.random.default_rng(2)
        n = 5000
        coords = np.stack([rng.integers(-3, 11, n), rng.integers(-3, 11, n), rng.integers(-9, 73, n),
                           rng.integers(-9, 73, n)], 1).astype(np.int32)
        hi = np.array([8, 8, 64, 64])
        clamped = np.clip(coords, 0, hi - 1).astype(np.int32)
        n_out = int((clamped != coords).any(axis=1).sum())
        got = L.decode_pixels(torch.from_numpy(coords).cuda()).cpu().numpy()
        assert np.array_equal(got, tiny_oracle.decode_at(clamped))
        assert L.clamped_coords() == n_out > 0
        L.decode_pixels(torch.from_numpy(clamped).cuda())
        assert L.clamped_coords() == n_out
        lod = np.array([[0, 0, 0, 0], [5, 0, 0, 0], [0, -1, 70, 3]], dtype=np.int32)  # level-1 grid is 4x4
        L.decode_nodes(1, torch.from_numpy(lod).cuda())
        assert L.clamped_coords() == n_out + 2
        L.close()
