"""Pins of the oracle's encoder and decoders.

* Lossless: with step 1 and zero thresholds every stored value is exact, so
  the decoded light field equals the input (the hierarchy uses lossless
  integer computations: Bounded Integer Sequence Encoding section).
* Random access equals full decoding (Decoding Procedure vs. materialising
  the whole tree).
* Without motion compensation the tree is the plain RLFC hierarchy: every
  level-(l+1) RKV is the rounded mean of its 2x2 cluster and every SRV is the
  view minus its RKV (RLFC: Hierarchical Compression Scheme).
* Closed-loop error bound: with zero thresholds each YCoCg channel of the
  decoded light field is within floor(step_0 / 2) of the input.
* Thresholds: a block whose energy is below the threshold is not stored.
* Malformed streams are rejected.
"""

import numpy as np
import pytest

import lfscene
import oracle
from conftest import crop_lf, stream_for


def _ycocg_lf(lf):
    return oracle.ycocg_fwd(lf.reshape(-1, 3)).reshape(lf.shape).astype(np.int64)


@pytest.mark.parametrize("no_mc", [False, True])
def test_lossless_roundtrip_tiny(tiny_lf, no_mc):
    s = stream_for("tiny", tiny_lf, step=1, no_mc=no_mc)
    o = oracle.OracleLF(s)
    assert np.array_equal(o.decode_full(), tiny_lf)


def test_lossless_roundtrip_mid(mid_lf):
    cfg = lfscene.get_config("path512", step=1)
    s = oracle.encode(mid_lf, cfg["enc"])
    o = oracle.OracleLF(s)
    assert (o.levels, o.block, o.na, o.nb) == (4, 16, 17, 17)
    assert np.array_equal(o.decode_full(), mid_lf)


def test_lossless_odd_grid():
    # ragged clusters at every level (7 -> 4 -> 2 -> 1), a 3-level tree, 4x4 blocks
    lf = crop_lf("tiny", 7, 5, 16, 24)
    enc = lfscene.get_config("tiny", levels=3, step=1, win=2)["enc"]
    enc.update(levels=3, block=4, step=[1] * 3, win=[2] * 3, t_ref=[0] * 3, t_pred=[0] * 3)
    o = oracle.OracleLF(oracle.encode(lf, enc))
    assert (o.root_na, o.root_nb) == (1, 1)
    assert np.array_equal(o.decode_full(), lf)


def test_random_access_equals_full_every_pixel(tiny_oracle):
    o = tiny_oracle
    full = o.decode_full()
    b, a, y, x = np.meshgrid(np.arange(o.nb), np.arange(o.na), np.arange(o.h), np.arange(o.w), indexing="ij")
    coords = np.stack([b.ravel(), a.ravel(), y.ravel(), x.ravel()], 1)
    assert np.array_equal(o.decode_at(coords).reshape(full.shape), full)


def test_random_access_equals_full_mid(mid_oracle):
    o = mid_oracle
    full = o.decode_full()
    rng = np.random.default_rng(5)
    n = 200000
    coords = np.stack([rng.integers(0, o.nb, n), rng.integers(0, o.na, n), rng.integers(0, o.h, n),
                       rng.integers(0, o.w, n)], 1)
    assert np.array_equal(o.decode_at(coords), full[coords[:, 0], coords[:, 1], coords[:, 2], coords[:, 3]])


def test_plain_hierarchy_without_mc(tiny_lf):
    s = stream_for("tiny", tiny_lf, step=1, no_mc=True)
    o = oracle.OracleLF(s)
    srv = o.decode_srv()  # [3][n_nodes][h][w], BFS: level 1 (4x4) first, then level 0 (8x8)
    I0 = np.moveaxis(_ycocg_lf(tiny_lf), -1, 0)  # [3][8][8][h][w]
    # level-1 RKVs: rounded mean of each 2x2 cluster (floor((sum + 2) / 4))
    I1 = np.floor_divide(I0.reshape(3, 4, 2, 4, 2, 64, 64).sum(axis=(2, 4)) + 2, 4)
    I2 = np.floor_divide(I1.reshape(3, 2, 2, 2, 2, 64, 64).sum(axis=(2, 4)) + 2, 4)
    up1 = np.repeat(np.repeat(I1, 2, axis=1), 2, axis=2)
    up2 = np.repeat(np.repeat(I2, 2, axis=1), 2, axis=2)
    assert np.array_equal(srv[:, 16:].reshape(3, 8, 8, 64, 64), I0 - up1)
    assert np.array_equal(srv[:, :16].reshape(3, 4, 4, 64, 64), I1 - up2)


@pytest.mark.parametrize("step", [2, 3, 4, 8])
def test_closed_loop_error_bound(tiny_lf, step):
    s = stream_for("tiny", tiny_lf, step=step)
    o = oracle.OracleLF(s)
    dec = o.decode_full_ycocg()  # [3][nb][na][h][w]
    ref = np.moveaxis(_ycocg_lf(tiny_lf), -1, 0)
    assert np.abs(dec - ref).max() <= step // 2


def test_threshold_drops_low_energy_blocks(tiny_lf):
    base = oracle.OracleLF(stream_for("tiny", tiny_lf))
    thr = oracle.OracleLF(stream_for("tiny", tiny_lf, t_ref=100000, t_pred=100000))
    # every SRV block's energy is below the threshold: all SRVs decode to zero
    assert np.all(thr.decode_srv() == 0)
    assert np.any(base.decode_srv() != 0)
    # the light field is then the root RKV of each view's subtree
    dec = thr.decode_full_ycocg()
    assert np.array_equal(dec[:, 0, 0], dec[:, 3, 3])


def test_malformed_streams_rejected(tiny_stream):
    bad = tiny_stream.copy()
    bad[0] ^= 0xFF
    with pytest.raises(ValueError):
        oracle.OracleLF(bad)
    with pytest.raises(ValueError):
        oracle.OracleLF(tiny_stream[:2000])
    bad = tiny_stream.copy()
    bad[136:144] = np.frombuffer(np.uint64(12345).tobytes(), np.uint8)  # table size
    with pytest.raises(ValueError):
        oracle.OracleLF(bad)


def _all_nodes(o, level):
    nb, na = -(-o.nb // (1 << level)), -(-o.na // (1 << level))
    B, A, y, x = np.meshgrid(np.arange(nb), np.arange(na), np.arange(o.h), np.arange(o.w), indexing="ij")
    return np.stack([B.ravel(), A.ravel(), y.ravel(), x.ravel()], 1).astype(np.int32), (nb, na)


@pytest.mark.parametrize("no_mc", [False, True])
def test_progressive_decode_is_the_rkv_pyramid(tiny_lf, no_mc):
    """Stopping the walk at level l gives the level-l node images; coded
    losslessly (step 1), those are the rounded-mean pyramid of the original
    views (Hierarchical Compression Scheme), whatever the motion vectors."""
    s = stream_for("tiny", tiny_lf, step=1, no_mc=no_mc)
    o = oracle.OracleLF(s)
    I0 = np.moveaxis(_ycocg_lf(tiny_lf), -1, 0)  # [3][8][8][h][w]
    I1 = np.floor_divide(I0.reshape(3, 4, 2, 4, 2, 64, 64).sum(axis=(2, 4)) + 2, 4)
    I2 = np.floor_divide(I1.reshape(3, 2, 2, 2, 2, 64, 64).sum(axis=(2, 4)) + 2, 4)
    for level, I in ((0, I0), (1, I1), (2, I2)):
        coords, (nb, na) = _all_nodes(o, level)
        got = o.decode_node(level, coords).reshape(nb, na, 64, 64, 3)
        expect = np.clip(oracle.ycocg_inv(np.moveaxis(I, 0, -1).reshape(-1, 3)), 0, 255)
        assert np.array_equal(got, expect.reshape(nb, na, 64, 64, 3).astype(np.uint8)), level
    with pytest.raises(ValueError):
        o.decode_node(3, coords[:1])


def test_progressive_decode_levels_lossy(tiny_lf):
    """Level 0 is the random-access decode; a level-l render reads each
    sample's level-l ancestor, so views of one cluster render alike."""
    o = oracle.OracleLF(stream_for("tiny", tiny_lf))
    coords = np.array([[5, 3, 10, 20], [7, 7, 63, 63], [0, 0, 0, 0]], dtype=np.int32)
    assert np.array_equal(o.decode_node(0, coords), o.decode_at(coords))
    node = o.decode_node(1, np.array([[2, 1, 10, 20]], dtype=np.int32))
    cams = np.stack([lfscene.cameras.fixed_uv_camera(4.0, 2.0, lfscene.full_frame_st(64, 64, 16, 16)),
                     lfscene.cameras.fixed_uv_camera(4.5, 2.5, lfscene.full_frame_st(64, 64, 16, 16))])
    r = o.render_lod(1, cams, 16, 16)
    assert np.array_equal(r[0], r[1])  # every sample of both reads views b 2..3, a 4..5: level-1 node (1, 2)
    assert np.array_equal(o.render_lod(0, cams, 16, 16), o.render(cams, 16, 16))
    assert node.shape == (1, 3)
