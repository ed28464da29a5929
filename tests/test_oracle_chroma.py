"""Pins for the 4:2:0 chroma variant of the oracle (Compressing HMLFC tree:
the chroma channels are sub-sampled).  Co and Cg are coded at half width and
height; decoding up-samples them with centred bilinear weights.  Pinned
against what fixes these definitions independently of the oracle's code:
  - grey content has zero chroma, so a lossless (step 1) stream decodes to
    the source exactly;
  - a lossless stream's chroma equals the 2x2 mean of the source chroma
    (NumPy reshape-mean, rounded half up) brought back by SciPy's order-1
    zoom with grid-centred sampling and edge replication, rounded half up;
    its luma equals the source's;
  - the closed loop bounds every half-resolution chroma value by step / 2;
  - random access equals the full decode;
  - grey content gives the same luma tree as its 4:4:4 stream."""

import numpy as np
import pytest
from scipy import ndimage

import lfscene
import oracle
from conftest import crop_lf, lf_for


def _enc(**over):
    e = lfscene.get_config("tiny")["enc"]
    e.update(chroma420=True)
    for k, v in over.items():
        e[k] = [v] * e["levels"] if k in ("step", "win", "t_ref", "t_pred") and np.isscalar(v) else v
    return e


def _ycocg(lf):
    r, g, b = (lf[..., k].astype(np.int64) for k in range(3))
    co = r - b
    t = b + (co >> 1)
    cg = g - t
    return t + (cg >> 1), co, cg


def _down_up(plane):
    """2x2 rounded mean, then centred bilinear x2 with edge replication, rounded half up."""
    h, w = plane.shape
    half = np.floor(plane.reshape(h // 2, 2, w // 2, 2).sum(axis=(1, 3)) / 4.0 + 0.5)
    up = ndimage.zoom(half, 2, order=1, mode="nearest", grid_mode=True)
    return half.astype(np.int64), np.floor(up + 0.5).astype(np.int64)


def test_grey_lossless():
    x = lf_for("tiny").copy()
    x[..., 1] = x[..., 0]
    x[..., 2] = x[..., 0]
    s = oracle.encode(x, _enc(step=1))
    assert np.array_equal(oracle.OracleLF(s).decode_full(), x)


@pytest.mark.parametrize("shape", [(8, 8, 64, 64), (5, 3, 32, 16)])
def test_lossless_chroma_is_down_up(shape):
    na, nb, h, w = shape
    x = crop_lf("tiny", na, nb, h, w)
    o = oracle.OracleLF(oracle.encode(x, _enc(step=1, block=8)))
    ycc = o.decode_full_ycocg()
    Y, Co, Cg = _ycocg(x)
    assert np.array_equal(ycc[0], Y)
    for c, src in ((1, Co), (2, Cg)):
        for b in range(nb):
            for a in range(na):
                half, up = _down_up(src[b, a])
                assert np.array_equal(ycc[c, b, a], up), (c, b, a)
                # the half-resolution decode is the 2x2 mean itself
                coords = np.array([(b, a, yy, xx) for yy in range(h // 2) for xx in range(w // 2)], dtype=np.int32)
                assert np.array_equal(o.decode_channel(c, coords).reshape(h // 2, w // 2), half)


def test_random_access_equals_full_decode_and_render():
    x = lf_for("tiny")
    o = oracle.OracleLF(oracle.encode(x, _enc()))
    full = o.decode_full()
    coords = np.array([(b, a, y, xx) for b in range(8) for a in range(8) for y in range(64) for xx in range(64)],
                      dtype=np.int32)
    assert np.array_equal(o.decode_at(coords).reshape(full.shape), full)
    # a ray at integer (u, v, s, t) renders the stored sample
    cams = lfscene.get_config("tiny")
    img = o.render(lfscene.make_views(cams), 64, 64)
    assert np.isfinite(img).all() and img.min() >= 0 and img.max() <= 1


@pytest.mark.parametrize("step", [2, 4, 7])
def test_closed_loop_bound_on_half_planes(step):
    x = crop_lf("tiny", 6, 5, 32, 32)
    o = oracle.OracleLF(oracle.encode(x, _enc(step=step, block=4)))
    Y, Co, Cg = _ycocg(x)
    coords = np.array([(b, a, yy, xx) for b in range(5) for a in range(6) for yy in range(16) for xx in range(16)],
                      dtype=np.int32)
    for c, src in ((1, Co), (2, Cg)):
        half = np.stack([_down_up(src[b, a])[0] for b in range(5) for a in range(6)])
        got = o.decode_channel(c, coords).reshape(half.shape)
        assert np.abs(got - half).max() <= step // 2
    fc = np.array([(b, a, yy, xx) for b in range(5) for a in range(6) for yy in range(32) for xx in range(32)],
                  dtype=np.int32)
    gotY = o.decode_channel(0, fc).reshape(5, 6, 32, 32)
    assert np.abs(gotY - Y).max() <= step // 2


def test_constant_chroma_keeps_the_luma_tree():
    """Grey content has zero chroma: every chroma block is insignificant, and
    the luma part of the 4:2:0 stream's table equals the 4:4:4 stream's byte
    for byte (the luma tree does not depend on the chroma format)."""
    x = lf_for("tiny").copy()
    x[..., 1] = x[..., 0]
    x[..., 2] = x[..., 0]
    s420 = oracle.encode(x, _enc())
    s444 = oracle.encode(x, dict(_enc(), chroma420=False))
    o4, o2 = oracle.OracleLF(s444), oracle.OracleLF(s420)
    nblk = (64 // 8) ** 2
    t4 = int(np.frombuffer(s444[128:136].tobytes(), np.uint64)[0])
    t2 = int(np.frombuffer(s420[128:136].tobytes(), np.uint64)[0])
    n_luma = o4.n_nodes * nblk * 8
    assert np.array_equal(s444[t4:t4 + n_luma], s420[t2:t2 + n_luma])
    assert o2.chroma420 == 1 and o4.chroma420 == 0


def test_chroma_rejects_odd_block_grids():
    x = crop_lf("tiny", 4, 4, 24, 24)  # 24 / 2 = 12 is not a multiple of 8
    with pytest.raises(ValueError):
        oracle.encode(x, _enc(block=8))
