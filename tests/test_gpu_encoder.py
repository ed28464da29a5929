"""The GPU encoder against the oracle's encoder.

The two are written independently from the same definitions (YCoCg-R, the
2x2-cluster rounded-mean hierarchy, the top-down closed loop, the Eq. 1-2
search with its tie-breaks, quantisation, block thresholds, bounded-integer
sequence layout, breadth-first node order), so equal streams check both.
Every byte must match: the stream is integer data end to end.
"""

import numpy as np
import pytest

import lfscene
import oracle
from conftest import crop_lf, stream_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("over", [{}, {"step": 1}, {"zero_phase": True}, {"no_mc": True},
                                  {"step": 8, "t_ref": 200, "t_pred": 400}, {"subpel": False},
                                  {"block": 2}, {"block": 4}, {"block": 32}, {"block": 64, "win": 8},
                                  {"block": 1, "no_mc": True}, {"step": 4096}, {"win": 0}])
def test_encoder_tiny(torch_mod, tiny_lf, over):
    from paper_1902_09396_amd import lf

    enc = lfscene.get_config("tiny", **over)["enc"]
    got = lf.encode(tiny_lf, enc)
    exp = stream_for("tiny", tiny_lf, **over)
    assert got.size == exp.size and np.array_equal(got, exp), over


def test_encoder_mid(torch_mod, mid_lf, mid_stream):
    from paper_1902_09396_amd import lf

    assert np.array_equal(lf.encode(mid_lf, lfscene.get_config("path512")["enc"]), mid_stream)


def test_encoder_odd_grids(torch_mod):
    """Ragged clusters at every level, per-level steps, windows and thresholds."""
    from paper_1902_09396_amd import lf

    x = crop_lf("tiny", 7, 5, 16, 24)
    enc = lfscene.get_config("tiny")["enc"]
    enc.update(levels=3, block=4, step=[3, 2, 5], win=[2, 1, 3], t_ref=[10, 0, 0], t_pred=[30, 5, 0])
    assert np.array_equal(lf.encode(x, enc), oracle.encode(x, enc))
    x = crop_lf("tiny", 1, 3, 8, 8)  # one column: no predictive node in even rows
    enc.update(levels=2, block=2, step=[1, 1], win=[1, 2], t_ref=[0, 0], t_pred=[0, 0])
    assert np.array_equal(lf.encode(x, enc), oracle.encode(x, enc))
    x = crop_lf("tiny", 1, 1, 8, 8)  # a single view: no predictive node at all
    assert np.array_equal(lf.encode(x, enc), oracle.encode(x, enc))


def test_encoder_full_range_content(torch_mod):
    """Random RGB (every channel over its whole range, no spatial structure):
    the largest SRV magnitudes, widest blocks and every BISE family."""
    from paper_1902_09396_amd import lf

    rng = np.random.default_rng(17)
    x = rng.integers(0, 256, (5, 6, 16, 32, 3), dtype=np.uint8)
    x[0, 0] = 255
    x[1, 1] = 0
    enc = lfscene.get_config("tiny")["enc"]
    for over in (dict(levels=2, block=8, step=[1, 1], win=[2, 3]), dict(levels=3, block=4, step=[7, 3, 2],
                                                                        win=[1, 1, 2], zero_phase=True)):
        e = dict(enc, **over)
        e["t_ref"], e["t_pred"] = [0] * e["levels"], [0] * e["levels"]
        assert np.array_equal(lf.encode(x, e), oracle.encode(x, e)), over


def test_encoder_rejects(torch_mod, tiny_lf):
    from paper_1902_09396_amd import lf

    x = crop_lf("tiny", 7, 5, 16, 24)
    enc = lfscene.get_config("tiny")["enc"]
    for over in (dict(block=3), dict(block=128), dict(win=[60, 4]), dict(step=[0, 4]), dict(step=[4097, 4]),
                 dict(block=1)):  # a search needs 2x2 blocks
        with pytest.raises(lf.LFError) as e:
            lf.encode(x, dict(enc, **over))
        assert e.value.status == lf.LF_EINVAL, over
