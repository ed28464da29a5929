"""The library's host encoder and the oracle's encoder are written
independently from the same definitions (closed-loop hierarchy, Eq. 1-2
search with the stated tie-breaks, quantisation, thresholds, BISE layout);
they must emit byte-identical streams."""

import numpy as np
import pytest

import lfscene
import oracle
from conftest import crop_lf, stream_for


@pytest.mark.parametrize("over", [{}, {"step": 1}, {"zero_phase": True}, {"no_mc": True},
                                  {"step": 8, "t_ref": 200, "t_pred": 400}, {"subpel": False}])
def test_identical_streams_tiny(tiny_lf, over):
    from paper_1902_09396_amd import lf

    enc = lfscene.get_config("tiny", **over)["enc"]
    assert np.array_equal(lf.encode(tiny_lf, enc), stream_for("tiny", tiny_lf, **over))


def test_identical_streams_mid(mid_lf, mid_stream):
    from paper_1902_09396_amd import lf

    assert np.array_equal(lf.encode(mid_lf, lfscene.get_config("path512")["enc"]), mid_stream)


def test_identical_streams_odd_grid():
    from paper_1902_09396_amd import lf

    x = crop_lf("tiny", 7, 5, 16, 24)
    enc = lfscene.get_config("tiny")["enc"]
    enc.update(levels=3, block=4, step=[3, 2, 5], win=[2, 1, 3], t_ref=[10, 0, 0], t_pred=[30, 5, 0])
    assert np.array_equal(lf.encode(x, enc), oracle.encode(x, enc))


def test_encoder_rejects_bad_geometry(tiny_lf):
    from paper_1902_09396_amd import lf

    enc = lfscene.get_config("tiny")["enc"]
    enc.update(block=7)  # 64 is not a multiple of 7
    with pytest.raises(lf.LFError) as e:
        lf.encode(tiny_lf, enc)
    assert e.value.status == lf.LF_EINVAL
