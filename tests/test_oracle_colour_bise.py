"""Pins of the oracle's colour transform and bounded-integer-sequence coding.

Colour (Compressing HMLFC tree: YCoCg decorrelation, dynamic range adjusted
so that nothing is lost): the reversible lifting must invert exactly on every
24-bit RGB value and agree with the real-valued YCoCg matrix up to its
rounding.  BISE (Bounded Integer Sequence Encoding): sizes equal the closed
forms, every mode round-trips, random access equals sequential decoding, and
a hand-worked trit/quint group has the documented bit layout.
"""

import numpy as np
import pytest

import oracle


def test_ycocg_exhaustive_roundtrip():
    v = np.arange(1 << 24, dtype=np.int64)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], axis=1).astype(np.int32)
    ycc = oracle.ycocg_fwd(rgb)
    back = oracle.ycocg_inv(ycc)
    assert np.array_equal(back, rgb)
    # dynamic range: Y in [0, 255], Co and Cg in [-255, 255]
    assert ycc[:, 0].min() == 0 and ycc[:, 0].max() == 255
    assert ycc[:, 1].min() == -255 and ycc[:, 1].max() == 255
    assert ycc[:, 2].min() == -255 and ycc[:, 2].max() == 255


def test_ycocg_matches_real_matrix():
    # Real YCoCg: Y = R/4 + G/2 + B/4, Co = R - B, Cg = G - (R + B)/2 (Co, Cg unscaled as in
    # the lifting form).  The integer lifting only floors two halvings.
    rng = np.random.default_rng(1)
    rgb = rng.integers(0, 256, size=(100000, 3)).astype(np.int32)
    ycc = oracle.ycocg_fwd(rgb).astype(np.float64)
    R, G, B = (rgb[:, i].astype(np.float64) for i in range(3))
    assert np.array_equal(ycc[:, 1], R - B)
    assert np.all(np.abs(ycc[:, 2] - (G - (R + B) / 2)) <= 0.5)
    assert np.all(np.abs(ycc[:, 0] - (R / 4 + G / 2 + B / 4)) <= 0.75)


def _modes():
    out = []
    for fam in range(3):
        for b in range(0, 12):
            out.append((fam << 5) | b)
    return out


@pytest.mark.parametrize("n", [1, 4, 5, 6, 64, 255, 256])
def test_bise_sizes_closed_form(n):
    for mode in _modes():
        fam, b = mode >> 5, mode & 31
        expect = {0: n * b, 1: -(-n // 5) * (8 + 5 * b), 2: -(-n // 3) * (7 + 3 * b)}[fam]
        assert oracle.bise_bits(mode, n) == expect


@pytest.mark.parametrize("n", [1, 3, 5, 7, 64, 256])
def test_bise_roundtrip_every_mode(n):
    rng = np.random.default_rng(n)
    for mode in _modes():
        fam, b = mode >> 5, mode & 31
        top = (1, 3, 5)[fam] << b
        v = rng.integers(0, top, size=n).astype(np.uint32)
        v[0] = top - 1  # include the largest value of the range
        words = oracle.bise_pack(v, mode)
        assert np.array_equal(oracle.bise_unpack(words, mode, n), v)
        for i in range(n):
            assert oracle.bise_get(words, mode, i) == v[i]


def test_bise_choose_is_smallest():
    rng = np.random.default_rng(7)
    for vmax in [0, 1, 2, 3, 4, 5, 6, 7, 9, 11, 15, 19, 23, 31, 40, 47, 63, 79, 95, 127, 500, 2047]:
        v = rng.integers(0, vmax + 1, size=256).astype(np.uint32)
        v[3] = vmax
        mode = oracle.bise_choose(v)
        fam, b = mode >> 5, mode & 31
        assert ((1, 3, 5)[fam] << b) > vmax
        best = min(oracle.bise_bits(m, 256) for m in _modes() if ((1, 3, 5)[m >> 5] << (m & 31)) > vmax)
        assert oracle.bise_bits(mode, 256) == best


def test_bise_trit_group_layout():
    # Five values with b = 1: high parts (trits) 0,1,2,0,1 and low bits 1,0,1,1,0.
    # Base-3 field = 0 + 1*3 + 2*9 + 0*27 + 1*81 = 102 in bits 0..7, then the
    # five low bits LSB-first in bits 8..12: 1,0,1,1,0 -> 0b01101 << 8.
    vals = np.array([0 * 2 + 1, 1 * 2 + 0, 2 * 2 + 1, 0 * 2 + 1, 1 * 2 + 0], dtype=np.uint32)
    words = oracle.bise_pack(vals, (1 << 5) | 1)
    assert int(words[0]) == 102 | (0b01101 << 8)


def test_bise_quint_group_layout():
    # Three values with b = 2: high parts (quints) 4,0,3 and low parts 3,1,2.
    # Base-5 field = 4 + 0*5 + 3*25 = 79 in bits 0..6, then 2-bit low parts.
    vals = np.array([4 * 4 + 3, 0 * 4 + 1, 3 * 4 + 2], dtype=np.uint32)
    words = oracle.bise_pack(vals, (2 << 5) | 2)
    assert int(words[0]) == 79 | (3 << 7) | (1 << 9) | (2 << 11)
