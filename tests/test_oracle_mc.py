"""Pins of the oracle's quarter-pel prediction and phase-shifted search.

Phase-shifted Motion Compensation (Eq. 1 and 2 and the min/select rule):
a predictive block that is an exact (shifted) copy of the reference is found
with zero error and phase +1; a negated copy is found with phase -1 (the
additive error of Eq. 2).  Sub-pel prediction (Future Work: bilinear sub-pel
motion compensation): integer shifts copy exactly, a ramp is shifted by
exactly mx/4, a constant plane stays constant, half-pel taps round half up.
"""

import numpy as np
import pytest

import oracle


def _plane(seed, h=40, w=40, lo=-60, hi=60):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(h, w)).astype(np.int32)


def test_qpel_integer_shift_is_copy():
    R = _plane(0)
    for mx, my in [(0, 0), (4, 0), (-8, 4), (12, -12)]:
        for y, x in [(10, 10), (0, 0), (39, 39), (5, 37)]:
            yy = min(max(y + my // 4, 0), 39)
            xx = min(max(x + mx // 4, 0), 39)
            assert oracle.qpel(R, y, x, mx, my) == R[yy, xx]


def test_qpel_ramp_shift_exact():
    # plane(y, x) = 4x + 8y: bilinear weights sum to 16, so the interpolated value is
    # exactly 4(x + mx/4) + 8(y + my/4) = 4x + mx + 8y + 2my away from the borders.
    yy, xx = np.mgrid[0:32, 0:32]
    R = (4 * xx + 8 * yy).astype(np.int32)
    for mx in range(-7, 8):
        for my in range(-7, 8):
            assert oracle.qpel(R, 12, 15, mx, my) == 4 * 15 + mx + 8 * 12 + 2 * my


def test_qpel_constant_and_half_pel_rounding():
    C = np.full((8, 8), -37, dtype=np.int32)
    for mx in range(-9, 10):
        assert oracle.qpel(C, 3, 4, mx, 3 - mx) == -37
    R = np.zeros((4, 4), dtype=np.int32)
    R[1, 1], R[1, 2] = 1, 2
    # half-pel in x between 1 and 2: (8*1 + 8*2 + 8) >> 4 = 2 (round half up)
    assert oracle.qpel(R, 1, 1, 2, 0) == 2
    R[1, 1], R[1, 2] = -2, -1
    # (8*-2 + 8*-1 + 8) >> 4 = floor(-16/16) = -1
    assert oracle.qpel(R, 1, 1, 2, 0) == -1
    # quarter-pel: (12*-2 + 4*-1 + 8) >> 4 = floor(-20/16) = -2
    assert oracle.qpel(R, 1, 1, 1, 0) == -2


@pytest.mark.parametrize("dx,dy", [(0, 0), (3, -2), (-5, 4), (6, 6)])
def test_search_finds_exact_copy(dx, dy):
    R = _plane(1, 48, 48)
    P = np.zeros_like(R)
    by0, bx0, bs = 16, 16, 8
    for y in range(by0, by0 + bs):
        for x in range(bx0, bx0 + bs):
            P[y, x] = R[y + dy, x + dx]
    cost, mx, my, sg = oracle.mc_search(P, R, by0, bx0, bs, win=8)
    assert (cost, mx, my, sg) == (0, 4 * dx, 4 * dy, 1)


@pytest.mark.parametrize("dx,dy", [(2, 1), (-4, -3)])
def test_search_finds_negated_copy(dx, dy):
    R = _plane(2, 48, 48)
    P = np.zeros_like(R)
    by0, bx0, bs = 16, 24, 8
    for y in range(by0, by0 + bs):
        for x in range(bx0, bx0 + bs):
            P[y, x] = -R[y + dy, x + dx]
    cost, mx, my, sg = oracle.mc_search(P, R, by0, bx0, bs, win=6)
    assert (cost, mx, my, sg) == (0, 4 * dx, 4 * dy, -1)


@pytest.mark.parametrize("mx,my,sign", [(5, -3, 1), (-10, 7, -1), (2, 2, 1)])
def test_search_finds_subpel_copy(mx, my, sign):
    # smooth random reference so that sub-pel predictions are distinct
    rng = np.random.default_rng(3)
    R = np.cumsum(np.cumsum(rng.integers(-3, 4, size=(48, 48)), 0), 1).astype(np.int32)
    P = np.zeros_like(R)
    by0, bx0, bs = 16, 16, 8
    for y in range(by0, by0 + bs):
        for x in range(bx0, bx0 + bs):
            P[y, x] = sign * oracle.qpel(R, y, x, mx, my)
    cost, fmx, fmy, sg = oracle.mc_search(P, R, by0, bx0, bs, win=4)
    assert cost == 0 and sg == sign
    # the found vector reproduces the block exactly
    for y in range(by0, by0 + bs):
        for x in range(bx0, bx0 + bs):
            assert sg * oracle.qpel(R, y, x, fmx, fmy) == P[y, x]


def test_search_zero_phase_option():
    R = _plane(4)
    P = np.zeros_like(R)
    P[8:16, 8:16] = 1  # almost nothing to predict: sigma = 0 wins when allowed
    cost, mx, my, sg = oracle.mc_search(P, R, 8, 8, 8, win=2, zero_phase=True)
    assert (mx, my, sg) == (0, 0, 0) and cost == 64
    cost2, _, _, sg2 = oracle.mc_search(P, R, 8, 8, 8, win=2, zero_phase=False)
    assert sg2 in (1, -1) and cost2 >= cost


def test_search_window_brute_force_integer():
    # With sub-pel off, the result is the argmin over the integer window of
    # min(Eq. 1, Eq. 2) with phase +1 preferred on ties; check it against a direct
    # NumPy evaluation of both sums over every (dx, dy).
    R = _plane(5, 32, 32, -20, 20)
    P = _plane(6, 32, 32, -20, 20)
    by0, bx0, bs, win = 12, 12, 4, 3
    best = None
    for sgn in (1, -1):
        for dy in range(-win, win + 1):
            for dx in range(-win, win + 1):
                ref = R[by0 + dy:by0 + dy + bs, bx0 + dx:bx0 + dx + bs]
                cost = int(np.abs(P[by0:by0 + bs, bx0:bx0 + bs] - sgn * ref).sum())
                key = (cost, 0 if sgn == 1 else 1, abs(dx) + abs(dy), dy, dx)
                if best is None or key < best[0]:
                    best = (key, 4 * dx, 4 * dy, sgn)
    cost, mx, my, sg = oracle.mc_search(P, R, by0, bx0, bs, win=win, subpel=False)
    assert (cost, mx, my, sg) == (best[0][0], best[1], best[2], best[3])
