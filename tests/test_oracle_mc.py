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


# ---------------------------------------------------------------------------
# Brute force over every quarter-pel position of the window (Eq. 1 and 2 with
# the sub-pel prediction of Future Work).  The prediction is evaluated here on
# an edge-padded copy of the reference (np.pad, mode "edge"), not by clamping
# indices; it is pinned on closed forms first.

def _qpel_all(R, by0, bx0, bs, mx, my):
    """sigma-free quarter-pel prediction of the block at (by0, bx0)."""
    pad = 64
    Rp = np.pad(R.astype(np.int64), pad, mode="edge")
    ys = 4 * np.arange(by0, by0 + bs)[:, None] + my
    xs = 4 * np.arange(bx0, bx0 + bs)[None, :] + mx
    y0, x0 = np.floor_divide(ys, 4), np.floor_divide(xs, 4)
    fy, fx = ys - 4 * y0, xs - 4 * x0
    t00 = Rp[y0 + pad, x0 + pad]
    t01 = Rp[y0 + pad, x0 + 1 + pad]
    t10 = Rp[y0 + 1 + pad, x0 + pad]
    t11 = Rp[y0 + 1 + pad, x0 + 1 + pad]
    acc = (4 - fx) * (4 - fy) * t00 + fx * (4 - fy) * t01 + (4 - fx) * fy * t10 + fx * fy * t11
    return np.floor_divide(acc + 8, 16)


def test_bruteforce_prediction_closed_forms():
    # a linear plane is reproduced exactly at every quarter-pel shift (bilinear
    # interpolation of a linear function is exact, the weights sum to 16)
    yy, xx = np.mgrid[0:16, 0:16]
    R = 16 * xx - 32 * yy + 5
    for mx in range(-6, 7):
        for my in range(-6, 7):
            got = _qpel_all(R, 4, 4, 8, mx, my)
            want = 16 * (xx[4:12, 4:12] + mx / 4) - 32 * (yy[4:12, 4:12] + my / 4) + 5
            assert np.array_equal(got, want.astype(np.int64))
    # beyond the border the edge sample is replicated
    C = _plane(9, 8, 8)
    assert np.array_equal(_qpel_all(C, 0, 0, 8, -40, -40), np.full((8, 8), C[0, 0]))


def _search_by_definition(P, R, by0, bx0, bs, win, zero_phase=False):
    """Per phase: the key-minimum over whole-pixel shifts, then over those plus
    the quarter-pel shifts within +-3 of it (inside the window); phase -1 only
    on a strictly lower cost; the zero phase only when strictly cheaper."""
    lim = 4 * win
    blk = P[by0:by0 + bs, bx0:bx0 + bs].astype(np.int64)
    pred = {(mx, my): _qpel_all(R, by0, bx0, bs, mx, my)
            for my in range(-lim, lim + 1) for mx in range(-lim, lim + 1)}
    best = []
    for sgn in (1, -1):
        cost = {m: int(np.abs(blk - sgn * q).sum()) for m, q in pred.items()}
        key = lambda m: (cost[m], abs(m[0]) + abs(m[1]), m[1], m[0])  # noqa: E731
        whole = [m for m in cost if m[0] % 4 == 0 and m[1] % 4 == 0]
        c0 = min(whole, key=key)
        near = [m for m in cost if abs(m[0] - c0[0]) <= 3 and abs(m[1] - c0[1]) <= 3]
        b = min(whole + near, key=key)
        best.append((cost[b], b[0], b[1], sgn, min(cost.values())))
    r = best[1] if best[1][0] < best[0][0] else best[0]
    if zero_phase and int(np.abs(blk).sum()) < r[0]:
        return (int(np.abs(blk).sum()), 0, 0, 0), None
    return r[:4], r[4]


@pytest.mark.parametrize("seed,by0,bx0,bs,win", [
    (20, 4, 4, 4, 2), (21, 0, 0, 4, 2), (22, 12, 8, 4, 1), (23, 6, 10, 2, 3), (24, 0, 12, 4, 2)])
def test_search_bruteforce_quarter_pel(seed, by0, bx0, bs, win):
    # noisy planes: ties and near-ties are common, so every branch of the rule runs
    R = _plane(seed, 16, 16, -9, 9)
    P = _plane(seed + 100, 16, 16, -9, 9)
    want, _ = _search_by_definition(P, R, by0, bx0, bs, win)
    assert oracle.mc_search(P, R, by0, bx0, bs, win=win) == want
    want0, _ = _search_by_definition(P, R, by0, bx0, bs, win, zero_phase=True)
    assert oracle.mc_search(P, R, by0, bx0, bs, win=win, zero_phase=True) == want0


@pytest.mark.parametrize("mx,my,sign", [(5, -3, 1), (-6, 7, -1), (2, 2, 1), (-1, -7, -1), (7, 1, 1)])
def test_search_global_quarter_pel_optimum(mx, my, sign):
    # A smooth reference and a block that is its phase-signed quarter-pel shift:
    # the global minimum over every quarter-pel position of the window is 0 at
    # the true shift, and the search reaches it.
    rng = np.random.default_rng(30 + mx)
    R = np.cumsum(np.cumsum(rng.integers(-2, 3, size=(24, 24)), 0), 1).astype(np.int32) * 3
    by0, bx0, bs, win = 8, 8, 4, 2
    P = np.zeros_like(R)
    P[by0:by0 + bs, bx0:bx0 + bs] = sign * _qpel_all(R, by0, bx0, bs, mx, my)
    want, global_min = _search_by_definition(P, R, by0, bx0, bs, win)
    assert global_min == 0 and want[0] == 0 and want[3] == sign
    got = oracle.mc_search(P, R, by0, bx0, bs, win=win)
    assert got == want
    assert np.array_equal(got[3] * _qpel_all(R, by0, bx0, bs, got[1], got[2]), P[by0:by0 + bs, bx0:bx0 + bs])
