"""Pins of the oracle's relaxed model and its derivatives.

The relaxed model replaces the integer decode by its real-valued analogue:
real dequantised residuals for every SRV value and real per-block shifts
(the motion vectors of Phase-shifted Motion Compensation divided by 4),
bilinear prediction without rounding, a linear colour inverse, no clamps.
The loss sum((render - target)^2) is then exactly quadratic in the residuals
and piecewise quadratic in each shift, so central differences are exact up
to round-off away from the bilinear kinks.  Three independent derivatives
must agree: central differences, forward-mode dual numbers and the explicit
reverse-mode transpose; the transpose also passes the dot-product test.
"""

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def relaxed_setup(tiny_oracle, tiny_lf, tiny_cams_ez):
    o = tiny_oracle
    res, sh = o.export_params()
    sh = sh + np.float32(0.125)  # keep every tap away from an integer position (kink)
    cams = tiny_cams_ez
    target = oracle.render_dense(tiny_lf, cams, 64, 64).astype(np.float32)
    return o, res, sh, cams, target


def _touched(o, res, sh, cams, target, kind, rng, want):
    out = []
    n = res.size if kind == 0 else sh.size
    tries = 0
    while len(out) < want and tries < 4000:
        tries += 1
        idx = int(rng.integers(0, n))
        fd, fwd, hits = o.param_check(res, sh, cams, 64, 64, target, kind, idx)
        if hits > 0 and abs(fwd) > 1e-8:
            out.append((idx, fd, fwd))
    return out


def test_fd_equals_forward_mode(relaxed_setup):
    o, res, sh, cams, target = relaxed_setup
    rng = np.random.default_rng(0)
    for kind in (0, 1):
        got = _touched(o, res, sh, cams, target, kind, rng, 12)
        assert len(got) >= 8
        for idx, fd, fwd in got:
            assert abs(fd - fwd) <= 1e-6 * max(1.0, abs(fwd)), (kind, idx, fd, fwd)


def test_reverse_mode_equals_forward_mode(relaxed_setup):
    o, res, sh, cams, target = relaxed_setup
    out = o.render_relaxed(res, sh, cams, 64, 64)
    g_res, g_sh = o.relaxed_grad(res, sh, cams, 64, 64, 2.0 * (out - target))
    rng = np.random.default_rng(1)
    for kind, g in ((0, g_res.ravel()), (1, g_sh.ravel())):
        for idx, fd, fwd in _touched(o, res, sh, cams, target, kind, rng, 12):
            assert abs(g[idx] - fwd) <= 1e-9 * max(1.0, abs(fwd)), (kind, idx, g[idx], fwd)
    # parameters no ray depends on get exactly zero
    assert np.count_nonzero(g_res) < g_res.size


def test_adjoint_dot_product(relaxed_setup):
    o, res, sh, cams, target = relaxed_setup
    rng = np.random.default_rng(2)
    v = rng.normal(size=res.shape).astype(np.float32)
    w = rng.normal(size=(cams.shape[0], 3, 64, 64))
    base = o.render_relaxed(res, sh, cams, 64, 64)
    # the render is affine in the residuals: J v = render(r + v) - render(r) (in float64
    # on float32 parameters, so r + v is formed exactly in float64 before narrowing)
    rv = (res.astype(np.float64) + v).astype(np.float32)
    dv = (rv.astype(np.float64) - res.astype(np.float64))
    Jv = o.render_relaxed(rv, sh, cams, 64, 64) - base
    g_res, _ = o.relaxed_grad(res, sh, cams, 64, 64, w)
    lhs = float(np.sum(Jv * w))
    rhs = float(np.sum(dv * g_res))
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs))


def test_residual_gradient_linear(relaxed_setup):
    o, res, sh, cams, target = relaxed_setup
    rng = np.random.default_rng(3)
    w = rng.normal(size=(cams.shape[0], 3, 64, 64))
    g1, s1 = o.relaxed_grad(res, sh, cams, 64, 64, w)
    g2, s2 = o.relaxed_grad(res, sh, cams, 64, 64, 2.0 * w)
    assert np.allclose(g2, 2.0 * g1, rtol=1e-12, atol=1e-12)
    # the residual gradient does not depend on the residual values themselves
    g3, _ = o.relaxed_grad(res * np.float32(0.5), sh, cams, 64, 64, w)
    assert np.allclose(g3, g1, rtol=1e-12, atol=1e-12)


def test_relaxed_close_to_integer_render(tiny_oracle, tiny_cams):
    # At the exported parameters the relaxed model differs from the integer decode
    # only by the prediction rounding (<= 1/2 per predictive level and channel) and
    # the integer colour lifting (<= 1 per RGB value), plus clamping.
    o = tiny_oracle
    res, sh = o.export_params()
    a = o.render_relaxed(res, sh, tiny_cams, 64, 64)
    b = o.render(tiny_cams, 64, 64)
    bound = (1.0 + 0.5 * o.levels * 2.0) / 255.0
    assert np.abs(a - b).max() <= bound + 1e-12
    assert np.abs(a - b).mean() <= 0.5 / 255.0
