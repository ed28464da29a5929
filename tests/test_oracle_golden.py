"""Regression fixture of the oracle (tests/golden/tiny_oracle.json, written
by tests/golden/make_golden.py from the oracle alone): the stream bytes,
sampled decoded and level-1 node samples, and rendered pixels of the seeded
8x8x64x64 scene must not change unless the oracle's arithmetic is changed on
purpose (and the fixture regenerated with it)."""

import json
import os

import numpy as np

from conftest import ROOT

GOLDEN = os.path.join(ROOT, "tests", "golden")


def test_oracle_matches_golden_fixture():
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    want = json.load(open(os.path.join(GOLDEN, "tiny_oracle.json")))
    got = mod.golden()
    for k in ("stream_bytes", "stream_sha256", "coords", "decode_rgb", "level1_rgb"):
        assert got[k] == want[k], k
    assert abs(got["render_16x16_first_two_views_sum"] - want["render_16x16_first_two_views_sum"]) <= 1e-9
    assert np.allclose(got["render_16x16_pixel_0_5_7"], want["render_16x16_pixel_0_5_7"], rtol=0, atol=1e-12)
