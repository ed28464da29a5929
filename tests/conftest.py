import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


import lfscene  # noqa: E402
import oracle  # noqa: E402

_CACHE = {}


def lf_for(name: str, **spec_over) -> np.ndarray:
    cfg = lfscene.get_config(name)
    L = cfg["lf"]
    spec = dict(L["spec"], **spec_over)
    key = ("lf", name, tuple(sorted(spec_over.items())))
    if key not in _CACHE:
        _CACHE[key] = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], spec, L["seed"])
    return _CACHE[key]


def stream_for(name: str, lf: np.ndarray | None = None, tag: str = "", **enc_over) -> np.ndarray:
    """Oracle-encoded stream of a config (cached per session)."""
    key = ("stream", name, tag, tuple(sorted((k, str(v)) for k, v in enc_over.items())))
    if key not in _CACHE:
        cfg = lfscene.get_config(name, **enc_over)
        if lf is None:
            lf = lf_for(name)
        _CACHE[key] = oracle.encode(lf, cfg["enc"])
    return _CACHE[key]


def crop_lf(name: str, na: int, nb: int, h: int, w: int) -> np.ndarray:
    """A corner crop of a config's light field (same scene statistics, smaller)."""
    key = ("crop", name, na, nb, h, w)
    if key not in _CACHE:
        full = lf_for(name) if name != "path512" else _path512_small()
        _CACHE[key] = np.ascontiguousarray(full[:nb, :na, :h, :w])
    return _CACHE[key]


def _path512_small():
    # The path512 scene rendered at 17x17x128x128 (its layer layout scaled to 128^2).
    key = ("lf", "path512-128")
    if key not in _CACHE:
        cfg = lfscene.get_config("path512")
        L = cfg["lf"]
        _CACHE[key] = lfscene.make_lf(L["na"], L["nb"], 128, 128, L["spec"], L["seed"])
    return _CACHE[key]


@pytest.fixture(scope="session")
def tiny_lf():
    return lf_for("tiny")


@pytest.fixture(scope="session")
def tiny_stream(tiny_lf):
    return stream_for("tiny", tiny_lf)


@pytest.fixture(scope="session")
def tiny_oracle(tiny_stream):
    return oracle.OracleLF(tiny_stream)


@pytest.fixture(scope="session")
def tiny_cams():
    return lfscene.make_views(lfscene.get_config("tiny"))


@pytest.fixture(scope="session")
def tiny_cams_ez():
    """Four pinhole cameras with ez != 0 (rays sweep across views) over the tiny grid."""
    return lfscene.random_pinhole_cameras(4, 8, 8, 64, 64, 64, 64, seed=13, ez_range=(-1.0, 0.5),
                                          zoom_range=(0.6, 1.2), rho=1.0 / 16.0)


@pytest.fixture(scope="session")
def mid_lf():
    """17x17x128x128 crop-scale version of the 17x17x512^2 scene (4-level tree, 16x16 blocks)."""
    return _path512_small()


@pytest.fixture(scope="session")
def mid_stream(mid_lf):
    cfg = lfscene.get_config("path512")
    key = ("stream", "mid")
    if key not in _CACHE:
        _CACHE[key] = oracle.encode(mid_lf, cfg["enc"])
    return _CACHE[key]


@pytest.fixture(scope="session")
def mid_oracle(mid_stream):
    return oracle.OracleLF(mid_stream)
