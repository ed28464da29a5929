"""Writes tiny_oracle.json: the oracle's stream digest, sampled decoded
samples, level-1 node samples and rendered pixels for the seeded 8x8x64x64
scene, so that any later change to the oracle's arithmetic shows up as a
test failure.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_golden.py
"""

import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lfscene  # noqa: E402
import oracle  # noqa: E402


def golden():
    cfg = lfscene.get_config("tiny")
    L = cfg["lf"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    stream = oracle.encode(light, cfg["enc"])
    o = oracle.OracleLF(stream)
    rng = np.random.default_rng(2024)
    coords = np.stack([rng.integers(0, L["nb"], 64), rng.integers(0, L["na"], 64), rng.integers(0, L["h"], 64),
                       rng.integers(0, L["w"], 64)], 1).astype(np.int32)
    nodes = coords.copy()
    nodes[:, :2] //= 2
    cams = lfscene.make_views(cfg)[:2]
    img = o.render(cams, 16, 16)
    return {
        "scene": "tiny (8x8 views of 64x64, seed %d), encoder settings of the tiny config" % L["seed"],
        "stream_bytes": int(stream.size),
        "stream_sha256": hashlib.sha256(stream.tobytes()).hexdigest(),
        "coords": coords.tolist(),
        "decode_rgb": o.decode_at(coords).tolist(),
        "level1_rgb": o.decode_node(1, nodes).tolist(),
        "render_16x16_first_two_views_sum": float(img.sum()),
        "render_16x16_pixel_0_5_7": [float(img[0, c, 5, 7]) for c in range(3)],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(golden(), f, indent=1)
    print("wrote", os.path.join(HERE, "tiny_oracle.json"))
