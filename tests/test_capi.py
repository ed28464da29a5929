"""The C-ABI library loads, exports every declared entry point, and its
host-only calls validate streams (no GPU needed)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "hmlfc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1902_09396_amd import lf, serve

    L = lf.lib()
    names = _declared()
    assert "lf_render_views" in names and "lf_decode_pixels" in names
    for n in names:
        assert hasattr(L, n), n
    # the binding declares a signature for every entry point of the header
    assert set(names) <= set(lf.SIGNATURES) | set(serve._SIGS)


def test_query_arena_and_format_errors(tiny_stream):
    from paper_1902_09396_amd import lf

    need = lf.query_arena(tiny_stream)
    assert need > tiny_stream.size  # stream sections plus resident reference planes
    bad = tiny_stream.copy()
    bad[3] ^= 0x55
    with pytest.raises(lf.LFError) as e:
        lf.query_arena(bad)
    assert e.value.status == lf.LF_EFORMAT
    with pytest.raises(lf.LFError):
        lf.query_arena(tiny_stream[:1500])
    bad = tiny_stream.copy()
    bad[120:128] = np.frombuffer(np.uint64(7).tobytes(), np.uint8)  # root size
    with pytest.raises(lf.LFError):
        lf.query_arena(bad)
    # a block offset pointing past the payload
    table_off = int(np.frombuffer(tiny_stream[128:136].tobytes(), np.uint64)[0])
    bad = tiny_stream.copy()
    for e in range(64):
        if bad[table_off + 8 * e + 6] != 0xFF:
            bad[table_off + 8 * e:table_off + 8 * e + 4] = np.frombuffer(np.uint32(0xFFFFFF00).tobytes(), np.uint8)
            break
    with pytest.raises(lf.LFError):
        lf.query_arena(bad)
