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


def _sparse_arena_expected(stream):
    """Arena of a sparse-residency load, derived from the stream header and
    table: [root][table][payload][mv][tiles][slots][status], 256-aligned."""
    s = np.asarray(stream, dtype=np.uint8)
    rd = lambda o, t: int(np.frombuffer(s[o:o + np.dtype(t).itemsize].tobytes(), t)[0])  # noqa: E731
    na, nb, w, h, H, bs = (rd(16 + 4 * k, np.int32) for k in range(6))
    al = lambda v: (v + 255) // 256 * 256  # noqa: E731
    root, table, payload, mv = (rd(120 + 16 * k, np.uint64) for k in range(4))
    na_l, nb_l = [na], [nb]
    for _ in range(H):
        na_l.append((na_l[-1] + 1) // 2)
        nb_l.append((nb_l[-1] + 1) // 2)
    node_base, n = {}, 0
    for lev in range(H - 1, -1, -1):
        node_base[lev] = n
        n += na_l[lev] * nb_l[lev]
    nblk = (w // bs) * (h // bs)
    toff = rd(128, np.uint64)
    modes = s[toff:toff + table].reshape(3, n, nblk, 8)[..., 6]
    tiles = 0
    n_refs = 0
    for lev in range(H):
        refs = [node_base[lev] + 2 * B * na_l[lev] + 2 * A for B in range(nb_l[lev + 1]) for A in range(na_l[lev + 1])]
        n_refs += len(refs)
        tiles += int((modes[:, refs, :] != 0xFF).sum())
    a = al(al(al(al(root) + table) + payload) + mv)
    a = al(al(a + tiles * bs * bs * 2) + 3 * n_refs * nblk * 4)
    return a + 256, tiles


def test_sparse_residency_arena(tiny_lf, tiny_stream):
    from conftest import stream_for
    from paper_1902_09396_amd import lf

    for s in (tiny_stream, stream_for("tiny", tiny_lf, step=8, t_ref=200, t_pred=400)):
        expect, tiles = _sparse_arena_expected(s)
        assert lf.query_arena(s, sparse_refs=True) == expect
        assert tiles > 0
    dense, sparse = lf.query_arena(s), lf.query_arena(s, sparse_refs=True)
    assert sparse < dense  # thresholds zero many reference blocks; no descriptors either
    with pytest.raises(lf.LFError) as e:  # unknown load flags
        lf.check(lf.lib().lf_query_arena_ex(s.ctypes.data_as(C.c_void_p), s.size, 6, C.byref(C.c_int64())))
    assert e.value.status == lf.LF_EINVAL


def test_encode_workspace_bytes():
    """Encoder workspace, as the header states it: 256-aligned sections for the
    uploaded field, the YCoCg planes of every level, level-0 coded SRVs,
    quantised values, 28 bytes per block of bookkeeping, prefix-sum tiles,
    motion records, level-0 search items, the 16-bit payload bound and the
    motion-vector words."""
    from paper_1902_09396_amd import lf

    import lfscene

    al = lambda v: (v + 255) // 256 * 256  # noqa: E731
    for name, over in (("tiny", {}), ("path512", {}), ("tiny", {"no_mc": True}), ("tiny", {"block": 2})):
        cfg = lfscene.get_config(name, **over)
        L, enc = cfg["lf"], cfg["enc"]
        na, nb, h, w, bs, H = L["na"], L["nb"], L["h"], L["w"], enc["block"], enc["levels"]
        n, nblk, plane = bs * bs, (w // bs) * (h // bs), w * h
        grids = [(na, nb)]
        for _ in range(H):
            grids.append(((grids[-1][0] + 1) // 2, (grids[-1][1] + 1) // 2))
        views = [a * b for a, b in grids]
        nent = 3 * sum(views[:H]) * nblk
        npred = [((b // 2) * a + ((b + 1) // 2) * (a // 2)) * nblk for a, b in grids[:H]]
        mv_words = 0
        for _ in range(3):
            for l in range(H):
                vmax, cnt = 8 * enc["win"][l], 2 * npred[l]
                sizes = []
                for fam, m in enumerate((1, 3, 5)):
                    b = (vmax // m).bit_length()
                    sizes.append(cnt * b if fam == 0 else (-(-cnt // 5) * (8 + 5 * b) if fam == 1
                                                           else -(-cnt // 3) * (7 + 3 * b)))
                mv_words += -(-min(sizes) // 32) + -(-cnt // 32)
        tiles = -(-nent // 4096)
        expect = (al(256) + al(views[0] * plane * 3) + sum(al(3 * v * plane * 2) for v in views)
                  + al(3 * views[0] * plane * 2) + al(nent * n * 2) + al(nent * 8) + al(nent * 4) + al(nent * 8)
                  + al(nent * 8) + al((tiles + 1) * 8) + al(3 * sum(npred) * 16) + al(3 * npred[0] * 12)
                  + al(nent * (-(-16 * n // 32)) * 4) + al(mv_words * 4))
        got = C.c_int64()
        p = lf._encode_params(enc)
        lf.check(lf.lib().lf_encode_workspace_bytes(L["nb"], L["na"], h, w, C.byref(p), C.byref(got)))
        assert got.value == expect, (name, over)


def test_encode_rejects_on_the_host():
    """Parameter checks happen before any device work."""
    from paper_1902_09396_amd import lf

    import lfscene

    cfg = lfscene.get_config("tiny")
    L = cfg["lf"]
    for over in ({"block": 3}, {"block": 128}, {"step": 0}, {"step": 5000}, {"win": 60}, {"win": 300},
                 {"block": 1}):
        enc = lfscene.get_config("tiny", **over)["enc"]
        p = lf._encode_params(enc)
        with pytest.raises(lf.LFError) as e:
            lf.check(lf.lib().lf_encode_workspace_bytes(L["nb"], L["na"], L["h"], L["w"], C.byref(p),
                                                        C.byref(C.c_int64())))
        assert e.value.status == lf.LF_EINVAL, over


def test_parse_bounds_residual_ranges():
    """A block whose mode can hold a dequantised residual beyond 2^24 is a
    format error (the decoders' int32 sums could wrap); the bound counts
    every value the mode can hold, (min + cap - 1) * step, not only the
    stored ones.  Streams written from the format alone (tests/streamkit)."""
    from paper_1902_09396_amd import lf
    from streamkit import Craft

    def stream(mn, b, step):
        k = Craft(na=2, nb=2, w=8, h=8, levels=1, block=4, step=[step], win=[2])
        k.set_block_raw(0, 0, 0, 1, 0, mn, b, np.zeros(16, dtype=np.int64))
        return k.build()

    def arena(s):
        need = C.c_int64()
        lf.check(lf.lib().lf_query_arena(s.ctypes.data_as(C.c_void_p), s.size, C.byref(need)))
        return need.value

    assert arena(stream(0, 12, 4096)) > 0          # (2^12 - 1) * 4096 < 2^24
    assert arena(stream(-4096, 0, 4096)) > 0        # |min * step| = 2^24 exactly
    for mn, b, step in ((0, 20, 4096), (0, 13, 4096), (-4097, 0, 4096), (-32768, 10, 1024), (32000, 15, 1024)):
        with pytest.raises(lf.LFError) as e:
            arena(stream(mn, b, step))
        assert e.value.status == lf.LF_EFORMAT, (mn, b, step)


def test_parse_chroma_formats():
    """A 4:2:0 stream parses (its root and table sections are sized by the
    half-size chroma planes); an unknown chroma format, or a 4:4:4 stream
    relabelled 4:2:0 (sections no longer match), is a format error."""
    from paper_1902_09396_amd import lf

    import lfscene
    import oracle
    from conftest import lf_for

    x = lf_for("tiny")
    enc = lfscene.get_config("tiny")["enc"]
    s444 = oracle.encode(x, enc)
    s420 = oracle.encode(x, dict(enc, chroma420=True))

    def arena(s):
        need = C.c_int64()
        lf.check(lf.lib().lf_query_arena(s.ctypes.data_as(C.c_void_p), s.size, C.byref(need)))
        return need.value

    assert 0 < arena(s420) < arena(s444)  # half-size chroma references, no descriptors
    for stream, flag in ((s420, 2), (s444, 1)):
        bad = stream.copy()
        bad[560:564] = np.frombuffer(np.uint32(flag).tobytes(), np.uint8)
        with pytest.raises(lf.LFError) as e:
            arena(bad)
        assert e.value.status == lf.LF_EFORMAT
    with pytest.raises(lf.LFError) as e:  # sparse residency is for full-size chroma
        lf.check(lf.lib().lf_query_arena_ex(s420.ctypes.data_as(C.c_void_p), s420.size, lf.LF_LOAD_SPARSE_REFS,
                                            C.byref(C.c_int64())))
    assert e.value.status == lf.LF_EINVAL


def test_csr_residency_arena(tiny_lf):
    """CSR residency reserves 4 bytes per pixel of every significant
    reference block (values and columns; the nonzero count is known only
    after decoding) and a row start for every reference row; combined with
    block tiles it is rejected."""
    from conftest import stream_for
    from paper_1902_09396_amd import lf

    s = stream_for("tiny", tiny_lf, step=8, t_ref=200, t_pred=400)
    sparse, tiles = _sparse_arena_expected(s)
    al = lambda v: (v + 255) // 256 * 256  # noqa: E731
    rd = lambda o: int(np.frombuffer(s[o:o + 8].tobytes(), np.uint64)[0])  # noqa: E731
    a = al(al(al(al(rd(120)) + rd(136)) + rd(152)) + rd(168))  # root, table, payload, mv
    bound = tiles * 8 * 8
    n_refs = 4 * 4 + 2 * 2  # reference nodes of the 8x8 grid's two levels
    expect = al(al(al(a + 2 * bound) + 2 * bound) + 4 * (3 * n_refs * 64 + 1)) + 256
    assert lf.query_arena(s, csr_refs=True) == expect
    with pytest.raises(lf.LFError) as e:
        lf.query_arena(s, sparse_refs=True, csr_refs=True)
    assert e.value.status == lf.LF_EINVAL
