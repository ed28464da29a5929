"""Hand-built HMLFC streams for tests.

Written from the stream format alone (1024-byte header, int16 root RKVs,
8-byte block table in breadth-first node order, bounded-integer payloads,
per-(channel, level) motion-vector sequences and 2-bit phase codes), with no
search, quantiser or mode choice: the caller states every block's quantised
values, every motion record and the root planes.  Every payload and motion
sequence uses the plain b-bit family.  It shares no code with either encoder
and lets a test set what an encoder would decide (a vector at the border, an
insignificant block, a value at the edge of an integer range).
"""

from __future__ import annotations

import struct

import numpy as np

HDR = 1024
MAX_LEVELS = 8
ZERO = 0xFF


def pack_plain(values, b: int) -> list[int]:
    """LSB-first b-bit fields packed into 32-bit words."""
    acc, nbits, words = 0, 0, []
    for v in values:
        acc |= (int(v) & ((1 << b) - 1)) << nbits
        nbits += b
        while nbits >= 32:
            words.append(acc & 0xFFFFFFFF)
            acc >>= 32
            nbits -= 32
    if nbits:
        words.append(acc & 0xFFFFFFFF)
    return words


class Craft:
    def __init__(self, na, nb, w, h, levels, block, step, win):
        self.na, self.nb, self.w, self.h, self.H, self.bs = na, nb, w, h, levels, block
        self.step = list(step)
        self.win = list(win)
        self.na_l, self.nb_l = [na], [nb]
        for _ in range(levels):
            self.na_l.append((self.na_l[-1] + 1) // 2)
            self.nb_l.append((self.nb_l[-1] + 1) // 2)
        self.node_base = [0] * levels
        n = 0
        for l in range(levels - 1, -1, -1):
            self.node_base[l] = n
            n += self.na_l[l] * self.nb_l[l]
        self.n_nodes = n
        self.nbx = w // block
        self.nblk = self.nbx * (h // block)
        self.root = np.zeros((3, self.nb_l[levels], self.na_l[levels], h, w), dtype=np.int16)
        self.blocks = {}  # (c, node, blk) -> (min, mode, values)
        self.mvs = {}     # (c, l, record) -> (mx, my, sigma)
        self.mv_bits = {}  # (c, l) -> b of the motion sequence (default: fits 8W)

    # -- addressing
    def node(self, l, B, A):
        return self.node_base[l] + B * self.na_l[l] + A

    def npred(self, l):
        nal, nbl = self.na_l[l], self.nb_l[l]
        return ((nbl // 2) * nal + ((nbl + 1) // 2) * (nal // 2)) * self.nblk

    def record(self, l, B, A, blk):
        """Motion record of block blk of predictive node (B, A): predictive
        nodes of a level are counted in raster order."""
        k = 0
        for b in range(self.nb_l[l]):
            for a in range(self.na_l[l]):
                if (a | b) & 1:
                    if (b, a) == (B, A):
                        return k * self.nblk + blk
                    k += 1
        raise ValueError("(%d, %d) is not a predictive node of level %d" % (B, A, l))

    # -- content
    def set_block(self, c, l, B, A, blk, q):
        """Quantised values q (bs*bs, raster order in the block); the stored
        minimum is q.min() and the mode the plain family with the fewest bits."""
        q = np.asarray(q, dtype=np.int64).reshape(-1)
        assert q.size == self.bs * self.bs
        mn = int(q.min())
        b = int((q - mn).max()).bit_length()
        self.blocks[(c, self.node(l, B, A), blk)] = (mn, b, q - mn)

    def set_block_raw(self, c, l, B, A, blk, mn, b, v):
        """Stored minimum, plain-family bit count and offsets as given."""
        self.blocks[(c, self.node(l, B, A), blk)] = (int(mn), int(b), np.asarray(v, dtype=np.int64).reshape(-1))

    def set_mv(self, c, l, B, A, blk, mx, my, sigma):
        self.mvs[(c, l, self.record(l, B, A, blk))] = (mx, my, sigma)

    # -- stream
    def build(self) -> np.ndarray:
        H, plane = self.H, self.w * self.h
        n_ent = 3 * self.n_nodes * self.nblk
        table = bytearray(8 * n_ent)
        payload = []
        for e in range(n_ent):
            c, rest = divmod(e, self.n_nodes * self.nblk)
            node, blk = divmod(rest, self.nblk)
            if (c, node, blk) not in self.blocks:
                table[8 * e + 6] = ZERO
                continue
            mn, b, v = self.blocks[(c, node, blk)]
            struct.pack_into("<IhBB", table, 8 * e, len(payload), mn, b, 0)
            payload += pack_plain(v, b)
        payload += [0, 0]  # trailing slack
        mv_words, directory = [], {}
        for c in range(3):
            for l in range(H - 1, -1, -1):
                cnt = self.npred(l)
                b = self.mv_bits.get((c, l), (8 * self.win[l]).bit_length())
                vals, codes = [], []
                for j in range(cnt):
                    mx, my, sg = self.mvs.get((c, l, j), (0, 0, 1))
                    vals += [mx + 4 * self.win[l], my + 4 * self.win[l]]
                    codes.append({1: 0, -1: 1, 0: 2}[sg])
                first = len(mv_words)
                mv_words += pack_plain(vals, b)
                sig = len(mv_words)
                mv_words += pack_plain(codes, 2)
                directory[(c, l)] = (first, sig, cnt, b)
        mv_words += [0, 0]
        root = self.root.tobytes()
        o_root = HDR
        o_table = o_root + len(root)
        o_payload = o_table + len(table)
        o_mv = o_payload + 4 * len(payload)
        total = o_mv + 4 * len(mv_words)
        s = bytearray(total)
        s[0:8] = b"HMLFCv1\0"
        struct.pack_into("<II", s, 8, HDR, 1)
        struct.pack_into("<8i", s, 16, self.na, self.nb, self.w, self.h, H, self.bs, 3, 4)
        for l in range(H):
            struct.pack_into("<I", s, 48 + 4 * l, self.step[l])
            struct.pack_into("<I", s, 80 + 4 * l, self.win[l])
        struct.pack_into("<8Q", s, 112, o_root, len(root), o_table, len(table), o_payload, 4 * len(payload),
                         o_mv, 4 * len(mv_words))
        for (c, l), (first, sig, cnt, b) in directory.items():
            struct.pack_into("<IIIB", s, 176 + (c * MAX_LEVELS + l) * 16, first, sig, cnt, b)
        s[o_root:o_table] = root
        s[o_table:o_payload] = table
        s[o_payload:o_mv] = np.asarray(payload, dtype=np.uint32).tobytes()
        s[o_mv:total] = np.asarray(mv_words, dtype=np.uint32).tobytes()
        return np.frombuffer(bytes(s), dtype=np.uint8).copy()

    # -- what the stream means, straight from the content (Decoding Procedure)
    def srv_planes(self) -> np.ndarray:
        """Decoded SRV planes [3][n_nodes][h][w]: residual * step, plus the
        phase-signed quarter-pel prediction from the cluster's reference."""
        bs, out = self.bs, np.zeros((3, self.n_nodes, self.h, self.w), dtype=np.int64)
        for (c, node, blk), (mn, b, v) in self.blocks.items():
            l = next(l for l in range(self.H) if node >= self.node_base[l]
                     and node < self.node_base[l] + self.na_l[l] * self.nb_l[l])
            by, bx = (blk // self.nbx) * bs, (blk % self.nbx) * bs
            out[c, node, by:by + bs, bx:bx + bs] = ((mn + v) * self.step[l]).reshape(bs, bs)
        pad = 4 * max(self.win + [1]) + 2
        for c in range(3):
            for l in range(self.H):
                for B in range(self.nb_l[l]):
                    for A in range(self.na_l[l]):
                        if not (A | B) & 1:
                            continue
                        ref = np.pad(out[c, self.node(l, B & ~1, A & ~1)], pad, mode="edge")
                        for blk in range(self.nblk):
                            mx, my, sg = self.mvs.get((c, l, self.record(l, B, A, blk)), (0, 0, 1))
                            by, bx = (blk // self.nbx) * bs, (blk % self.nbx) * bs
                            Y = 4 * np.arange(by, by + bs)[:, None] + my
                            X = 4 * np.arange(bx, bx + bs)[None, :] + mx
                            y0, x0 = Y // 4, X // 4
                            fy, fx = Y - 4 * y0, X - 4 * x0
                            t = lambda dy, dx: ref[y0 + dy + pad, x0 + dx + pad]  # noqa: E731
                            acc = ((4 - fx) * (4 - fy) * t(0, 0) + fx * (4 - fy) * t(0, 1)
                                   + (4 - fx) * fy * t(1, 0) + fx * fy * t(1, 1))
                            out[c, self.node(l, B, A), by:by + bs, bx:bx + bs] += sg * ((acc + 8) // 16)
        return out

    def decode_ycocg(self) -> np.ndarray:
        """[3][nb][na][h][w]: root RKV + the SRVs on each view's path."""
        srv = self.srv_planes()
        out = np.zeros((3, self.nb, self.na, self.h, self.w), dtype=np.int64)
        for b in range(self.nb):
            for a in range(self.na):
                v = self.root[:, b >> self.H, a >> self.H].astype(np.int64)
                for l in range(self.H):
                    v = v + srv[:, self.node(l, b >> l, a >> l)]
                out[:, b, a] = v
        return out
