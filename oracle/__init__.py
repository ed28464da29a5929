"""ctypes front end of the HMLFC CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The GPU library does not import it and
shares no code with it; the only module both sides use is ``lfscene`` (seeded
inputs, no codec arithmetic).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("codec.c", "render.c")]
_HDR = [os.path.join(_HERE, f) for f in ("oracle.h", "internal.h")]
MAX_LEVELS = 8


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11, -O2, OpenMP, no FP contraction)."""
    newest = max(os.path.getmtime(f) for f in _SRC + _HDR)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp] + _SRC + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        sig = {
            "orc_ycocg_fwd_n": (None, [P, i64, P]),
            "orc_ycocg_inv_n": (None, [P, i64, P]),
            "orc_qpel": (i32, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
            "orc_mc_search": (i64, [P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.c_int, P, P, P]),
            "orc_bise_choose": (C.c_int, [P, C.c_int]),
            "orc_bise_bits": (i64, [C.c_int, C.c_int]),
            "orc_bise_pack": (None, [P, C.c_int, C.c_int, P]),
            "orc_bise_get": (C.c_uint32, [P, C.c_int, C.c_int]),
            "orc_bise_unpack": (None, [P, C.c_int, C.c_int, P]),
            "orc_encode": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, P, C.c_int, P, P]),
            "orc_free": (None, [P]),
            "orc_set_threads": (C.c_int, [C.c_int]),
            "orc_open": (C.c_int, [P, C.c_size_t, P]),
            "orc_close": (None, [P]),
            "orc_info": (None, [P, P]),
            "orc_decode_channel_at": (C.c_int, [P, C.c_int, C.c_int, P, i64, P]),
            "orc_chroma_down": (None, [P, C.c_int, C.c_int, P]),
            "orc_chroma_up": (None, [P, C.c_int, C.c_int, P]),
            "orc_decode_at": (C.c_int, [P, P, i64, P]),
            "orc_decode_at_ycocg": (C.c_int, [P, P, i64, P]),
            "orc_decode_node": (C.c_int, [P, C.c_int, P, i64, P]),
            "orc_render_lod": (C.c_int, [P, C.c_int, P, C.c_int, C.c_int, C.c_int, P]),
            "orc_decode_full": (C.c_int, [P, P]),
            "orc_decode_full_ycocg": (C.c_int, [P, P]),
            "orc_decode_srv": (C.c_int, [P, P]),
            "orc_ray_coords": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, P]),
            "orc_render": (C.c_int, [P, P, C.c_int, C.c_int, C.c_int, C.c_int, P]),
            "orc_render_rays": (C.c_int, [P, P, C.c_int, C.c_int, P, i64, P]),
            "orc_render_dense": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, P, C.c_int, C.c_int,
                                           C.c_int, P]),
            "orc_footprint_bytes": (C.c_int, [P, P, C.c_int, C.c_int, C.c_int, P]),
            "orc_export_params": (C.c_int, [P, P, P]),
            "orc_render_relaxed": (C.c_int, [P, P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, P]),
            "orc_relaxed_grad": (C.c_int, [P, P, P, P, C.c_int, C.c_int, C.c_int, P, P, P]),
            "orc_param_check": (i64, [P, P, P, P, C.c_int, C.c_int, C.c_int, P, C.c_int, i64, f64, P, P]),
            "orc_relaxed_loss": (f64, [P, P, P, P, C.c_int, C.c_int, C.c_int, P, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _Params(C.Structure):
    _fields_ = [("levels", C.c_int32), ("block", C.c_int32), ("step", C.c_int32 * MAX_LEVELS),
                ("t_ref", C.c_int32 * MAX_LEVELS), ("t_pred", C.c_int32 * MAX_LEVELS),
                ("win", C.c_int32 * MAX_LEVELS), ("subpel", C.c_int32), ("zero_phase", C.c_int32),
                ("no_mc", C.c_int32), ("chroma420", C.c_int32)]


def _params(enc: dict) -> _Params:
    p = _Params()
    p.levels = enc["levels"]
    p.block = enc["block"]
    for l in range(enc["levels"]):
        p.step[l] = enc["step"][l]
        p.t_ref[l] = enc["t_ref"][l]
        p.t_pred[l] = enc["t_pred"][l]
        p.win[l] = enc["win"][l]
    p.subpel = int(enc.get("subpel", True))
    p.zero_phase = int(enc.get("zero_phase", False))
    p.no_mc = int(enc.get("no_mc", False))
    p.chroma420 = int(enc.get("chroma420", False))
    return p


# ---------------------------------------------------------------- pieces

def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops from now on (n <= 0: all); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def ycocg_fwd(rgb: np.ndarray) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.int32).reshape(-1, 3)
    out = np.empty_like(rgb)
    lib().orc_ycocg_fwd_n(_p(rgb), rgb.shape[0], _p(out))
    return out


def ycocg_inv(ycc: np.ndarray) -> np.ndarray:
    ycc = np.ascontiguousarray(ycc, dtype=np.int32).reshape(-1, 3)
    out = np.empty_like(ycc)
    lib().orc_ycocg_inv_n(_p(ycc), ycc.shape[0], _p(out))
    return out


def qpel(plane: np.ndarray, y: int, x: int, mx: int, my: int) -> int:
    plane = np.ascontiguousarray(plane, dtype=np.int32)
    h, w = plane.shape
    return int(lib().orc_qpel(_p(plane), w, h, y, x, mx, my))


def mc_search(p: np.ndarray, r: np.ndarray, by0: int, bx0: int, bs: int, win: int,
              subpel: bool = True, zero_phase: bool = False):
    p = np.ascontiguousarray(p, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    h, w = p.shape
    mx, my, sg = C.c_int(), C.c_int(), C.c_int()
    cost = lib().orc_mc_search(_p(p), _p(r), w, h, by0, bx0, bs, win, int(subpel), int(zero_phase),
                               C.byref(mx), C.byref(my), C.byref(sg))
    return int(cost), mx.value, my.value, sg.value


def bise_choose(v: np.ndarray) -> int:
    v = np.ascontiguousarray(v, dtype=np.uint32)
    return int(lib().orc_bise_choose(_p(v), v.size))


def bise_bits(mode: int, n: int) -> int:
    return int(lib().orc_bise_bits(mode, n))


def bise_pack(v: np.ndarray, mode: int) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.uint32)
    words = np.zeros((bise_bits(mode, v.size) + 31) // 32 + 2, dtype=np.uint32)
    lib().orc_bise_pack(_p(v), v.size, mode, _p(words))
    return words


def bise_get(words: np.ndarray, mode: int, i: int) -> int:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    return int(lib().orc_bise_get(_p(words), mode, i))


def bise_unpack(words: np.ndarray, mode: int, n: int) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.empty(n, dtype=np.uint32)
    lib().orc_bise_unpack(_p(words), mode, n, _p(out))
    return out


def ray_coords(cam: np.ndarray, wo: int, ho: int, i: int, j: int) -> np.ndarray:
    cam = np.ascontiguousarray(cam, dtype=np.float32)
    out = np.empty(4, dtype=np.float32)
    lib().orc_ray_coords(_p(cam), wo, ho, i, j, _p(out))
    return out


def render_dense(lf: np.ndarray, cams: np.ndarray, wo: int, ho: int) -> np.ndarray:
    lf = np.ascontiguousarray(lf, dtype=np.uint8)
    nb, na, h, w, _ = lf.shape
    cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
    out = np.empty((cams.shape[0], 3, ho, wo), dtype=np.float64)
    lib().orc_render_dense(_p(lf), nb, na, h, w, _p(cams), cams.shape[0], wo, ho, _p(out))
    return out


# ---------------------------------------------------------------- encoder

def encode(lf: np.ndarray, enc: dict, nthreads: int = 0) -> np.ndarray:
    """Encode a uint8[nb][na][h][w][3] light field; returns the stream as uint8."""
    lf = np.ascontiguousarray(lf, dtype=np.uint8)
    nb, na, h, w, _ = lf.shape
    prm = _params(enc)
    out = C.c_void_p()
    n = C.c_size_t()
    rc = lib().orc_encode(_p(lf), nb, na, h, w, C.byref(prm), nthreads, C.byref(out), C.byref(n))
    if rc != 0:
        raise ValueError("oracle encode failed (%d)" % rc)
    buf = np.ctypeslib.as_array(C.cast(out, C.POINTER(C.c_uint8)), shape=(n.value,)).copy()
    lib().orc_free(out)
    return buf


# ---------------------------------------------------------------- stream

class OracleLF:
    """A parsed stream (the stream bytes are kept alive by this object)."""

    def __init__(self, stream: np.ndarray):
        self.stream = np.ascontiguousarray(stream, dtype=np.uint8)
        h = C.c_void_p()
        rc = lib().orc_open(_p(self.stream), self.stream.size, C.byref(h))
        if rc != 0:
            raise ValueError("oracle: malformed stream (%d)" % rc)
        self._h = h
        info = np.zeros(11, dtype=np.int64)
        lib().orc_info(self._h, _p(info))
        (self.na, self.nb, self.w, self.h, self.levels, self.block, self.n_nodes, self.n_pred,
         self.root_na, self.root_nb, self.chroma420) = (int(v) for v in info)

    def close(self):
        if self._h:
            lib().orc_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def decode_at(self, coords: np.ndarray) -> np.ndarray:
        coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 4)
        out = np.empty((coords.shape[0], 3), dtype=np.uint8)
        if lib().orc_decode_at(self._h, _p(coords), coords.shape[0], _p(out)) != 0:
            raise ValueError("coordinate out of range")
        return out

    def decode_at_ycocg(self, coords: np.ndarray) -> np.ndarray:
        coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 4)
        out = np.empty((coords.shape[0], 3), dtype=np.int32)
        if lib().orc_decode_at_ycocg(self._h, _p(coords), coords.shape[0], _p(out)) != 0:
            raise ValueError("coordinate out of range")
        return out

    def decode_node(self, level: int, coords: np.ndarray) -> np.ndarray:
        """Node images of `level` (0 .. H) at (B, A, y, x): progressive decode."""
        coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 4)
        out = np.empty((coords.shape[0], 3), dtype=np.uint8)
        if lib().orc_decode_node(self._h, int(level), _p(coords), coords.shape[0], _p(out)) != 0:
            raise ValueError("level or coordinate out of range")
        return out

    def render_lod(self, level: int, cams: np.ndarray, wo: int, ho: int) -> np.ndarray:
        """render() with every sample's walk stopped at `level`."""
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        out = np.empty((cams.shape[0], 3, ho, wo), dtype=np.float64)
        if lib().orc_render_lod(self._h, int(level), _p(cams), cams.shape[0], wo, ho, _p(out)) != 0:
            raise ValueError("level out of range")
        return out

    def decode_channel(self, c: int, coords: np.ndarray, lod: int = 0) -> np.ndarray:
        """Channel c at its own resolution (half size for 4:2:0 chroma): coords (b, a, y, x) -> int32."""
        coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 4)
        out = np.empty(coords.shape[0], dtype=np.int32)
        if lib().orc_decode_channel_at(self._h, int(c), int(lod), _p(coords), coords.shape[0], _p(out)) != 0:
            raise ValueError("channel, level or coordinate out of range")
        return out

    def decode_full(self) -> np.ndarray:
        out = np.empty((self.nb, self.na, self.h, self.w, 3), dtype=np.uint8)
        lib().orc_decode_full(self._h, _p(out))
        return out

    def decode_full_ycocg(self) -> np.ndarray:
        out = np.empty((3, self.nb, self.na, self.h, self.w), dtype=np.int32)
        lib().orc_decode_full_ycocg(self._h, _p(out))
        return out

    def decode_srv(self) -> np.ndarray:
        out = np.empty((3, self.n_nodes, self.h, self.w), dtype=np.int32)
        lib().orc_decode_srv(self._h, _p(out))
        return out

    def render(self, cams: np.ndarray, wo: int, ho: int) -> np.ndarray:
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        out = np.empty((cams.shape[0], 3, ho, wo), dtype=np.float64)
        lib().orc_render(self._h, _p(cams), cams.shape[0], wo, ho, 0, _p(out))
        return out

    def render_rays(self, cams: np.ndarray, wo: int, ho: int, rays: np.ndarray) -> np.ndarray:
        """Selected rays (view, i, j) -> float64 [n][3]."""
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        rays = np.ascontiguousarray(rays, dtype=np.int32).reshape(-1, 3)
        if rays.size and (rays[:, 0].max() >= cams.shape[0] or rays[:, 0].min() < 0):
            raise ValueError("view index out of range")
        out = np.empty((rays.shape[0], 3), dtype=np.float64)
        if lib().orc_render_rays(self._h, _p(cams), wo, ho, _p(rays), rays.shape[0], _p(out)) != 0:
            raise ValueError("ray out of range")
        return out

    def footprint_bytes(self, cams: np.ndarray, wo: int, ho: int) -> np.ndarray:
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        out = np.empty(cams.shape[0], dtype=np.float64)
        lib().orc_footprint_bytes(self._h, _p(cams), cams.shape[0], wo, ho, _p(out))
        return out

    # relaxed model
    def export_params(self):
        res = np.empty((3, self.n_nodes, self.h, self.w), dtype=np.float32)
        sh = np.empty((self.n_pred, 2), dtype=np.float32)
        lib().orc_export_params(self._h, _p(res), _p(sh))
        return res, sh

    def render_relaxed(self, residual, shift, cams, wo, ho) -> np.ndarray:
        residual = np.ascontiguousarray(residual, dtype=np.float32)
        shift = np.ascontiguousarray(shift, dtype=np.float32)
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        out = np.empty((cams.shape[0], 3, ho, wo), dtype=np.float64)
        lib().orc_render_relaxed(self._h, _p(residual), _p(shift), _p(cams), cams.shape[0], wo, ho, 0, _p(out))
        return out

    def relaxed_grad(self, residual, shift, cams, wo, ho, grad_out):
        residual = np.ascontiguousarray(residual, dtype=np.float32)
        shift = np.ascontiguousarray(shift, dtype=np.float32)
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        grad_out = np.ascontiguousarray(grad_out, dtype=np.float64)
        g_res = np.empty((3, self.n_nodes, self.h, self.w), dtype=np.float64)
        g_sh = np.empty((self.n_pred, 2), dtype=np.float64)
        lib().orc_relaxed_grad(self._h, _p(residual), _p(shift), _p(cams), cams.shape[0], wo, ho,
                               _p(grad_out), _p(g_res), _p(g_sh))
        return g_res, g_sh

    def param_check(self, residual, shift, cams, wo, ho, target, kind, index, eps=1e-3):
        residual = np.ascontiguousarray(residual, dtype=np.float32)
        shift = np.ascontiguousarray(shift, dtype=np.float32)
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        target = np.ascontiguousarray(target, dtype=np.float32)
        fd, fwd = C.c_double(), C.c_double()
        hits = lib().orc_param_check(self._h, _p(residual), _p(shift), _p(cams), cams.shape[0], wo, ho,
                                     _p(target), kind, index, eps, C.byref(fd), C.byref(fwd))
        return fd.value, fwd.value, int(hits)

    def relaxed_loss(self, residual, shift, cams, wo, ho, target) -> float:
        residual = np.ascontiguousarray(residual, dtype=np.float32)
        shift = np.ascontiguousarray(shift, dtype=np.float32)
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        target = np.ascontiguousarray(target, dtype=np.float32)
        return float(lib().orc_relaxed_loss(self._h, _p(residual), _p(shift), _p(cams), cams.shape[0], wo, ho,
                                            _p(target), 0))
