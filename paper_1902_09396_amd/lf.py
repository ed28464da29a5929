"""Python binding of libhmlfc.so: argument marshalling only.

Every step of decoding and rendering runs in the library's HIP kernels; torch
provides device memory and the current stream.  There is no CPU fallback: if
the library is missing or no GPU is visible, calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhmlfc.so")

LF_OK, LF_EINVAL, LF_ENOMEM, LF_EFORMAT, LF_EDEVICE = 0, -1, -2, -3, -4
LF_LOAD_SPARSE_REFS = 1
LF_LOAD_CSR_REFS = 2
_NAMES = {LF_EINVAL: "LF_EINVAL", LF_ENOMEM: "LF_ENOMEM", LF_EFORMAT: "LF_EFORMAT", LF_EDEVICE: "LF_EDEVICE"}


class LFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), msg))
        self.status = status


class LfInfo(C.Structure):
    _fields_ = [("na", C.c_int32), ("nb", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("levels", C.c_int32), ("block", C.c_int32), ("root_na", C.c_int32), ("root_nb", C.c_int32),
                ("n_nodes", C.c_int64), ("n_pred_records", C.c_int64), ("n_refs", C.c_int64),
                ("arena_bytes", C.c_int64), ("stream_bytes", C.c_int64), ("payload_bytes", C.c_int64),
                ("ref_bytes", C.c_int64), ("sparse_refs", C.c_int32), ("clamped_coords", C.c_int64),
                ("chroma420", C.c_int32)]


_lib = None

# C-ABI entry points: name -> (restype, argtypes)
_P, _I32, _I64, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
SIGNATURES = {
    "lf_query_arena": (C.c_int, [_P, _SZ, _P]),
    "lf_load_compressed": (C.c_int, [_P, _SZ, _P, _I64, _P, _P]),
    "lf_query_arena_ex": (C.c_int, [_P, _SZ, _I32, _P]),
    "lf_load_compressed_ex": (C.c_int, [_P, _SZ, _I32, _P, _I64, _P, _P]),
    "lf_free": (C.c_int, [_P]),
    "lf_get_info": (C.c_int, [_P, _P]),
    "lf_decode_pixels": (C.c_int, [_P, _P, _I64, _P, _P]),
    "lf_render_views": (C.c_int, [_P, _P, _I32, _I32, _I32, _P, _P]),
    "lf_render_views_per_ray": (C.c_int, [_P, _P, _I32, _I32, _I32, _P, _P]),
    "lf_decode_pixels_lod": (C.c_int, [_P, _I32, _P, _I64, _P, _P]),
    "lf_render_views_lod": (C.c_int, [_P, _I32, _P, _I32, _I32, _I32, _P, _P]),
    "lf_get_render_config": (C.c_int, [_I32, _I32, _I32, _P, _P]),
    "lf_ray_coords": (C.c_int, [_P, _I32, _I32, _I32, _P, _P]),
    "lf_footprint_bytes": (C.c_int, [_P, _P, _I32, _I32, _I32, _P, _P]),
    "lf_footprint_bytes_noalloc": (C.c_int, [_P, _P, _I32, _I32, _I32, _P, _P]),
    "lf_export_params": (C.c_int, [_P, _P, _P, _P]),
    "lf_render_relaxed": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _P, _P]),
    "lf_backward_workspace": (C.c_int, [_P, _I32, _I32, _I32, _P]),
    "lf_render_backward": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _I32, _P, _P, _P, _P, _I64, _P]),
    "lf_encode_free": (None, [_P]),
    "lf_encode_workspace_bytes": (C.c_int, [_I32, _I32, _I32, _I32, _P, _P]),
    "lf_encode_device": (C.c_int, [_P, _I32, _I32, _I32, _I32, _P, _P, _I64, _P, _P, _P]),
    "lf_mc_search": (C.c_int, [_P, _I64, _P, _I64, _I32, _I32, _I32, _I32, _I32, _I32, _P, _I64, _P, _P]),
    "lf_last_error": (C.c_char_p, []),
}


def lib():
    """Load libhmlfc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhmlfc.so is not built; run __graft_entry__.build() or "
                               "python paper_1902_09396_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != LF_OK:
        raise LFError(status, lib().lf_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    return t.contiguous()


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HMLFC library runs only on the GPU")


class LightField:
    """A compressed light field resident in device memory."""

    def __init__(self, stream, device=None, sparse_refs: bool = False, csr_refs: bool = False):
        """sparse_refs=True keeps only the significant reference blocks resident,
        csr_refs=True only the nonzero reference pixels as compressed sparse rows
        (same results; rendered one thread per ray)."""
        require_gpu()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        host = np.ascontiguousarray(np.frombuffer(bytes(stream), np.uint8) if isinstance(stream, (bytes, bytearray))
                                    else np.asarray(stream, dtype=np.uint8))
        self.stream_bytes = host.size
        flags = (LF_LOAD_SPARSE_REFS if sparse_refs else 0) | (LF_LOAD_CSR_REFS if csr_refs else 0)
        need = C.c_int64()
        check(lib().lf_query_arena_ex(host.ctypes.data_as(C.c_void_p), host.size, flags, C.byref(need)))
        with torch.cuda.device(self.device):
            # torch's caching allocator returns 512-byte aligned blocks
            self.arena = torch.empty(int(need.value), dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            check(lib().lf_load_compressed_ex(host.ctypes.data_as(C.c_void_p), host.size, flags, _ptr(self.arena),
                                              int(need.value), _stream(), C.byref(h)))
        self._h = h
        info = LfInfo()
        check(lib().lf_get_info(self._h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in LfInfo._fields_}
        self.na, self.nb = info.na, info.nb
        self.width, self.height = info.width, info.height
        self.levels, self.block = info.levels, info.block

    def clamped_coords(self) -> int:
        """Decode requests clamped to the grid since load (after this device's current stream finishes)."""
        torch.cuda.current_stream(self.device).synchronize()
        info = LfInfo()
        check(lib().lf_get_info(self._h, C.byref(info)))
        return int(info.clamped_coords)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().lf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def decode_pixels(self, coords: torch.Tensor) -> torch.Tensor:
        """coords: int32 [n, 4] (b, a, y, x) on the device -> uint8 [n, 3] RGB."""
        coords = _dev(coords, torch.int32, "coords").reshape(-1, 4)
        out = torch.empty((coords.shape[0], 3), dtype=torch.uint8, device=coords.device)
        check(lib().lf_decode_pixels(self._h, _ptr(coords), coords.shape[0], _ptr(out), _stream()))
        return out

    def decode_nodes(self, level: int, coords: torch.Tensor) -> torch.Tensor:
        """Progressive decode: coords int32 [n, 4] (B, A, y, x) of level-`level`
        nodes on the device -> uint8 [n, 3] RGB of their reconstructed images."""
        coords = _dev(coords, torch.int32, "coords").reshape(-1, 4)
        out = torch.empty((coords.shape[0], 3), dtype=torch.uint8, device=coords.device)
        check(lib().lf_decode_pixels_lod(self._h, level, _ptr(coords), coords.shape[0], _ptr(out), _stream()))
        return out

    def render_views_lod(self, level: int, cams: torch.Tensor, width: int, height: int) -> torch.Tensor:
        """Level-of-detail render: every view reads its level-`level` ancestor's image."""
        cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
        out = torch.empty((cams.shape[0], 3, height, width), dtype=torch.float32, device=cams.device)
        check(lib().lf_render_views_lod(self._h, level, _ptr(cams), cams.shape[0], width, height, _ptr(out),
                                        _stream()))
        return out

    def render_views(self, cams: torch.Tensor, width: int, height: int, out: torch.Tensor | None = None,
                     per_ray: bool = False):
        """cams: float32 [V, 18] on the device -> float32 [V, 3, height, width].

        per_ray=True selects the unstaged one-thread-per-ray kernel (same results)."""
        cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
        if out is None:
            out = torch.empty((cams.shape[0], 3, height, width), dtype=torch.float32, device=cams.device)
        elif out.shape != (cams.shape[0], 3, height, width) or not out.is_contiguous() or out.dtype != torch.float32:
            raise ValueError("out must be a contiguous float32 [V, 3, H, W] tensor")
        fn = lib().lf_render_views_per_ray if per_ray else lib().lf_render_views
        check(fn(self._h, _ptr(cams), cams.shape[0], width, height, _ptr(out), _stream()))
        return out

    # ---- relaxed model (encoder-side refinement) ----
    def export_params(self):
        """(residual float32 [3, n_nodes, h, w], shift float32 [n_records, 2]) on the device."""
        res = torch.empty((3, self.info["n_nodes"], self.height, self.width), dtype=torch.float32, device=self.device)
        sh = torch.empty((max(self.info["n_pred_records"], 0), 2), dtype=torch.float32, device=self.device)
        check(lib().lf_export_params(self._h, _ptr(res), _ptr(sh), _stream()))
        return res, sh

    def render_relaxed(self, residual: torch.Tensor, shift: torch.Tensor, cams: torch.Tensor, width: int,
                       height: int) -> torch.Tensor:
        residual = _dev(residual, torch.float32, "residual")
        shift = _dev(shift, torch.float32, "shift")
        self._check_params(residual, shift)
        cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
        out = torch.empty((cams.shape[0], 3, height, width), dtype=torch.float32, device=cams.device)
        check(lib().lf_render_relaxed(self._h, _ptr(residual), _ptr(shift), _ptr(cams), cams.shape[0], width, height,
                                      _ptr(out), _stream()))
        return out

    def render_backward(self, residual, shift, cams, width, height, grad_out):
        residual = _dev(residual, torch.float32, "residual")
        shift = _dev(shift, torch.float32, "shift")
        self._check_params(residual, shift)
        cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
        grad_out = _dev(grad_out, torch.float32, "grad_out")
        if tuple(grad_out.shape) != (cams.shape[0], 3, height, width):
            raise ValueError("grad_out must be [V, 3, H, W]")
        need = C.c_int64()
        check(lib().lf_backward_workspace(self._h, cams.shape[0], width, height, C.byref(need)))
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=cams.device)
        g_res = torch.empty_like(residual)
        g_sh = torch.empty_like(shift)
        check(lib().lf_render_backward(self._h, _ptr(residual), _ptr(shift), _ptr(cams), cams.shape[0], width, height,
                                       _ptr(grad_out), _ptr(g_res), _ptr(g_sh), _ptr(ws), int(need.value), _stream()))
        return g_res, g_sh

    def _check_params(self, residual, shift):
        if tuple(residual.shape) != (3, self.info["n_nodes"], self.height, self.width):
            raise ValueError("residual must be [3, n_nodes, h, w]")
        if tuple(shift.shape) != (self.info["n_pred_records"], 2):
            raise ValueError("shift must be [n_records, 2]")

    def footprint_bytes(self, cams: torch.Tensor, width: int, height: int) -> np.ndarray:
        cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
        out = np.zeros(cams.shape[0], dtype=np.float64)
        check(lib().lf_footprint_bytes(self._h, _ptr(cams), cams.shape[0], width, height,
                                       out.ctypes.data_as(C.c_void_p), _stream()))
        return out


def render_config(n_views: int, width: int, height: int) -> tuple[int, int]:
    """(views decoded per group, views per workgroup chunk) render_views uses for n_views views."""
    g, c = C.c_int32(), C.c_int32()
    check(lib().lf_get_render_config(n_views, width, height, C.byref(g), C.byref(c)))
    return g.value, c.value


def ray_coords(cams: torch.Tensor, width: int, height: int) -> torch.Tensor:
    """(u, v, s, t) per output pixel as the renderer computes them: [V, H, W, 4]."""
    cams = _dev(cams, torch.float32, "cams").reshape(-1, 18)
    out = torch.empty((cams.shape[0], height, width, 4), dtype=torch.float32, device=cams.device)
    check(lib().lf_ray_coords(_ptr(cams), cams.shape[0], width, height, _ptr(out), _stream()))
    return out


class EncodeParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("block", C.c_int32), ("step", C.c_int32 * 8), ("t_ref", C.c_int32 * 8),
                ("t_pred", C.c_int32 * 8), ("win", C.c_int32 * 8), ("subpel", C.c_int32), ("zero_phase", C.c_int32),
                ("no_mc", C.c_int32), ("chroma420", C.c_int32)]


def encode(light_field: np.ndarray, enc: dict) -> np.ndarray:
    """Encode a uint8 [nb][na][h][w][3] light field on the current GPU; returns the stream bytes."""
    lf = np.ascontiguousarray(light_field, dtype=np.uint8)
    nb, na, h, w, _ = lf.shape
    p = _encode_params(enc)
    out = C.c_void_p()
    n = C.c_size_t()
    need = C.c_int64()
    check(lib().lf_encode_workspace_bytes(nb, na, h, w, C.byref(p), C.byref(need)))
    work = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device="cuda")
    check(lib().lf_encode_device(lf.ctypes.data_as(C.c_void_p), nb, na, h, w, C.byref(p), _ptr(work), work.numel(),
                                 _stream(), C.byref(out), C.byref(n)))
    del work
    buf = np.ctypeslib.as_array(C.cast(out, C.POINTER(C.c_uint8)), shape=(n.value,)).copy()
    lib().lf_encode_free(out)
    return buf


def mc_search(pred: torch.Tensor, ref: torch.Tensor, items: torch.Tensor, block: int, win: int,
              subpel: bool = True, zero_phase: bool = False) -> torch.Tensor:
    """Phase-shifted motion search on the device.

    pred, ref: int16 [planes, h, w]; items: int32 [n, 3] (pred plane, ref plane,
    block index) -> int32 [n, 4] (mx, my, sigma, cost)."""
    pred = _dev(pred, torch.int16, "pred")
    ref = _dev(ref, torch.int16, "ref")
    items = _dev(items, torch.int32, "items").reshape(-1, 3)
    if pred.dim() != 3 or ref.dim() != 3 or pred.shape[1:] != ref.shape[1:]:
        raise ValueError("pred and ref must be [planes, h, w] with the same plane size")
    out = torch.empty((items.shape[0], 4), dtype=torch.int32, device=items.device)
    check(lib().lf_mc_search(_ptr(pred), pred.shape[0], _ptr(ref), ref.shape[0], pred.shape[2], pred.shape[1], block,
                             win, int(subpel), int(zero_phase), _ptr(items), items.shape[0], _ptr(out), _stream()))
    return out


def _encode_params(enc: dict):
    p = EncodeParams()
    p.levels, p.block = enc["levels"], enc["block"]
    for l in range(enc["levels"]):
        p.step[l], p.t_ref[l], p.t_pred[l], p.win[l] = enc["step"][l], enc["t_ref"][l], enc["t_pred"][l], enc["win"][l]
    p.subpel, p.zero_phase, p.no_mc = int(enc.get("subpel", True)), int(enc.get("zero_phase", False)), \
        int(enc.get("no_mc", False))
    p.chroma420 = int(enc.get("chroma420", False))
    return p


def query_arena(stream, sparse_refs: bool = False, csr_refs: bool = False) -> int:
    host = np.ascontiguousarray(np.asarray(stream, dtype=np.uint8))
    need = C.c_int64()
    check(lib().lf_query_arena_ex(host.ctypes.data_as(C.c_void_p), host.size,
                                  (LF_LOAD_SPARSE_REFS if sparse_refs else 0) | (LF_LOAD_CSR_REFS if csr_refs else 0),
                                  C.byref(need)))
    return int(need.value)
