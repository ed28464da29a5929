"""Python binding of the serving loop (argument marshalling only).

The scheduler, admission, batching and graph replays run in the library's C++
thread and HIP kernels; torch only provides the output pool.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .lf import LightField, check, lib

_P, _I32, _I64, _F64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double


class ServerConfig(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_tiles", C.c_int32), ("chunk_tiles", C.c_int32),
                ("n_streams", C.c_int32), ("use_graphs", C.c_int32), ("grid", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("launches", C.c_int64), ("tiles", C.c_int64), ("graph_launches", C.c_int64),
                ("queue_ms", C.c_double), ("flight_ms", C.c_double)]


_SIGS = {
    "lf_server_create": (C.c_int, [_P, _I32, _P, _I64, _P, _P]),
    "lf_server_submit": (C.c_int, [_P, _I32, _P, _I32, _I32, _I32, _P]),
    "lf_server_wait": (C.c_int, [_P, _I64, _F64, _P, _P]),
    "lf_server_release": (C.c_int, [_P, _I64]),
    "lf_server_get_stats": (C.c_int, [_P, _P]),
    "lf_server_destroy": (C.c_int, [_P]),
    "lf_server_replay": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P]),
    "lf_serve_baseline": (C.c_int, [_P, _I32, _I64, _P, _P, _P, _P, _P, _I64, _P, _P]),
}


def _lib():
    L = lib()
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args
    return L


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


class Server:
    """Resident light fields + continuous-batching request server."""

    def __init__(self, fields: list[LightField], pool_bytes: int, max_slots: int = 64, max_tiles: int = 8192,
                 chunk_tiles: int = 512, n_streams: int = 2, use_graphs: bool = True, grid: int = 0):
        self.fields = list(fields)
        dev = self.fields[0].device
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        handles = (C.c_void_p * len(self.fields))(*[f.handle.value for f in self.fields])
        self._handles = handles
        cfg = ServerConfig(max_slots, max_tiles, chunk_tiles, n_streams, int(use_graphs), grid)
        h = C.c_void_p()
        torch.cuda.synchronize()
        check(_lib().lf_server_create(handles, len(self.fields), C.c_void_p(self.pool.data_ptr()), int(pool_bytes),
                                      C.byref(cfg), C.byref(h)))
        self._h = h

    def submit(self, field: int, cam: np.ndarray, width: int, height: int, auto_release: bool = False) -> int:
        cam = np.ascontiguousarray(cam, dtype=np.float32).reshape(18)
        rid = C.c_int64()
        check(_lib().lf_server_submit(self._h, field, _np(cam), width, height, int(auto_release), C.byref(rid)))
        return rid.value

    def wait(self, rid: int, width: int, height: int, timeout_s: float = 60.0):
        """(output tensor view [3, height, width] in the pool, latency ms)."""
        off, lat = C.c_int64(), C.c_double()
        check(_lib().lf_server_wait(self._h, rid, timeout_s, C.byref(off), C.byref(lat)))
        n = 3 * width * height * 4
        out = self.pool[off.value:off.value + n].view(torch.float32).view(3, height, width)
        return out, lat.value

    def release(self, rid: int):
        check(_lib().lf_server_release(self._h, rid))

    def stats(self) -> dict:
        s = ServerStats()
        check(_lib().lf_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def replay(self, field: np.ndarray, cams: np.ndarray, wh: np.ndarray, arrival_s: np.ndarray):
        """Open-loop replay of a schedule; returns (latency ms per request, makespan s)."""
        field = np.ascontiguousarray(field, dtype=np.int32)
        cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
        wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
        arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
        lat = np.zeros(field.size, dtype=np.float64)
        mk = C.c_double()
        check(_lib().lf_server_replay(self._h, field.size, _np(field), _np(cams), _np(wh), _np(arrival_s), _np(lat),
                                      C.byref(mk)))
        return lat, mk.value

    def close(self):
        if getattr(self, "_h", None):
            _lib().lf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def baseline(fields: list[LightField], field, cams, wh, arrival_s):
    """One lf_render_views launch per request, in arrival order on one stream."""
    field = np.ascontiguousarray(field, dtype=np.int32)
    cams = np.ascontiguousarray(cams, dtype=np.float32).reshape(-1, 18)
    wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
    arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
    out_bytes = int(3 * 4 * (wh[:, 0].astype(np.int64) * wh[:, 1]).max())
    out = torch.empty(out_bytes, dtype=torch.uint8, device=fields[0].device)
    handles = (C.c_void_p * len(fields))(*[f.handle.value for f in fields])
    lat = np.zeros(field.size, dtype=np.float64)
    mk = C.c_double()
    torch.cuda.synchronize()
    check(_lib().lf_serve_baseline(handles, len(fields), field.size, _np(field), _np(cams), _np(wh), _np(arrival_s),
                                   C.c_void_p(out.data_ptr()), out_bytes, _np(lat), C.byref(mk)))
    return lat, mk.value
