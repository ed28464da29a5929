"""The allocation-free footprint call against lf_footprint_bytes, through the
C ABI: equal per-view figures, bit for bit, on two calls in a row (the second
on a smaller light field and fewer, smaller views), and its scratch limit."""

import ctypes as C

import numpy as np
import pytest

import lfscene

pytestmark = pytest.mark.gpu


def _noalloc(lib, field, cams, w, h):
    import torch

    out = torch.full((cams.shape[0],), -1.0, dtype=torch.float64, device="cuda")
    st = lib.lf_footprint_bytes_noalloc(field.handle, C.c_void_p(cams.data_ptr()), cams.shape[0], w, h,
                                        C.c_void_p(out.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    return out.cpu().numpy()


def _alloc(lib, field, cams, w, h):
    import torch

    out = np.zeros(cams.shape[0], dtype=np.float64)
    st = lib.lf_footprint_bytes(field.handle, C.c_void_p(cams.data_ptr()), cams.shape[0], w, h,
                                out.ctypes.data_as(C.c_void_p), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    return out


def test_footprint_noalloc_matches(mid_stream, tiny_stream, tiny_cams_ez):
    import torch

    from paper_1902_09396_amd import lf

    lib = lf.lib()
    mid, tiny = lf.LightField(mid_stream), lf.LightField(tiny_stream)
    orbit = torch.from_numpy(lfscene.camera_path_orbit(24, 17, 17, 128, 128, 128, 96, radius=6.0)).cuda()
    a = _noalloc(lib, mid, orbit, 128, 96)
    b = _alloc(lib, mid, orbit, 128, 96)
    assert np.array_equal(a, b) and np.all(a > 12 * 128 * 96)
    small = torch.from_numpy(np.ascontiguousarray(tiny_cams_ez[:3])).cuda()
    a = _noalloc(lib, tiny, small, 40, 24)  # the scratch keeps the last call's marks: they must be cleared
    b = _alloc(lib, tiny, small, 40, 24)
    assert np.array_equal(a, b)
    # zero views: nothing enqueued; bad sizes: rejected before anything runs
    assert lib.lf_footprint_bytes_noalloc(tiny.handle, C.c_void_p(small.data_ptr()), 0, 40, 24, None, None) == 0
    assert lib.lf_footprint_bytes_noalloc(tiny.handle, C.c_void_p(small.data_ptr()), 3, 0, 24,
                                          C.c_void_p(small.data_ptr()), None) == lf.LF_EINVAL
    mid.close()
    tiny.close()
