"""GPU relaxed forward and adjoint against the oracle.

The oracle's relaxed model is FP64 with three independently pinned
derivatives (central differences, forward mode, explicit transpose).  The
GPU's FP32 forward must match it to 1e-5; its gradients must match the
oracle's reverse-mode gradient elementwise to a small fraction of the largest
gradient, and on the 17x17x512^2 light field with 16 orbit views they must be
within 1e-3 relative of central differences (eps 1e-3) and of the exact
forward-mode derivative at 64 sampled parameters (48 residual values and 16
shift components, shifts moved to quarter-pel + 1/8 so that no tap sits at a
bilinear kink).
"""

import numpy as np
import pytest

import lfscene
import oracle
from conftest import stream_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    assert torch.cuda.is_available()
    return torch


def _setup_tiny(torch, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez):
    from paper_1902_09396_amd import lf

    field = lf.LightField(tiny_stream)
    res, sh = field.export_params()
    sh = sh + 0.125
    cams = torch.from_numpy(tiny_cams_ez).cuda()
    target = oracle.render_dense(tiny_lf, tiny_cams_ez, 64, 64).astype(np.float32)
    return field, res, sh, cams, target


def test_export_params_match_oracle(torch_mod, tiny_stream, tiny_oracle):
    from paper_1902_09396_amd import lf

    field = lf.LightField(tiny_stream)
    res, sh = field.export_params()
    ores, osh = tiny_oracle.export_params()
    assert np.array_equal(res.cpu().numpy(), ores)
    assert np.array_equal(sh.cpu().numpy(), osh)


def test_relaxed_forward_matches_oracle(torch_mod, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez):
    torch = torch_mod
    field, res, sh, cams, target = _setup_tiny(torch, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez)
    got = field.render_relaxed(res, sh, cams, 64, 64).cpu().numpy().astype(np.float64)
    expect = tiny_oracle.render_relaxed(res.cpu().numpy(), sh.cpu().numpy(), tiny_cams_ez, 64, 64)
    assert np.abs(got - expect).max() <= 1e-5


def test_adjoint_matches_oracle_reverse_mode(torch_mod, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez):
    torch = torch_mod
    field, res, sh, cams, target = _setup_tiny(torch, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez)
    rng = np.random.default_rng(3)
    w = rng.normal(size=(tiny_cams_ez.shape[0], 3, 64, 64)).astype(np.float32)
    g_res, g_sh = field.render_backward(res, sh, cams, 64, 64, torch.from_numpy(w).cuda())
    o_res, o_sh = tiny_oracle.relaxed_grad(res.cpu().numpy(), sh.cpu().numpy(), tiny_cams_ez, 64, 64,
                                           w.astype(np.float64))
    _check_grads(g_res, g_sh, o_res, o_sh)


def _check_grads(g_res, g_sh, o_res, o_sh):
    """FP32 adjoint vs FP64 reverse mode: every element within 1e-3 of its own
    magnitude plus 1e-6 (residuals) or 1e-5 (shifts) of the largest one (the
    FP32 sums of a sample's contributions cancel down to that floor)."""
    g_res, g_sh = g_res.cpu().numpy().astype(np.float64), g_sh.cpu().numpy().astype(np.float64)
    err_r = np.abs(g_res - o_res)
    err_s = np.abs(g_sh - o_sh)
    assert np.all(err_r <= 1e-3 * np.abs(o_res) + 1e-6 * np.abs(o_res).max() + 1e-12), err_r.max()
    assert np.all(err_s <= 1e-3 * np.abs(o_sh) + 1e-5 * np.abs(o_sh).max() + 1e-12), err_s.max()
    assert err_r.max() <= 1e-5 * np.abs(o_res).max() + 1e-9
    # untouched parameters get exactly zero
    assert np.array_equal(g_res == 0, o_res == 0)


@pytest.mark.parametrize("block", [8, 2])
def test_adjoint_far_shifts(torch_mod, tiny_lf, tiny_cams_ez, block):
    """Shifts moved up to 6 pixels from their stored vectors, one of them by
    20 pixels: every reference tile's reach grows.  With 2x2 blocks a 16x16
    tile can then be reached by more predictive blocks than its LDS list
    holds (3 * 31^2 > 192), so the reference pull runs its unstaged path;
    with 8x8 blocks the list holds them (3 * 8^2 = 192) but the sibling windows (the whole
    64x64 plane, three times) exceed the LDS window, so the taps are read
    from global memory.  Both must match the oracle."""
    torch = torch_mod
    from paper_1902_09396_amd import lf

    stream = stream_for("tiny", tiny_lf, block=block)
    o = oracle.OracleLF(stream)
    field = lf.LightField(stream)
    res, sh = field.export_params()
    cams = torch.from_numpy(tiny_cams_ez).cuda()
    rng = np.random.default_rng(9)
    far = sh.cpu().numpy() + rng.uniform(-6.0, 6.0, size=tuple(sh.shape)).astype(np.float32)
    far[len(far) // 2] = (20.375, -19.625)
    far_d = torch.from_numpy(far).cuda()
    w = rng.normal(size=(tiny_cams_ez.shape[0], 3, 64, 64)).astype(np.float32)
    g_res, g_sh = field.render_backward(res, far_d, cams, 64, 64, torch.from_numpy(w).cuda())
    o_res, o_sh = o.relaxed_grad(res.cpu().numpy(), far, tiny_cams_ez, 64, 64, w.astype(np.float64))
    _check_grads(g_res, g_sh, o_res, o_sh)
    got = field.render_relaxed(res, far_d, cams, 64, 64).cpu().numpy().astype(np.float64)
    assert np.abs(got - o.render_relaxed(res.cpu().numpy(), far, tiny_cams_ez, 64, 64)).max() <= 1e-5


@pytest.mark.parametrize("na,nb", [(5, 1), (1, 3), (2, 2)])
def test_adjoint_thin_grids(torch_mod, tiny_lf, na, nb):
    """Grids with a single row or column of views (both blend corners of that
    axis are the same view) and a 2x2 grid: gradients match the oracle's."""
    torch = torch_mod
    from paper_1902_09396_amd import lf

    x = np.ascontiguousarray(tiny_lf[:nb, :na])
    enc = lfscene.get_config("tiny")["enc"]
    stream = oracle.encode(x, enc)
    o = oracle.OracleLF(stream)
    field = lf.LightField(stream)
    res, sh = field.export_params()
    sh = sh + 0.125
    cams_np = lfscene.random_pinhole_cameras(3, na, nb, 64, 64, 48, 40, seed=na * 10 + nb)
    cams = torch.from_numpy(cams_np).cuda()
    rng = np.random.default_rng(na + 7 * nb)
    w = rng.normal(size=(3, 3, 40, 48)).astype(np.float32)
    g_res, g_sh = field.render_backward(res, sh, cams, 48, 40, torch.from_numpy(w).cuda())
    o_res, o_sh = o.relaxed_grad(res.cpu().numpy(), sh.cpu().numpy(), cams_np, 48, 40, w.astype(np.float64))
    _check_grads(g_res, g_sh, o_res, o_sh)


def test_backward_batch_limit(torch_mod, tiny_stream):
    """At most 2^29 - 1 rays per backward call (4 sort records per ray, an int
    count): larger batches are rejected by the host-side size query."""
    import ctypes as C

    from paper_1902_09396_amd import lf

    field = lf.LightField(tiny_stream)
    need = C.c_int64()
    lf.check(lf.lib().lf_backward_workspace(field.handle, 127, 2048, 2048, C.byref(need)))
    assert need.value > 127 * 2048 * 2048 * (4 * 16 + 16)  # sort keys and values twice, blend fractions
    for nv in (128, 129, 260):
        assert lf.lib().lf_backward_workspace(field.handle, nv, 2048, 2048, C.byref(need)) == lf.LF_EINVAL
    assert lf.lib().lf_backward_workspace(field.handle, 259, 1920, 1080, C.byref(need)) == lf.LF_EINVAL


def test_adjoint_deterministic_and_autograd(torch_mod, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez):
    torch = torch_mod
    from paper_1902_09396_amd.autograd import render_relaxed

    field, res, sh, cams, target = _setup_tiny(torch, tiny_stream, tiny_oracle, tiny_lf, tiny_cams_ez)
    tgt = torch.from_numpy(target).cuda()
    grads = []
    for _ in range(2):
        r = res.clone().requires_grad_(True)
        s = sh.clone().requires_grad_(True)
        loss = ((render_relaxed(field, r, s, cams, 64, 64) - tgt) ** 2).sum()
        loss.backward()
        grads.append((r.grad.cpu().numpy(), s.grad.cpu().numpy()))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    # the autograd path is the library adjoint applied to dL/dout = 2 (out - target)
    out = field.render_relaxed(res, sh, cams, 64, 64)
    g_res, g_sh = field.render_backward(res, sh, cams, 64, 64, 2.0 * (out - tgt))
    assert np.array_equal(g_res.cpu().numpy(), grads[0][0])
    assert np.array_equal(g_sh.cpu().numpy(), grads[0][1])


def test_workspace_too_small_rejected(torch_mod, tiny_stream, tiny_cams_ez):
    torch = torch_mod
    import ctypes as C

    from paper_1902_09396_amd import lf

    field = lf.LightField(tiny_stream)
    res, sh = field.export_params()
    cams = torch.from_numpy(tiny_cams_ez).cuda()
    g = torch.zeros((4, 3, 64, 64), device="cuda")
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    gr, gs = torch.empty_like(res), torch.empty_like(sh)
    st = lf.lib().lf_render_backward(field.handle, C.c_void_p(res.data_ptr()), C.c_void_p(sh.data_ptr()),
                                     C.c_void_p(cams.data_ptr()), 4, 64, 64, C.c_void_p(g.data_ptr()),
                                     C.c_void_p(gr.data_ptr()), C.c_void_p(gs.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     1024, None)
    assert st == lf.LF_ENOMEM


def test_fullsize_gradients_vs_fd(torch_mod):
    torch = torch_mod
    from paper_1902_09396_amd import lf

    cfg = lfscene.get_config("grad512")
    L = cfg["lf"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    stream = lf.encode(light, cfg["enc"])  # the GPU encoder (byte-identical to the oracle's, test_gpu_encoder)
    o = oracle.OracleLF(stream)
    field = lf.LightField(stream)
    cams_np = lfscene.make_views(cfg)
    cams = torch.from_numpy(cams_np).cuda()
    res, sh = field.export_params()
    sh = torch.floor(sh * 4.0) / 4.0 + 0.125
    target = oracle.render_dense(light, cams_np, 512, 512).astype(np.float32)
    tgt = torch.from_numpy(target).cuda()
    out = field.render_relaxed(res, sh, cams, 512, 512)
    # the relaxed forward itself, every ray of the 16 views, against the oracle's FP64 forward
    expect = o.render_relaxed(res.cpu().numpy(), sh.cpu().numpy(), cams_np, 512, 512)
    assert np.abs(out.cpu().numpy().astype(np.float64) - expect).max() <= 1e-5
    del expect
    g_res, g_sh = field.render_backward(res, sh, cams, 512, 512, 2.0 * (out - tgt))
    g_res, g_sh = g_res.cpu().numpy().ravel(), g_sh.cpu().numpy().ravel()
    res_np, sh_np = res.cpu().numpy(), sh.cpu().numpy()
    rng = np.random.default_rng(42)
    # sample touched parameters: residuals with a non-negligible gradient, shifts likewise
    cand_r = np.flatnonzero(np.abs(g_res) > 1e-2 * np.abs(g_res).max())
    cand_s = np.flatnonzero(np.abs(g_sh) > 1e-2 * np.abs(g_sh).max())
    picks = [(0, int(i)) for i in rng.choice(cand_r, 48, replace=False)] + \
            [(1, int(i)) for i in rng.choice(cand_s, 16, replace=False)]
    worst_fd, worst_fwd = 0.0, 0.0
    for kind, idx in picks:
        fd, fwd, hits = o.param_check(res_np, sh_np, cams_np, 512, 512, target, kind, idx, eps=1e-3)
        assert hits > 0
        g = float(g_res[idx] if kind == 0 else g_sh[idx])
        worst_fd = max(worst_fd, abs(g - fd) / max(abs(fd), 1e-12))
        worst_fwd = max(worst_fwd, abs(g - fwd) / max(abs(fwd), 1e-12))
    assert worst_fd <= 1e-3, worst_fd
    assert worst_fwd <= 1e-3, worst_fwd
