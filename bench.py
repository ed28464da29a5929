"""Benchmark: fused random-access decode + novel-view rendering on one MI355X.

Workload: a 17x17 grid of 512x512 RGB views (seeded layered scene with six
planes in front of a smooth-depth terrain, disparity in [-4, 4] px), encoded
with a 4-level tree, 16x16 blocks, quarter-pel motion vectors and step 4;
a step renders the 120-frame 512x512 orbit camera path in one launch.

Prints one JSON line: rays/s for the whole job, the render kernel's achieved
algorithmic bytes per second against the HBM peak (algorithmic bytes = the
per-view footprint bytes of the 120 views), p50/p99 single-view latency, and
the CPU oracle timed on a bounded sample of the same rays.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "rendered rays/sec (Grays/s) + achieved HBM GB/s; p50/p99 view latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_path512_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lf_geom.h", "lf_render_tile.h", "lf_render.hip"):
        with open(os.path.join(ROOT, "paper_1902_09396_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters():
    """Counter figures of the render kernel from committed rocprofv3 runs
    (HBM bytes per launch, L2 hit rate, VALU busy), if taken on this kernel
    source; None otherwise."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed launches (default 50 for the render line, whose launches take 0.5 ms, else 10)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="path512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true", help="skip the one-view-per-launch latency pass")
    ap.add_argument("--cpu-rays", type=int, default=0, help="oracle sample size (0: automatic)")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload instead: resident light fields, Poisson view requests")
    ap.add_argument("--serve-fields", default="serve256,path512,serve1024,batch1080")
    ap.add_argument("--encode", action="store_true",
                    help="encoder: GPU phase-shifted motion search throughput and whole-field encode time")
    ap.add_argument("--rd", action="store_true",
                    help="rate-distortion sweeps (block size, search window, block threshold) on the synthetic field")
    ap.add_argument("--grad", action="store_true",
                    help="differentiation workload instead: relaxed render + adjoint of 16 views")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-sweep", default="", help="more request rates (comma list) for a saturation sweep")
    ap.add_argument("--serve-sweep-seconds", type=float, default=2.0)
    ap.add_argument("--serve-streams", type=int, default=4, help="launches in flight at once (1..4)")
    ap.add_argument("--quant-sweep", default="",
                    help="comma list of quantisation steps: render the workload's path from a stream coded at each")
    args = ap.parse_args()
    if args.steps is None:
        render_line = not (args.serve or args.encode or args.rd or args.grad or args.quant_sweep)
        args.steps = 50 if render_line else 10
    return args


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (views are independent, so "
              "each GPU would render its own chunks of views with no per-frame exchange). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import lfscene
    from paper_1902_09396_amd import lf

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.serve:
        serve_bench(args)
        return
    if args.grad:
        grad_bench(args)
        return
    if args.encode:
        encode_bench(args)
        return
    if args.rd:
        rd_bench(args)
        return
    if args.quant_sweep:
        quant_sweep(args)
        return
    cfg = lfscene.get_config(args.workload)
    L = cfg["lf"]
    t0 = time.time()
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    log("scene %.1fs" % (time.time() - t0))
    t0 = time.time()
    stream = lf.encode(light, cfg["enc"])
    log("encode %.1fs, %d bytes" % (time.time() - t0, stream.size))
    field = lf.LightField(stream, device="cuda:0")
    cams_np = lfscene.make_views(cfg)
    V, wo, ho = cams_np.shape[0], cfg["views"]["wo"], cfg["views"]["ho"]
    cams = torch.from_numpy(cams_np).cuda()
    out = torch.empty((V, 3, ho, wo), dtype=torch.float32, device="cuda")
    rays_per_step = V * wo * ho

    t0 = time.time()
    fp = field.footprint_bytes(cams, wo, ho)
    bytes_per_launch = float(fp.sum())
    log("footprint %.1fs: %.2f MB/view mean" % (time.time() - t0, fp.mean() / 1e6))

    stream_t = torch.cuda.current_stream()
    for _ in range(args.warmup):
        field.render_views(cams, wo, ho, out)
    torch.cuda.synchronize()
    # HIP events on the launch stream bracket the timed region; the kernels'
    # time per launch is their elapsed time over the number of launches
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream_t)
    for k in range(args.steps):
        field.render_views(cams, wo, ho, out)
    ev1.record(stream_t)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = 1e3 * t_total / args.steps
    value = rays_per_step / (ms_per_step * 1e-3) / 1e9

    # single-view latency: each view alone in its own launch
    lat = []
    one = torch.empty((1, 3, ho, wo), dtype=torch.float32, device="cuda")
    for v in range(0 if args.no_latency else V):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream_t)
        field.render_views(cams[v:v + 1], wo, ho, one)
        b.record(stream_t)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    lat = np.array(lat)

    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    counters = load_counters() if args.workload == "path512" else None  # counters were taken on that workload
    traffic = counters.get("bytes_per_launch") if counters else None
    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Grays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "context": "the paper's decoder: about 200 frames/s at 512x512 (52.4 Mrays/s) on a GTX-980, on its "
                   "Lego Knights light field at block 4, tree height 3; different hardware, scene and settings, "
                   "so not a baseline for this line",
        "dtype": "i16x2 decode + f32 blend",
        "views_per_group": lf.render_config(V, wo, ho)[0],
        "views_per_chunk": lf.render_config(V, wo, ho)[1],
        "data": "synthetic",
        "config": {
            "workload": "%dx%d views of %dx%d RGB, %d-level tree, %dx%d blocks, step %d, quarter-pel MVs; %s" % (
                L["na"], L["nb"], L["w"], L["h"], cfg["enc"]["levels"], cfg["enc"]["block"], cfg["enc"]["block"],
                cfg["enc"]["step"][0],
                ("%d-frame %dx%d orbit path per step" % (V, wo, ho)) if cfg["views"]["kind"] == "orbit" else
                ("a batch of %d random %dx%d pinhole cameras per step" % (V, wo, ho))),
            "views_per_step": V,
            "width": wo,
            "height": ho,
            "stream_bytes": int(stream.size),
        },
        "algorithmic_gbs": round(achieved, 1),
        "measured": None if not counters else {
            "dram_bytes_per_launch": traffic,
            "dram_gbs": round(traffic / (kernel_ms * 1e-3) / 1e9, 1),
            "dram_frac": round(traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "l2_hit_rate": counters.get("l2_hit_rate"), "valu_busy": counters.get("valu_busy"),
            "source": counters.get("source"),
            "note": "DRAM bytes from committed counter runs on this kernel source, divided by this run's kernel "
                    "time; below the algorithmic bytes because views of a chunk share decoded values in LDS"},
        "latency_ms": None if not len(lat) else {
            "p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
            "unit": "ms per %dx%d view, one view per launch" % (wo, ho)},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_render_batch",
            "kernel_ms": round(kernel_ms, 4),
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(stream, cams_np, wo, ho, args.cpu_rays)
    print(json.dumps(result), flush=True)


def serve_bench(args):
    """Resident light fields; Poisson requests at --serve-rate for --serve-seconds with output
    resolutions drawn from {256^2, 512^2, 1920x1080, 2048^2} and uniformly random light field and
    pinhole camera; served by the continuous-batching server and, on the same schedule, by one
    render launch per request."""
    import torch

    import lfscene
    from paper_1902_09396_amd import lf
    from paper_1902_09396_amd.serve import Server, baseline

    fields, shapes = [], []
    os.environ.setdefault("HMLFC_ENCODE_PROGRESS", "1")
    os.environ.setdefault("HMLFC_SERVE_PROGRESS", "1")
    for name in args.serve_fields.split(","):
        cfg = lfscene.get_config(name)
        L = cfg["lf"]
        t0 = time.time()
        light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"],
                                progress=lambda d, t, nm=name: log("field %s: %d of %d views generated" % (nm, d, t)))
        stream = lf.encode(light, cfg["enc"])
        del light
        fields.append(lf.LightField(stream, device="cuda:0"))
        shapes.append((L["na"], L["nb"], L["w"], L["h"]))
        log("field %s: %d bytes, %.1fs" % (name, stream.size, time.time() - t0))
    def schedule(rate, seconds, seed):
        rng = np.random.default_rng(seed)
        n = int(rate * seconds)
        arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
        res = np.array([[256, 256], [512, 512], [1920, 1080], [2048, 2048]])
        wh = res[rng.integers(0, 4, size=n)]
        field = rng.integers(0, len(fields), size=n).astype(np.int32)
        cams = np.zeros((n, 18), dtype=np.float32)
        for k in range(n):
            na, nb, w, h = shapes[field[k]]
            cams[k] = lfscene.random_pinhole_cameras(1, na, nb, w, h, int(wh[k, 0]), int(wh[k, 1]),
                                                     seed=int(rng.integers(1 << 30)))[0]
        return field, cams, wh, arrival

    def summary(l, m, rays):
        return {"p50_ms": round(float(np.percentile(l, 50)), 3), "p99_ms": round(float(np.percentile(l, 99)), 3),
                "mean_ms": round(float(l.mean()), 3), "grays_per_s": round(rays / m / 1e9, 4), "makespan_s": round(m, 3)}

    def run(rate, seconds, seed):
        field, cams, wh, arrival = schedule(rate, seconds, seed)
        rays = float((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
        log("%.0f req/s: %d requests, %.2f Grays offered over %.1f s" % (rate, field.size, rays / 1e9, arrival[-1]))
        srv = Server(fields, pool_bytes=4 << 30, max_slots=64, max_tiles=16384, chunk_tiles=1024,
                     n_streams=args.serve_streams)
        t0 = time.time()
        lat, mk = srv.replay(field, cams, wh, arrival)
        stats = srv.stats()
        srv.close()
        log("server replay %.1fs: %s" % (time.time() - t0, stats))
        t0 = time.time()
        lat_b, mk_b = baseline(fields, field, cams, wh, arrival)
        log("baseline %.1fs" % (time.time() - t0))
        return {"rate": rate, "requests": int(field.size), "offered_grays_per_s": round(rays / arrival[-1] / 1e9, 4),
                "server": summary(lat, mk, rays), "per_request_launches": summary(lat_b, mk_b, rays),
                "server_stats": stats}

    main_run = run(args.serve_rate, args.serve_seconds, 55)
    sweep = [run(float(r), args.serve_sweep_seconds, 56 + k)
             for k, r in enumerate(x for x in args.serve_sweep.split(",") if x)]
    print(json.dumps({
        "metric": "serving: p50/p99 request latency and rays/s",
        "value": main_run["server"]["p99_ms"], "unit": "ms (p99)", "higher_is_better": False, "n_gpus": 1,
        "data": "synthetic",
        "config": {"workload": "%d resident light fields (%s); %d Poisson requests at %.0f/s; resolutions "
                               "256^2/512^2/1920x1080/2048^2" % (len(fields), args.serve_fields, main_run["requests"],
                                                                 args.serve_rate),
                   "offered_grays_per_s": main_run["offered_grays_per_s"]},
        "server": main_run["server"], "per_request_launches": main_run["per_request_launches"],
        "server_stats": main_run["server_stats"], "sweep": sweep,
    }), flush=True)


def grad_bench(args):
    """Relaxed forward render and its adjoint (gradients w.r.t. every residual
    value and every block shift) for the 16-view 512x512 differentiation
    workload; the loss gradient is 2 (render - target) against the integer
    decoder's render of the same views."""
    import torch

    import lfscene
    from paper_1902_09396_amd import lf

    cfg = lfscene.get_config("grad512")
    L = cfg["lf"]
    t0 = time.time()
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    stream = lf.encode(light, cfg["enc"])
    del light
    log("grad field: %d bytes, %.1fs" % (stream.size, time.time() - t0))
    field = lf.LightField(stream, device="cuda:0")
    cams_np = lfscene.make_views(cfg)
    V, wo, ho = cams_np.shape[0], cfg["views"]["wo"], cfg["views"]["ho"]
    cams = torch.from_numpy(cams_np).cuda()
    res, sh = field.export_params()
    sh = torch.floor(sh * 4.0) / 4.0 + 0.125
    target = field.render_views(cams, wo, ho)
    s = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(args.steps):
            r = fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps, r

    fwd_ms, out = timed(lambda: field.render_relaxed(res, sh, cams, wo, ho))
    g = 2.0 * (out - target)
    bwd_ms, (g_res, g_sh) = timed(lambda: field.render_backward(res, sh, cams, wo, ho, g))
    rays = V * wo * ho
    # compulsory bytes of one backward: every residual gradient and shift
    # gradient written once; the output gradient, the reference residual
    # planes (the shift gradients' taps) and the shifts read once
    info = field.info
    plane = field.width * field.height
    bwd_bytes = (4 * res.numel() + 8 * sh.shape[0] + 4 * V * 3 * wo * ho + 4 * 3 * info["n_refs"] * plane
                 + 8 * sh.shape[0])
    achieved = bwd_bytes / (bwd_ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "relaxed render + adjoint: rays/s through forward and backward",
        "value": round(rays / ((fwd_ms + bwd_ms) * 1e-3) / 1e9, 4), "unit": "Grays/s", "higher_is_better": True,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "17x17x512x512 field, 16 orbit views of 512x512; gradients w.r.t. %d residual "
                               "values and %d block shifts" % (res.numel(), sh.shape[0])},
        "forward_ms": round(fwd_ms, 3), "backward_ms": round(bwd_ms, 3),
        "gradient_bytes": int((res.numel() + sh.numel()) * 4),
        "nonzero_residual_grads": int((g_res != 0).sum().item()),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "lf_render_backward (all kernels)",
                     "compulsory_bytes": int(bwd_bytes)},
    }), flush=True)


def encode_bench(args):
    """Encoder side of the 17x17x512x512 field: the phase-shifted motion
    search of every level-0 predictive block (3 channels x 208 views x 1024
    blocks of 16x16, W = 8, quarter-pel refinement) as one lf_mc_search
    launch, and the whole-field encode on the GPU (every stage a kernel).  Search planes: channel c of each predictive view
    and of its cluster's reference view; the kernel's work does not depend on
    the values."""
    import torch

    import lfscene
    from paper_1902_09396_amd import lf

    cfg = lfscene.get_config(args.workload)
    L, enc = cfg["lf"], cfg["enc"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    lf.encode(light, enc)  # first call pays for module load and allocator growth
    torch.cuda.synchronize()
    t_dev = []
    for _ in range(3):
        t0 = time.time()
        dev_stream = lf.encode(light, enc)
        t_dev.append(time.time() - t0)
    t_dev = sorted(t_dev)[1]
    log("GPU encode %.3fs (median of 3), %d bytes" % (t_dev, dev_stream.size))

    nb, na, h, w = light.shape[:4]
    bs, win = enc["block"], enc["win"][0]
    pred_views = [(b, a) for b in range(nb) for a in range(na) if (a | b) & 1]
    ref_views = [(b, a) for b in range(0, nb, 2) for a in range(0, na, 2)]
    ref_index = {v: i for i, v in enumerate(ref_views)}
    pred = np.stack([light[b, a, :, :, c] for c in range(3) for (b, a) in pred_views]).astype(np.int16)
    ref = np.stack([light[b, a, :, :, c] for c in range(3) for (b, a) in ref_views]).astype(np.int16)
    nblk = (h // bs) * (w // bs)
    items = np.array([(c * len(pred_views) + j, c * len(ref_views) + ref_index[(b & ~1, a & ~1)], k)
                      for c in range(3) for j, (b, a) in enumerate(pred_views) for k in range(nblk)], dtype=np.int32)
    P, R, I = (torch.from_numpy(x).cuda() for x in (pred, ref, items))
    s = torch.cuda.current_stream()
    for _ in range(args.warmup):
        out = lf.mc_search(P, R, I, bs, win)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(args.steps):
        out = lf.mc_search(P, R, I, bs, win)
    b.record(s)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    n = items.shape[0]
    # algorithmic work: one |p - prediction| term per pixel, candidate and phase
    ops_per_block = bs * bs * (2 * (2 * win + 1) ** 2 + 2 * 48)
    achieved = n * ops_per_block / (ms * 1e-3) / 1e12
    peak = 256 * 64 * 2 * 2.4e9 / 1e12  # v_sad_u16: two pixel terms per lane and clock
    result = {
        "metric": "phase-shifted motion search: predictive blocks searched per second",
        "value": round(n / (ms * 1e-3) / 1e6, 3), "unit": "Mblocks/s", "higher_is_better": True,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "dtype": "i16/u32",
        "data": "synthetic",
        "config": {"workload": "level-0 search of the 17x17x512x512 field: %d blocks of %dx%d, W = %d, both "
                               "phases, quarter-pel refinement" % (n, bs, bs, win)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "Tops/s",
                     "frac": round(achieved / peak, 4), "traffic": None, "kernel": "k_mc_search",
                     "ops_per_block": ops_per_block},
        "encode_seconds": {"gpu_whole_field": round(t_dev, 3), "stream_bytes": int(dev_stream.size),
                           "note": "upload, every encoder stage on the GPU, copy-back of the stream"},
    }
    if not args.no_cpu_baseline:
        import oracle

        rng = np.random.default_rng(3)
        order = rng.permutation(n)[:200000]
        p32 = [pred[i].astype(np.int32) for i in sorted(set(items[order, 0]))]  # planes converted once, untimed
        p32 = dict(zip(sorted(set(items[order, 0])), p32))
        r32 = {i: ref[i].astype(np.int32) for i in sorted(set(items[order, 1]))}
        t0 = time.perf_counter()
        done = 0
        for idx in order:
            pi, ri, k = items[idx]
            oracle.mc_search(p32[pi], r32[ri], (k // (w // bs)) * bs, (k % (w // bs)) * bs, bs, win, True, False)
            done += 1
            if time.perf_counter() - t0 > 12.0:
                break
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(done / dt / 1e6, 6), "unit": "Mblocks/s", "cores": 1,
                                  "kind": "oracle", "sample": "%d random blocks of the same search, %.1f s" % (done, dt)}
    print(json.dumps(result), flush=True)


def decode_field(field, nb, na, h, w):
    """Every sample of every view, decoded on the GPU: uint8 [nb][na][h][w][3]."""
    import torch

    y, x = torch.meshgrid(torch.arange(h, dtype=torch.int32, device="cuda"),
                          torch.arange(w, dtype=torch.int32, device="cuda"), indexing="ij")
    yx = torch.stack([y.reshape(-1), x.reshape(-1)], 1)
    out = torch.empty((nb, na, h * w, 3), dtype=torch.uint8, device="cuda")
    coords = torch.empty((h * w, 4), dtype=torch.int32, device="cuda")
    coords[:, 2:] = yx
    for b in range(nb):
        for a in range(na):
            coords[:, 0] = b
            coords[:, 1] = a
            out[b, a] = field.decode_pixels(coords)
    return out.reshape(nb, na, h, w, 3)


def quant_sweep(args):
    """The render path of a workload from streams coded at several uniform
    quantisation steps (the 17x17x512^2 configuration names steps 2 to 8):
    stream size, PSNR of the decoded field, and the render kernel's time and
    roofline fraction on each."""
    import torch

    import lfscene
    from paper_1902_09396_amd import lf

    cfg = lfscene.get_config(args.workload)
    L = cfg["lf"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    light_dev = torch.from_numpy(light).cuda()
    cams = torch.from_numpy(lfscene.make_views(cfg)).cuda()
    V, wo, ho = cams.shape[0], cfg["views"]["wo"], cfg["views"]["ho"]
    out = torch.empty((V, 3, ho, wo), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    points = {}
    for step in (int(x) for x in args.quant_sweep.split(",") if x):
        e = dict(cfg["enc"])
        e["step"] = [step] * e["levels"]
        bpp, psnr, nbytes, _ = rd_point(light, e, light_dev)
        field = lf.LightField(lf.encode(light, e), device="cuda:0")
        fp = float(field.footprint_bytes(cams, wo, ho).sum())
        for _ in range(args.warmup):
            field.render_views(cams, wo, ho, out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(s)
        for _ in range(args.steps):
            field.render_views(cams, wo, ho, out)
        b.record(s)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        field.close()
        points[str(step)] = {"stream_bytes": nbytes, "bpp": round(bpp, 4), "psnr_db": round(psnr, 3),
                             "kernel_ms": round(ms, 4), "grays_per_s": round(V * wo * ho / (ms * 1e-3) / 1e9, 3),
                             "algorithmic_bytes_per_launch": int(fp),
                             "roofline_frac": round(fp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("step %d: %d bytes, %.2f dB, %.4f ms, frac %.4f" % (step, nbytes, psnr, ms, points[str(step)]["roofline_frac"]))
    print(json.dumps({"metric": "render path over quantisation steps", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": args.workload, "views": V, "width": wo, "height": ho}, "steps": points}),
          flush=True)


def rd_point(light, enc, light_dev=None):
    """(bits per light-field pixel, PSNR in dB over all RGB samples, stream
    bytes, bytes of the per-block random-access table inside the stream)."""
    import torch

    from paper_1902_09396_amd import lf

    stream = lf.encode(light, enc)
    nb, na, h, w = light.shape[:4]
    field = lf.LightField(stream, device="cuda:0")
    dec = decode_field(field, nb, na, h, w)
    field.close()
    src = light_dev if light_dev is not None else torch.from_numpy(light).cuda()
    mse = ((dec.to(torch.float64) - src.to(torch.float64)) ** 2).mean().item()
    psnr = float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)
    table_bytes = int(np.frombuffer(stream[136:144].tobytes(), np.uint64)[0])
    return 8.0 * stream.size / (nb * na * h * w), psnr, int(stream.size), table_bytes


def rd_bench(args):
    """Synthetic analogues of the paper's rate-distortion studies (Table 2:
    block size at threshold 75, window 16, tree height 3; Fig. 5: search
    window at block size 4, tree height 3; the threshold sweep of HMLFC
    against the plain hierarchy without motion compensation) on the
    17x17x512x512 synthetic field.  Streams come from the encoder with the
    GPU search; PSNR is over every decoded RGB sample of every view."""
    import torch

    import lfscene

    cfg = lfscene.get_config(args.workload)
    L = cfg["lf"]
    light = lfscene.make_lf(L["na"], L["nb"], L["h"], L["w"], L["spec"], L["seed"])
    light_dev = torch.from_numpy(light).cuda()
    H = 3

    def enc(block, win, thr, no_mc=False, step=4):
        e = dict(cfg["enc"])
        e.update(levels=H, block=block, step=[step] * H, win=[win] * H, t_ref=[thr] * H, t_pred=[thr] * H,
                 no_mc=no_mc)
        return e

    def point(name, e):
        t0 = time.time()
        bpp, psnr, nbytes, tbytes = rd_point(light, e, light_dev)
        log("%s: %.4f bpp, %.2f dB (%.1fs)" % (name, bpp, psnr, time.time() - t0))
        return {"bpp": round(bpp, 5), "bpp_without_table": round(bpp * (nbytes - tbytes) / nbytes, 5),
                "psnr_db": round(psnr, 3), "bytes": nbytes}

    table2 = {str(bs): point("block %d" % bs, enc(bs, 16, 75)) for bs in (2, 4, 8)}
    fig5 = {str(wn): point("window %d" % wn, enc(4, wn, 75)) for wn in (1, 2, 4, 8, 16)}
    thr = {}
    for t in (0, 25, 75, 150, 300, 600):
        thr[str(t)] = {"hmlfc": point("threshold %d" % t, enc(4, 16, t)),
                       "no_mc": point("threshold %d, no MC" % t, enc(4, 16, t, no_mc=True))}
    paper = residency_point(cfg, light, enc(4, 16, 75) | {"subpel": False}, args)
    print(json.dumps({
        "metric": "rate-distortion sweeps: bits per light-field pixel and PSNR",
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": "17x17x512x512 synthetic field, tree height %d, quantisation step 4" % H},
        "block_size_at_threshold75_window16": table2,
        "window_at_block4_threshold75": fig5,
        "threshold_at_block4_window16": thr,
        "residency_block4_window16_threshold75_integer_pel": paper,
    }), flush=True)


def residency_point(cfg, light, enc, args):
    """Reference residencies for one stream: dense planes, block tiles and
    per-pixel compressed sparse rows; resident reference bytes, arena bytes,
    and the 120-frame 512x512 orbit rendered with each (the tile kernel, and
    one thread per ray on every residency)."""
    import torch

    import lfscene
    from paper_1902_09396_amd import lf

    stream = lf.encode(light, enc)
    cams_np = lfscene.make_views(cfg)
    cams = torch.from_numpy(cams_np).cuda()
    wo, ho = cfg["views"]["wo"], cfg["views"]["ho"]
    out = {}
    for name, kw, per_ray in (("dense", {}, False), ("dense_per_ray", {}, True),
                              ("sparse", {"sparse_refs": True}, True), ("csr", {"csr_refs": True}, True)):
        field = lf.LightField(stream, device="cuda:0", **kw)
        img = torch.empty((cams.shape[0], 3, ho, wo), dtype=torch.float32, device="cuda")
        for _ in range(2):
            field.render_views(cams, wo, ho, out=img, per_ray=per_ray)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            field.render_views(cams, wo, ho, out=img, per_ray=per_ray)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        out[name] = {"ref_bytes": int(field.info["ref_bytes"]), "arena_bytes": int(field.info["arena_bytes"]),
                     "ms_per_frame": round(ms / cams.shape[0], 5)}
        log("%s residency: refs %.2f MB, arena %.2f MB, %.4f ms per 512x512 frame" %
            (name, field.info["ref_bytes"] / 1e6, field.info["arena_bytes"] / 1e6, ms / cams.shape[0]))
        field.close()
    out["stream_bytes"] = int(stream.size)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(stream, cams_np, wo, ho, n_rays):
    """The oracle on the host cores, on the same stream the GPU renders:
    a bounded random sample of the path's rays on every core (the reported
    value) and on one core, and random-access decoding of 10^7 samples."""
    import oracle

    o = oracle.OracleLF(stream)
    cores = oracle.set_threads(0)
    rng = np.random.default_rng(7)

    def rays_of(n):
        return np.stack([rng.integers(0, cams_np.shape[0], n), rng.integers(0, wo, n), rng.integers(0, ho, n)],
                        1).astype(np.int32)

    def rate(n):
        r = rays_of(n)
        t0 = time.perf_counter()
        o.render_rays(cams_np, wo, ho, r)
        return n, time.perf_counter() - t0

    # calibrate on a small sample, then size the timed samples to about 12 s and 4 s
    n0, t = rate(50000)
    per_ray = t / n0
    n = n_rays or int(min(max(12.0 / max(per_ray, 1e-9), 10000), 50_000_000))
    n, dt = rate(n)
    oracle.set_threads(1)
    n1, t1 = rate(max(2000, int(4.0 / max(per_ray * cores, 1e-9))))
    oracle.set_threads(0)
    # random-access decode (decode_at) of 10^7 uniformly random samples, every core
    nd = 10_000_000
    nb, na, h, w = o.nb, o.na, o.h, o.w
    coords = np.stack([rng.integers(0, nb, nd), rng.integers(0, na, nd), rng.integers(0, h, nd),
                       rng.integers(0, w, nd)], 1).astype(np.int32)
    t0 = time.perf_counter()
    o.decode_at(coords)
    td = time.perf_counter() - t0
    o.close()
    return {"value": round(n / dt / 1e9, 6), "unit": "Grays/s", "cores": cores, "kind": "oracle",
            "sample": "%d uniformly random rays of the step's views (seed 7), OpenMP over rays, %.1f s" % (n, dt),
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(n1 / t1 / 1e9, 8), "unit": "Grays/s",
                              "sample": "%d random rays, %.1f s" % (n1, t1)},
            "decode_at": {"value": round(nd / td / 1e6, 3), "unit": "Msamples/s", "cores": cores,
                          "sample": "10^7 uniformly random samples (b, a, y, x), %.1f s" % td}}


if __name__ == "__main__":
    main()
