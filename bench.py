"""Benchmark of the PVG rasterizer on one MI355X.

A step is one training-shaped iteration of the 1M-Gaussian, 1920x1280,
degree-3 workload: three cameras (yaw -45, 0, +45 degrees) at one time t, each
rendered as H(t) and as the flow-translated H^(t + dt) with dt = 0.05
(Eq. (12)), an L1 loss against a uniform target for each of the six images,
and the backward of all six into one set of parameter gradients.  Inputs are
synthetic (seeded) and resident in HBM before the timed region.

The six views run concurrently on side streams and share one per-Gaussian
adjoint pass; their lists stay resident from forward to backward.

Prints one JSON line: value = training-shaped iterations per second; the
forward-only rate (Mpix/s over the three H(t) renders), per-stage times from
HIP events recorded on the launch stream in a serial pass (one view at a
time), the dominant kernel's roofline, the serving workload and the
single-threaded CPU oracle timed on a bounded sample are extra fields.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd and fwd+bwd iters/s @1M Gaussians 1920x1280; serving p50/p99 ms"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# FP32 operations per evaluated (pixel, Gaussian) pair, counted from the
# kernels' arithmetic: forward 25 (incl. one exp), adjoint 70 (recomputed
# alpha, transmittance recovery, nine partial derivatives).
FLOPS_PER_PAIR = {"render_fwd": 25.0, "render_bwd": 70.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=None, help="override the Gaussian count")
    ap.add_argument("--period", type=int, default=200,
                    help="iterations of the timed training-loop period (the densify interval)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the 2k, 200k and 6M workloads")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the 200 req/s serving trace (its first 2 s are excluded from the statistics)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--profile-sky", action="store_true",
                    help="after the warm-up run only the sky adjoint's timing pass (both entry points) and print it")
    ap.add_argument("--profile-pass", action="store_true",
                    help="after the warm-up run only the serial per-stage pass (the one the roofline's kernel "
                         "times come from) and print its stage times: the run to put under a kernel profiler")
    return ap.parse_args()


def stage_bytes(stage, n, n_vis, M, Lst, visited, K, tiles, tile_passes, views=1):
    """Algorithmic HBM bytes of one invocation of a stage.  M: rectangle
    instances, Lst: listed (culled) instances, visited: (Gaussian, tile)
    records the adjoint writes and the gather reads."""
    if stage == "preprocess":
        return n * (68 + 12) + n_vis * (12 * K + 36)
    if stage == "compact":
        return n * 8 + n_vis * 8
    if stage == "depth_sort":
        return 4 * 16 * n_vis
    if stage == "scan_emit":
        # tile counts and offsets, each owner's record read by the count and
        # the write pass, and the listed instances written
        return n_vis * 16 + 2 * n_vis * 36 + Lst * 8
    if stage == "tile_sort":
        return tile_passes * 16 * Lst
    if stage == "ranges":
        return Lst * 4 + tiles * 8
    if stage == "grad_gather":
        # per visible Gaussian its record (40 B) in and nine sums out, the cut keys, the visited records
        return n * 4 + n_vis * (40 + 36) + tiles * 8 + visited * 36
    if stage == "preprocess_bwd":
        # per view: radii and the visible Gaussians' screen-space gradients; once:
        # the visible Gaussians' parameters in, every gradient entry out
        return views * (n * 4 + n_vis * 36) + n * (17 + 3 * K) * 4 + n_vis * (68 + 12 * K)
    return 0


# stages that are one kernel each (the roofline is reported for the dominant one)
SINGLE_KERNEL = {"preprocess": "k_preprocess", "render_fwd": "k_render_fwd", "render_bwd": "k_render_bwd",
                 "grad_gather": "k_grad_gather", "preprocess_bwd": "k_preprocess_bwd"}
KERNEL_SOURCES = ("render.hip", "blend.hpp", "preprocess.hip", "pvg_math.hpp", "pvg_internal.hpp")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_18561_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, scaled by the plain-copy calibration; None when there is none or
    when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_1M_1920x1280_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    return (rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_scale"]
            + rec["write_kib_per_dispatch"] * 1024 * rec["write_scale"])


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, rows_sampled=8):
    """The oracle (single thread, as it stands) on one camera's H(t) view of
    the same scene, forward and backward: FP32 per-Gaussian stage and
    instance sort of all Gaussians, FP32 compositing and the FP64 adjoint
    (the oracle's gradient path: the per-Gaussian chain of every Gaussian
    once, the compositing adjoint per tile) of `rows_sampled` tile rows
    spread evenly over the frame, the per-row parts scaled to the whole
    frame; the training-shaped step is six such views."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    scene, cam, t = cfg["scene"], cfg["cameras"][1], cfg["t"]
    GX, GY = oracle.grid(cam)
    W, H = cam["width"], cam["height"]
    t0 = time.perf_counter()
    pre = oracle.preprocess_f32(scene, cam, t)
    bins = oracle.bin_sort(pre, cam)
    t_setup = time.perf_counter() - t0
    rows = [int(r) for r in np.linspace(0, GY - 1, rows_sampled).round()]
    t_fwd = 0.0
    for r in rows:
        t1 = time.perf_counter()
        oracle.render_f32(pre, bins, cam, t, tiles=(r * GX, (r + 1) * GX))
        t_fwd += time.perf_counter() - t1
    sc64 = oracle.scene64(scene)
    mask = np.zeros(GX * GY, np.uint8)
    t1 = time.perf_counter()
    oracle.backward_f64(sc64, cam, t, 0.0, 0, (0.0, 0.0, 0.0), pre, bins, np.zeros((3, H, W)), tile_mask=mask)
    t_bwd_fixed = time.perf_counter() - t1
    dimg = np.zeros((3, H, W))
    rng = np.random.default_rng(0)
    for r in rows:
        mask[r * GX:(r + 1) * GX] = 1
        dimg[:, r * 16:(r + 1) * 16] = rng.standard_normal((3, 16, W))
    t1 = time.perf_counter()
    oracle.backward_f64(sc64, cam, t, 0.0, 0, (0.0, 0.0, 0.0), pre, bins, dimg, tile_mask=mask)
    t_bwd_rows = max(time.perf_counter() - t1 - t_bwd_fixed, 0.0)
    scale = GY / len(rows)
    t_view_fwd = t_setup + t_fwd * scale
    t_view = t_view_fwd + t_bwd_fixed + t_bwd_rows * scale
    views = 2 * len(cfg["cameras"])
    return {
        "value": 1.0 / (views * t_view),
        "unit": "iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one 1920x1280 H(t) view of the 1M-Gaussian scene through the single-threaded oracle: FP32 "
                   f"per-Gaussian stage + instance sort of all {scene['n']} Gaussians ({t_setup:.1f} s), FP32 "
                   f"compositing of {len(rows)}/{GY} tile rows spread over the frame ({t_fwd:.1f} s), the FP64 "
                   f"adjoint's per-Gaussian chain ({t_bwd_fixed:.1f} s) and its compositing adjoint on the same rows "
                   f"({t_bwd_rows:.1f} s); rows scaled to the frame, {views} such views per step"),
        "mpix_per_s_fwd": W * H / t_view_fwd / 1e6,
        "seconds_per_view": t_view,
        "host_cpu": host_cpu_model(),
        "host_cores_available": os.cpu_count(),
    }


def cpu_other_workloads():
    """The oracle (single thread) on the two small workloads in their own
    units, whole (no sampling): the 2k-Gaussian 128x96 forward (three
    repetitions) and one forward + backward of the 200k-Gaussian 960x640
    step (FP32 forward, FP64 adjoint of an L1-shaped upstream gradient)."""
    import numpy as np

    import gen
    import oracle
    out = {}
    cfg = gen.make_config(0)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    t0 = time.perf_counter()
    for _ in range(3):
        pre = oracle.preprocess_f32(scene, cam, t)
        bins = oracle.bin_sort(pre, cam)
        oracle.render_f32(pre, bins, cam, t)
    sec = (time.perf_counter() - t0) / 3
    out["forward_2k_128x96"] = {"mpix_per_s_fwd": cam["width"] * cam["height"] / sec / 1e6, "seconds": sec}
    cfg = gen.make_config(1)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    t0 = time.perf_counter()
    pre = oracle.preprocess_f32(scene, cam, t)
    bins = oracle.bin_sort(pre, cam)
    img = oracle.render_f32(pre, bins, cam, t)[0]
    dimg = np.sign(img.astype(np.float64) - 0.5) / (3 * H * W)
    oracle.backward_f64(oracle.scene64(scene), cam, t, 0.0, 0, (0.0, 0.0, 0.0), pre, bins, dimg)
    sec = time.perf_counter() - t0
    out["train_200k_960x640"] = {"iters_per_s": 1.0 / sec, "seconds": sec}
    return out


def config_legs(steps):
    """The other workloads in the headline's units, each with seeded
    synthetic inputs resident in HBM before its timed region:
    - 2k Gaussians, degree 0, 128x96 (forward only): Mpix/s;
    - 200k Gaussians, degree 3, 960x640 (forward + L1 backward): it/s;
    - 6M Gaussians (40% far field), degree 3, six 1920x1280 cameras at one t
      (forward + L1 backward of all six): it/s with the lists kept and with
      them rebuilt in the backward, and the peak device memory of each."""
    import torch

    import gen
    import paper_2311_18561_amd as pvg

    def timed(fn, reps, warm=2):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {}
    c = gen.make_config(0)
    p = [torch.from_numpy(c["scene"][f]).cuda() for f in pvg.FIELDS]
    view = [(c["cameras"][0], c["t"])]

    def fwd0():
        with torch.no_grad():
            pvg.render_views(p, view)

    s0 = timed(fwd0, max(50, 10 * steps))
    out["forward_2k_128x96"] = {"mpix_per_s_fwd": c["width"] * c["height"] / s0 / 1e6, "ms_per_render": s0 * 1e3,
                                "gaussians": c["scene"]["n"]}
    del p
    print("# config legs: 2k forward done", file=sys.stderr, flush=True)

    def fwd_bwd_leg(cfg, views, recompute):
        params = [torch.from_numpy(cfg["scene"][f]).cuda().requires_grad_(True) for f in pvg.FIELDS]
        tg = torch.stack([torch.from_numpy(x).cuda() for x in cfg["targets"]])

        def step():
            for q in params:
                q.grad = None
            imgs = pvg.pvg_render_views(params, views, recompute=recompute, stack=True)
            (pvg.l1_loss(imgs, tg) * len(views)).backward()

        step()
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        sec = timed(step, steps, warm=1)
        peak = torch.cuda.max_memory_allocated()
        del params, tg
        torch.cuda.empty_cache()
        return sec, peak

    c = gen.make_config(1)
    s1, peak1 = fwd_bwd_leg(c, [(c["cameras"][0], c["t"])], "auto")
    out["train_200k_960x640"] = {"iters_per_s": 1.0 / s1, "ms_per_step": s1 * 1e3, "gaussians": c["scene"]["n"],
                                 "peak_bytes": peak1}
    print("# config legs: 200k forward+backward done", file=sys.stderr, flush=True)
    c = gen.make_config(4)
    views = [(cam, c["t"]) for cam in c["cameras"]]
    s4k, peak4k = fwd_bwd_leg(c, views, False)
    s4r, peak4r = fwd_bwd_leg(c, views, True)
    out["train_6M_6x1920x1280"] = {
        "iters_per_s_kept_lists": 1.0 / s4k, "iters_per_s_recompute": 1.0 / s4r,
        "ms_per_step_kept_lists": s4k * 1e3, "ms_per_step_recompute": s4r * 1e3,
        "peak_bytes_kept_lists": peak4k, "peak_bytes_recompute": peak4r, "gaussians": c["scene"]["n"],
        "views": len(views), "mpix_per_step": len(views) * c["width"] * c["height"] / 1e6}
    print("# config legs: 6M forward+backward done", file=sys.stderr, flush=True)
    return out


SERVE_SCENES = ((500_000, 30), (1_000_000, 31), (2_000_000, 32), (3_000_000, 33))
SERVE_RATES = ((200.0, 3), (1200.0, 4))  # (requests per second, trace seed)


def serve_bench(seconds: float, warm: float = 2.0, high_seconds: float = 3.0):
    """The serving workload: four resident scenes (0.5M, 1M, 2M, 3M Gaussians,
    degree 3, driving-path layout), Poisson request streams, each request a
    random scene, a camera on the 100 m path (yaw in [-45, 45] degrees), t in
    [0, 1] and a resolution from {640x480, 960x640, 1920x1280}.  Each stream is
    replayed open loop (arrival times honoured; latency = result on the host -
    scheduled arrival) against the batched server and against the same server
    restricted to one request per launch and no overlap: at 200 requests/s
    and at a rate above what one-at-a-time service sustains.  Then the 200/s
    stream as a burst (all queued at once) gives the saturation throughput."""
    import threading

    import torch

    import gen
    import paper_2311_18561_amd as pvg
    from paper_2311_18561_amd.serve import Server

    scenes = []
    for n, seed in SERVE_SCENES:
        sc = gen.make_scene(n, seed, sh_degree=3, layout="path")
        scenes.append([torch.from_numpy(sc[f]).cuda() for f in pvg.FIELDS])
    traces = {rate: gen.make_trace(seed=seed, rate=rate, duration=seconds if rate <= 200.0 else high_seconds)
              for rate, seed in SERVE_RATES}
    keys = sorted({(r["camera"]["width"], r["camera"]["height"]) for tr in traces.values() for r in tr})
    bufs = {k: [torch.empty((3, k[1], k[0]), dtype=torch.float32, device="cuda") for _ in range(192)]
            for k in keys}

    def replay(srv, sids, trace, open_loop):
        tickets = [None] * len(trace)
        arrival_ns = [0] * len(trace)
        owner = {k: [None] * len(v) for k, v in bufs.items()}
        nxt = {k: 0 for k in bufs}
        done = threading.Event()
        results = [None] * len(trace)

        def waiter():
            for i in range(len(trace)):
                while tickets[i] is None:
                    time.sleep(0.0002)
                results[i] = srv.wait(tickets[i])
            done.set()

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.monotonic_ns()
        for i, r in enumerate(trace):
            cam = r["camera"]
            key = (cam["width"], cam["height"])
            slot = nxt[key]
            nxt[key] = (slot + 1) % len(bufs[key])
            prev = owner[key][slot]
            if prev is not None:
                while results[prev] is None:
                    time.sleep(0.0002)
            owner[key][slot] = i
            if open_loop:
                arrival_ns[i] = t0 + int(r["arrival"] * 1e9)
                delay = (arrival_ns[i] - time.monotonic_ns()) * 1e-9
                if delay > 0:
                    time.sleep(delay)
            tickets[i] = srv.submit(sids[r["scene"]], cam, r["t"], bufs[key][slot])
            if not open_loop:
                arrival_ns[i] = time.monotonic_ns()
        done.wait()
        th.join()
        return results, arrival_ns

    def summarize(trace, results, arrival_ns, skip_s):
        lat = []
        px = 0
        t_first = min(arrival_ns)
        kept = [(r, tr, a) for r, tr, a in zip(results, trace, arrival_ns) if (a - t_first) * 1e-9 >= skip_s]
        for r, tr, a in kept:
            assert r.status == 0, r.status
            lat.append((r.t_done_ns - a) * 1e-6)
            px += tr["camera"]["width"] * tr["camera"]["height"]
        span = (max(r.t_done_ns for r, _, _ in kept) - min(a for _, _, a in kept)) * 1e-9
        lat.sort()
        pct = lambda q: lat[min(len(lat) - 1, int(q * (len(lat) - 1) + 0.5))]
        return {"requests": len(kept), "p50_ms": pct(0.5), "p99_ms": pct(0.99), "mpix_per_s": px / span / 1e6,
                "req_per_s": len(kept) / span,
                "mean_batch": sum(r.batch_size for r, _, _ in kept) / max(1, len(kept))}

    out = {"trace": {"rates_per_s": [r for r, _ in SERVE_RATES],
                     "requests": {str(int(r)): len(tr) for r, tr in traces.items()},
                     "seconds": {str(int(r)): seconds if r <= 200.0 else high_seconds for r, _ in SERVE_RATES},
                     "warmup_s": warm, "scenes": [n for n, _ in SERVE_SCENES],
                     "resolutions": ["640x480", "960x640", "1920x1280"]}}
    modes = {"batched": dict(max_batch=8, max_inflight=2),
             "one_at_a_time": dict(max_batch=1, max_inflight=1)}
    base = traces[SERVE_RATES[0][0]]
    for name, kw in modes.items():
        with Server(use_graphs=True, max_batch_gaussians=24_000_000, max_batch_pixels=8 * 1920 * 1280,
                    instance_capacity=(1 << 30) - 1, **kw) as srv:
            sids = [srv.load_scene(p) for p in scenes]
            torch.cuda.synchronize()
            replay(srv, sids, base, open_loop=False)  # warm-up: builds the graphs
            print(f"# serving {name}: warm", file=sys.stderr, flush=True)
            out[name] = {}
            for rate, _ in SERVE_RATES:
                tr = traces[rate]
                res, arr = replay(srv, sids, tr, open_loop=True)
                out[name][f"rate_{int(rate)}"] = summarize(tr, res, arr, warm if rate <= 200.0 else 0.5)
                print(f"# serving {name} @ {rate:.0f}/s: {out[name][f'rate_{int(rate)}']}", file=sys.stderr,
                      flush=True)
            res, arr = replay(srv, sids, base, open_loop=False)
            sat = summarize(base, res, arr, 0.0)
            out[name]["saturation_mpix_per_s"] = sat["mpix_per_s"]
            out[name]["saturation_req_per_s"] = sat["req_per_s"]
            out[name]["retries"] = srv.stats()["retries"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_2311_18561_amd as pvg
    from paper_2311_18561_amd import _lib as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = gen.make_config(2, n=args.n)
    scene = cfg["scene"]
    N, K = scene["n"], (scene["sh_degree"] + 1) ** 2
    params = [torch.from_numpy(scene[f]).cuda().requires_grad_(True) for f in pvg.FIELDS]
    targets = [torch.from_numpy(x).cuda() for x in cfg["targets"]]
    cams, t, dt = cfg["cameras"], cfg["t"], cfg["dt"]
    W, H = cfg["width"], cfg["height"]
    lib = L.load()
    print(f"# workload: N={N} {W}x{H} views={len(cams)} t={t:.4f} dt={dt}", file=sys.stderr, flush=True)

    views = [(cam, t, d) for cam in cams for d in (0.0, dt)]
    view_targets = [tgt for tgt in targets for _ in (0.0, dt)]
    stacked_targets = torch.stack(view_targets)

    def train_step(recompute="auto"):
        # the six L1 losses (each the mean over its image), on the stacked images
        for p in params:
            p.grad = None
        imgs = pvg.pvg_render_views(params, views, recompute=recompute, stack=True)
        loss = pvg.l1_loss(imgs, stacked_targets) * len(views)  # = the sum of the six per-image means
        loss.backward()
        return loss

    # the step with the flexible-rendering channels (Sec. 3.1) and the sky
    # (Sec. 3.4) in the loss: each view composited over a learnable cube map
    # (faces of 1024 x 1024, rays jittered inside their pixel each step), L1
    # on the composite plus an L1 on the inverse normalized depth against a
    # sparse synthetic target (5% of the pixels, standing in for projected
    # LiDAR), the opacity entropy term with a synthetic sky mask (the top
    # eighth of each view) and the sparse velocity term on the velocity map,
    # weights 0.1, 0.05, 0.01 (Sec. 4); the backward also accumulates the
    # view-space gradient statistics of the adaptive control (Sec. 3.3), as
    # every training iteration of the densification phase does
    gch = torch.Generator(device="cuda").manual_seed(7)
    d_acc = torch.zeros(N, device="cuda")
    d_cnt = torch.zeros(N, device="cuda")
    V = len(views)
    sparse = (torch.rand((V, H, W), device="cuda", generator=gch) < 0.05).float()
    inv_depth_target = sparse / (5.0 + 45.0 * torch.rand((V, H, W), device="cuda", generator=gch))
    sky = torch.zeros((V, H, W), device="cuda")
    sky[:, : H // 8] = 1.0

    cube = torch.full((6, 3, 1024, 1024), 0.5, device="cuda").requires_grad_(True)

    def train_step_channels():
        for p in params:
            p.grad = None
        cube.grad = None
        imgs, dn, opac, vbar, _ = pvg.pvg_render_views(params, views, channels=True, normalized_depth=True,
                                                       densify_stats=(d_acc, d_cnt))
        jit = torch.rand((V, 2, H, W), device="cuda", generator=gch) - 0.5
        final = pvg.pvg_sky_composite_views(imgs, opac, cube, [v[0] for v in views], jit)
        o = opac.clamp(1e-6, 1.0 - 1e-6)
        inv = 1.0 / dn.clamp_min(1e-3)  # the inverse of the normalized depth
        loss = (pvg.l1_loss(final, stacked_targets) * V + 0.1 * (sparse * (inv - inv_depth_target).abs()).mean()
                + 0.05 * (-(o * o.log()).mean() - (sky * (1.0 - o).log()).mean()) + 0.01 * vbar.abs().mean())
        loss.backward()
        return loss

    def fwd_step():
        with torch.no_grad():
            pvg.render_views(params, [(cam, t) for cam in cams])

    for _ in range(args.warmup):
        train_step()
        fwd_step()
    torch.cuda.synchronize()
    # Python's cyclic collector: a full collection over the interpreter's
    # objects (torch's included) stalls the host for 40-80 ms, once every few
    # dozen steps, and the GPU waits for it.  Collect once now and move every
    # live object to the permanent generation, so later collections only scan
    # what the steps allocate.
    gc.collect()
    gc.freeze()
    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_mib} MiB read + {args.copy_mib} MiB written", file=sys.stderr, flush=True)
        del src, dst

    import ctypes as C

    def read_stages():
        out = {}
        for s, name in enumerate(L.STAGES):
            ms, calls, work = C.c_double(), C.c_int64(), C.c_int64()
            lib.pvg_profile_read(s, C.byref(ms), C.byref(calls), C.byref(work))
            out[name] = {"ms": ms.value, "calls": calls.value, "work": work.value}
        return out

    # Per-kernel durations come from a separate pass that runs the same six
    # renders one view at a time (single-view calls on one stream), since the
    # timed step overlaps views and a shared GPU stretches each launch.
    def serial_step():
        for p in params:
            p.grad = None
        loss = None
        for (cam, tt, d), tgt in zip(views, view_targets):
            l1 = pvg.l1_loss(pvg.pvg_render(params, cam, tt, d, recompute=False), tgt)
            loss = l1 if loss is None else loss + l1
        loss.backward()

    serial_steps = 2  # profiled serial steps

    def serial_stage_pass():
        serial_step()
        torch.cuda.synchronize()
        lib.pvg_profile_reset()
        lib.pvg_profile_enable(1)
        for _ in range(serial_steps):
            serial_step()
        torch.cuda.synchronize()
        lib.pvg_profile_collect()
        lib.pvg_profile_enable(0)
        stages = read_stages()
        lib.pvg_profile_reset()
        # one more serial step with the render kernels counting evaluated pairs
        # (the counts are deterministic: same inputs, same pairs)
        lib.pvg_profile_enable(2)
        serial_step()
        torch.cuda.synchronize()
        lib.pvg_profile_collect()
        lib.pvg_profile_enable(0)
        counted = read_stages()
        lib.pvg_profile_reset()
        for name in ("render_fwd", "render_bwd"):
            if counted[name]["calls"]:
                stages[name]["work"] = counted[name]["work"] / counted[name]["calls"] * stages[name]["calls"]
        return stages

    def sky_adjoint_pass(reps=20):
        """The sky adjoint alone (pvg_sky_composite_bwd and its deterministic
        form) on each camera's 1920x1280 view over the 1024^2 cube map, with
        jittered rays: microseconds per view from HIP events on the launch
        stream, after three untimed calls."""
        import ctypes
        from paper_2311_18561_amd.render import camera_struct
        gs = torch.Generator(device="cuda").manual_seed(5)
        g = torch.randn((3, H, W), device="cuda", generator=gs)
        op = torch.rand((H, W), device="cuda", generator=gs)
        jt = torch.rand((2, H, W), device="cuda", generator=gs) - 0.5
        d_op = torch.empty_like(op)
        d_cube = torch.zeros_like(cube)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        out = {}
        for name in ("pvg_sky_composite_bwd", "pvg_sky_composite_bwd_deterministic"):
            fn = getattr(lib, name)
            per_view = []
            for cam in cams:
                c = camera_struct(cam)
                args_c = (ctypes.byref(c), ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(op.data_ptr()),
                          ctypes.c_void_p(cube.data_ptr()), int(cube.shape[-1]), ctypes.c_void_p(jt.data_ptr()),
                          ctypes.c_void_p(d_op.data_ptr()), ctypes.c_void_p(d_cube.data_ptr()), st)
                for _ in range(3):
                    L.check(fn(*args_c))
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn(*args_c)
                e1.record()
                torch.cuda.synchronize()
                per_view.append(e0.elapsed_time(e1) / reps * 1e3)
            out[name] = per_view
        return out

    if args.profile_sky:
        print(json.dumps({"profile_sky": sky_adjoint_pass()}), flush=True)
        return

    if args.profile_pass:
        stages = serial_stage_pass()
        print(json.dumps({"profile_pass": {k: {"ms_per_call": v["ms"] / max(v["calls"], 1), "calls": v["calls"],
                                                "work": v["work"]} for k, v in stages.items()}}), flush=True)
        return

    # timed region: K training-shaped steps, stage events on the launch stream
    # each step's span on the launch stream from events recorded between the
    # steps (no synchronisation inside the timed region), and the host time
    # each step takes to return
    import importlib
    render_mod = importlib.import_module("paper_2311_18561_amd.render")
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    host_s = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev[0].record()
    for i in range(args.steps):
        h0 = time.perf_counter()
        train_step()
        host_s.append(time.perf_counter() - h0)
        step_ev[i + 1].record()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    step_ms = sorted(step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps))
    host_ms = sorted(h * 1e3 for h in host_s)
    policy_recompute = render_mod.last_recompute

    stages = serial_stage_pass()

    # the same step with the lists rebuilt in the backward (memory O(N + pixels + one view's instances))
    train_step(recompute=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        train_step(recompute=True)
    torch.cuda.synchronize()
    t_recompute = time.perf_counter() - t0

    # the same step with the depth and opacity channels and their loss terms
    train_step_channels()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        train_step_channels()
    torch.cuda.synchronize()
    t_channels = time.perf_counter() - t0
    ch_steps = []  # the same step timed one at a time (a rare slow step, e.g. a new allocation, shows as an outlier)
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        train_step_channels()
        torch.cuda.synchronize()
        ch_steps.append(time.perf_counter() - t0)
    ch_med = sorted(ch_steps)[len(ch_steps) // 2]
    sky_us = sky_adjoint_pass()

    # A period of the training loop (Sec. 4 and the appendix): PERIOD
    # iterations that each sample one view per camera at the next training
    # frame (frames 0.02 apart on the 100 m path, the camera centre moving
    # with t) with the temporal smoothing of Sec. 3.4 (dt = 0 with
    # probability eta = 0.5, else dt from a 1.5-frame span and the state at
    # t - dt translated by v_bar dt), render them with the channels over the
    # sky cube map, take the loss (1 - 0.2) L1 + 0.2 (1 - SSIM) + the depth,
    # opacity and velocity terms, run the backward with the densification
    # statistics, and step Adam on the Gaussians and on the cube map; the
    # period's first iteration ends with the densify pass (every 200
    # iterations), and the opacity reset (every 3000) is added amortized.  On
    # copies of the parameters, so the other measurements see the same scene.
    import random

    train_params = [p.detach().clone().requires_grad_(True) for p in params]
    adam = pvg.PVGAdam(train_params, pvg.default_lrs(30.0))
    train_cube = cube.detach().clone().requires_grad_(True)
    cube_adam = pvg.DenseAdam(train_cube, pvg.SKY_LR)
    yaws = (-45.0, 0.0, 45.0)
    sample_rng = random.Random(11)
    state = {"acc": torch.zeros(N, device="cuda"), "cnt": torch.zeros(N, device="cuda"), "frame": 0,
             "views": 0, "translated": 0}
    tg = stacked_targets[0::2].contiguous()  # each camera's target (the H(t) slots)
    n_frames, frame_dt = 50, 0.02
    dcfg = pvg.densify_config(30.0)

    def train_iteration(densify_after=False):
        nonlocal train_params
        f = state["frame"] % n_frames
        state["frame"] += 1
        t_f = f * frame_dt
        cams_f = [gen.yaw_camera(W, H, y, (0.0, 0.0, 100.0 * t_f)) for y in yaws]
        vs, _ = pvg.temporal_smoothing_views(cams_f, t_f, frame_dt, eta=0.5, rng=sample_rng)
        state["views"] += len(vs)
        state["translated"] += sum(1 for v in vs if v[2] != 0.0)
        for p in train_params:
            p.grad = None
        train_cube.grad = None
        Vf = len(vs)
        imgs, dn, opac, vbar, _ = pvg.pvg_render_views(train_params, vs, channels=True, normalized_depth=True,
                                                       densify_stats=(state["acc"], state["cnt"]))
        jit = torch.rand((Vf, 2, H, W), device="cuda", generator=gch) - 0.5
        final = pvg.pvg_sky_composite_views(imgs, opac, train_cube, [v[0] for v in vs], jit)
        o = opac.clamp(1e-6, 1.0 - 1e-6)
        inv = 1.0 / dn.clamp_min(1e-3)
        ssim = torch.stack([pvg.pvg_ssim(final[k], tg[k]).mean() for k in range(Vf)])
        rgb = 0.8 * pvg.l1_loss(final, tg) * Vf + 0.2 * (1.0 - ssim).sum()
        loss = (rgb + 0.1 * (sparse[:Vf] * (inv - inv_depth_target[:Vf]).abs()).mean()
                + 0.05 * (-(o * o.log()).mean() - (sky[:Vf] * (1.0 - o).log()).mean())
                + 0.01 * vbar.abs().mean())
        loss.backward()
        adam.step(train_params)
        cube_adam.step(train_cube)
        if densify_after:
            n_now = train_params[0].shape[1]
            dnz = torch.randn((8, n_now), device="cuda", generator=gch)
            new, rows = pvg.densify(train_params, state["acc"], state["cnt"], dnz, dcfg, adam.moments_rows())
            adam.set_moments_rows(rows)
            train_params = [p.requires_grad_(True) for p in new]
            m = train_params[0].shape[1]
            state["acc"], state["cnt"] = torch.zeros(m, device="cuda"), torch.zeros(m, device="cuda")

    for _ in range(2):
        train_iteration()
    torch.cuda.synchronize()
    n_period_start = train_params[0].shape[1]
    state["views"] = state["translated"] = 0
    t0 = time.perf_counter()
    for i in range(args.period):
        train_iteration(densify_after=(i == 0))
    torch.cuda.synchronize()
    t_period = time.perf_counter() - t0
    n_period_end = train_params[0].shape[1]
    reset_reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reset_reps):
        adam.reset_opacity(train_params, 0.01)
    torch.cuda.synchronize()
    t_reset = (time.perf_counter() - t0) / reset_reps
    t_full = t_period / args.period + t_reset / 3000.0
    del train_params, adam, train_cube, cube_adam

    # semantic rendering (Sec. 4.1): 19 class scores per Gaussian composited
    # over the six views and differentiated (vectors and Gaussians)
    sem = torch.randn((N, 19), device="cuda", generator=gch).requires_grad_(True)
    sem_w = torch.randn((V, 19, H, W), device="cuda", generator=gch)

    def semantic_step():
        for p in params:
            p.grad = None
        sem.grad = None
        torch.dot(pvg.pvg_render_semantic(params, views, sem).reshape(-1), sem_w.reshape(-1)).backward()

    semantic_step()
    torch.cuda.synchronize()
    sem_reps = 3
    t0 = time.perf_counter()
    for _ in range(sem_reps):
        semantic_step()
    torch.cuda.synchronize()
    t_sem = (time.perf_counter() - t0) / sem_reps
    del sem, sem_w

    # one adaptive-control pass (Sec. 3.3) on the statistics those steps
    # accumulated: r = 30 m (the foreground radius of Sec. 4), the densify
    # threshold 1.7e-4, g = 0.01 r, b = 0.1 r; the Adam moments of every
    # parameter row (2 x 65 rows) are carried along
    rows = sum(p.numel() // N for p in params)
    dcfg = pvg.densify_config(30.0)
    dnoise = torch.randn((8, N), device="cuda", generator=gch)
    moments = torch.zeros((2 * rows, N), device="cuda")
    new_params, _ = pvg.densify(params, d_acc, d_cnt, dnoise, dcfg, moments)  # warm
    n_after = int(new_params[0].shape[1])
    del new_params
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        new_params, new_m = pvg.densify(params, d_acc, d_cnt, dnoise, dcfg, moments)
        del new_params, new_m
    torch.cuda.synchronize()
    t_dens = (time.perf_counter() - t0) / reps
    # algorithmic bytes: the decisions read mean, scale, opacity and the two
    # statistics (36 B) and write a code byte; each output Gaussian reads its
    # parent's rows and moments and writes its own (rows and moments: 4 B x
    # (rows + 2 rows) each way)
    dens_bytes = N * (36 + 1) + N + n_after * 2 * 4 * 3 * rows

    # forward-only rate over the three H(t) renders
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_step()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    mpix_fwd = args.steps * len(cams) * W * H / t_fwd / 1e6

    # per-render counts for the byte model (the middle camera)
    img, T, nc, geom, bins = pvg.render(params, cams[1], t)
    n_vis = bins.num_visible
    Lst = bins.num_listed()
    M = int(geom.tiles.long().clamp(min=0).sum().item())  # rectangle instances
    GXt, GYt = (W + 15) // 16, (H + 15) // 16
    tiles = GXt * GYt
    rng = bins.ranges.long()
    lmax = torch.nn.functional.pad(nc, (0, GXt * 16 - W, 0, GYt * 16 - H)).reshape(GYt, 16, GXt, 16)
    lmax = lmax.amax(dim=(1, 3)).reshape(-1).long()
    visited = int(torch.minimum(lmax, rng[:, 1] - rng[:, 0]).sum().item())
    tile_passes = (max(1, (tiles - 1).bit_length()) + 7) // 8
    table = {}
    for name, st in stages.items():
        if st["calls"] == 0:
            continue
        per_launch_ms = st["ms"] / st["calls"]
        row = {"ms_per_step": st["ms"] / serial_steps, "ms_per_call": per_launch_ms, "calls_per_step":
               st["calls"] / serial_steps}
        if name in FLOPS_PER_PAIR:
            pairs = st["work"] / st["calls"]
            row.update(bound="alu", pairs_per_call=pairs,
                       tflops=pairs * FLOPS_PER_PAIR[name] / (per_launch_ms * 1e-3) / 1e12)
        else:
            b = stage_bytes(name, N, n_vis, M, Lst, visited, K, tiles, tile_passes, views=1)
            row.update(bound="hbm", bytes_per_call=b, gbs=b / (per_launch_ms * 1e-3) / 1e9)
        table[name] = row
    dom = max((k for k in table if k in SINGLE_KERNEL), key=lambda k: table[k]["ms_per_step"])
    d = table[dom]
    kernel = SINGLE_KERNEL[dom]
    traffic = measured_traffic(kernel)
    if d["bound"] == "alu":
        roof = {"bound": "alu", "kernel": kernel, "achieved": d["tflops"], "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": d["tflops"] / FP32_PEAK_TFLOPS, "traffic": traffic,
                "per_launch": {"pairs": d["pairs_per_call"], "flops_per_pair": FLOPS_PER_PAIR[dom],
                               "avg_ms": d["ms_per_call"]},
                "measured": "HIP events on the launch stream, serial pass (one view at a time)"}
    else:
        roof = {"bound": "hbm", "kernel": kernel, "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "per_launch": {"bytes": d["bytes_per_call"], "avg_ms": d["ms_per_call"]},
                "measured": "HIP events on the launch stream, serial pass (one view at a time)"}

    out = {
        "metric": METRIC,
        "value": args.steps / t_train,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_train / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pvg-train-step 1M Gaussians SH3 1920x1280, 3 cameras x {H(t), H^(t+0.05)}",
                   "gaussians": N, "width": W, "height": H, "views_per_step": 2 * len(cams)},
        "mpix_per_s_fwd": mpix_fwd,
        "iters_per_s_recompute": args.steps / t_recompute,
        "iters_per_s_channels": args.steps / t_channels,
        "iters_per_s_channels_median_step": 1.0 / ch_med,
        "iters_per_s_full_iteration": 1.0 / t_full,
        "sky_adjoint": {"us_per_view": sky_us,
                        "note": ("the sky composite's adjoint alone on each camera's 1920x1280 view over the 1024^2 "
                                 "cube map with jittered rays (HIP events, 20 calls after 3): the pixel-tile scatter "
                                 "the training steps use, and the deterministic texel-block gather")},
        "semantic_ms_per_step": t_sem * 1e3,
        "semantic_note": ("pvg_render_semantic forward and backward of 19 class scores per Gaussian over the six "
                          "views: one list walk per view for all 19 channels, forward and adjoint, and the loss "
                          "<maps, w> for a fixed random w"),
        "full_iteration_note": (f"a {args.period}-iteration period of the training loop (timed whole): each "
                                "iteration samples one view per camera (3) at the next frame with the temporal "
                                "smoothing of Sec. 3.4 (eta = 0.5, dt from a 1.5-frame span), renders the channels "
                                "over the 1024^2 sky cube map, takes (1 - 0.2) L1 + 0.2 (1 - SSIM) with the depth, "
                                "opacity and velocity terms, runs the backward with the densification statistics and "
                                "steps Adam on the Gaussians (pvg_adam_step) and on the cube map (pvg_adam_dense); "
                                "the first iteration ends with the densify pass (every 200 iterations) and the "
                                "opacity reset (every 3000) is added amortized"),
        "full_iteration": {"period": args.period, "gaussians_before": n_period_start,
                           "gaussians_after": n_period_end, "ms_per_period": t_period * 1e3,
                           "opacity_reset_ms": t_reset * 1e3, "views_rendered": state["views"],
                           "views_translated": state["translated"]},
        "densify": {"ms_per_pass": t_dens * 1e3, "gaussians_in": N, "gaussians_out": n_after,
                    "statistics_views": int(d_cnt.max().item()), "GB_per_s": dens_bytes / t_dens / 1e9,
                    "note": ("pvg_densify_plan + pvg_densify_apply on the channel steps' statistics (r = 30, "
                             "threshold 1.7e-4, g = 0.01 r, b = 0.1 r), Adam moments carried; wall time per pass "
                             "including the count read-back and the output allocation")},
        "channels_note": ("the same step with pvg_render_views(channels=True, normalized_depth=True): normalized "
                          "depth sum T alpha z / sum T alpha, opacity 1 - final_T, velocity and staticness maps "
                          "rendered, each view composited over a learnable 6 x 3 x 1024 x 1024 sky cube map with "
                          "jittered rays (pvg_sky_composite, its gradient into the cube map included); L1 on the "
                          "composite, an inverse-depth L1 on 5% of the pixels, the opacity entropy term with a sky "
                          "mask and the sparse velocity term, weights 0.1, 0.05, 0.01 (synthetic targets); the "
                          "backward also accumulates the adaptive control's view-space gradient statistics"),
        "lists": ("rebuilt in the backward" if policy_recompute else "kept from the forward") +
                 " (recompute='auto': kept while they fit in a tenth of HBM)",
        "step_ms": {"mean": sum(step_ms) / len(step_ms), "median": step_ms[len(step_ms) // 2], "min": step_ms[0],
                    "max": step_ms[-1], "measured": "events on the launch stream between consecutive steps"},
        "host_ms_per_step": {"median": host_ms[len(host_ms) // 2], "max": host_ms[-1],
                             "note": "host time until the step's launches return (the forward waits for binning)"},
        "instances_per_render": {"rectangle": M, "listed": Lst, "adjoint_records": visited},
        "visible_per_render": n_vis,
        "roofline": roof,
        "stages": table,
        "stages_note": ("per-kernel times of a serial pass of the same six renders through the single-view calls "
                        "(the timed step runs views concurrently on side streams and adds all views' per-Gaussian "
                        "adjoints in one pass)"),
    }
    if not args.no_configs:
        del params, targets
        torch.cuda.empty_cache()
        params = targets = None
        out["other_workloads"] = config_legs(args.steps)
    if not args.no_serve:
        del params, targets
        torch.cuda.empty_cache()
        out["serving"] = serve_bench(args.serve_seconds)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
        out["cpu_baseline"]["other_workloads"] = cpu_other_workloads()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
