"""Benchmark: fwd+bwd Mpix/s of the Beta-splatting rasterizer on one MI355X,
batched multi-view (one call per stage, replayed from a HIP graph) vs per-view
(the same calls once per view, eager).

    python bench.py [--steps K] [--warmup W] [--repeats R] [--config 3] [--no-cpu-baseline]

A step is one training iteration of the whole hot path over every view:
preprocess -> bin/sort -> forward -> L1 loss gradient -> backward (gradients
of every splat parameter).  Inputs are resident in HBM before timing starts.
`value` comes from K steps timed together; the step-time distribution
(median, p10, p90) from R more replays timed one by one with HIP events, and
the forward-only rate from R replays of a graph of the forward half.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published (packed FP32, an FMA counted as 2)
# The same chip without packed FP32 (which this build does not issue): 256 CUs
# x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-operations/s, 78.6 TFLOP/s with
# an FMA counted as 2.
LANE_OPS_PEAK_T = 256 * 64 * 2.4e9 / 1e12

# Algorithmic operations per (pixel, pair) of the reverse raster pass, two
# counting conventions:
#  - per operation (each add, multiply, FMA, compare or transcendental is 1):
#    6 for a support test that rejects the pair (r^2 >= 1), 47 for a pair
#    with r^2 < 1 (its test, the reverse arithmetic of Eq. 6 with two
#    transcendentals, and its share of the ten per-splat sums);
#  - FLOP with an FMA counted as 2: 9 per support test (evaluated pair) and
#    68 more per pair with r^2 < 1.
OPS_BWD_REJECT = 6
OPS_BWD_CONTRIB = 47
FLOP_TEST = 9
FLOP_FWD_CONTRIB = 15
FLOP_BWD_CONTRIB = 68


def step_bytes(q_floats: int, n: int, visible: int, pairs: int, pixels: int) -> int:
    """Algorithmic HBM bytes of one training step (batched): parameters read
    twice and gradients written once (12 Q N), 128 B per visible record
    (projection record, depth, count written; read by the sort; screen-space
    gradient written and read), 124 B per (tile, splat) pair (emission, one
    stable sort pass, raster reads in both directions), 40 B per pixel (image,
    T, last index, dL/dimage)."""
    return 12 * q_floats * n + 128 * visible + 124 * pairs + 40 * pixels


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_counters_config3.txt")
TRAFFIC_SOURCES = ("paper_2501_18630_amd/csrc/raster.hip", "paper_2501_18630_amd/csrc/wave_reduce.h",
                   "paper_2501_18630_amd/csrc/dbs_internal.h")


def measured_traffic(workload: str):
    """HBM bytes per launch of the raster reverse pass from the committed
    counter summary (TCC read and write requests weighted by their size, checked
    against copies of known size), or None when the summary is for another
    workload or the kernel sources changed since it was taken."""
    import hashlib
    try:
        fields = dict(line.split(": ", 1) for line in open(TRAFFIC_FILE).read().splitlines()
                      if line.startswith("traffic_"))
    except OSError:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("traffic_sources_sha256") != h.hexdigest() or fields.get("traffic_workload") != workload:
        return None
    return int(fields["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=50,
                    help="graph replays timed one by one with HIP events for the step-time distribution")
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--tile", default="auto", help="WxH, or auto (autotuned, outside the timed region)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pixels", type=int, default=2048)
    ap.add_argument("--cpu-sample-pixels-1t", type=int, default=128)
    ap.add_argument("--step-only", action="store_true",
                    help="only the batched step (warm-up, then K timed steps): the run profiled with counters")
    ap.add_argument("--copy-calibration", choices=["full", "half-lines"], default=None,
                    help="only copy a buffer and exit (reference for the HBM byte counters): 'full' copies "
                         "1 GiB; 'half-lines' reads the first 32 bytes of every 64-byte line of 1 GiB")
    return ap.parse_args()


def timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def step_distribution(fn, repeats):
    """Per-step milliseconds of `repeats` calls, each bracketed by HIP events
    on torch's current stream (the stream the graph replays on)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(repeats + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for k in range(repeats):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(repeats)])
    return {"n": repeats, "median_ms": round(float(np.median(ms)), 4),
            "p10_ms": round(float(np.percentile(ms, 10)), 4), "p90_ms": round(float(np.percentile(ms, 90)), 4),
            "min_ms": round(float(ms.min()), 4), "max_ms": round(float(ms.max()), 4)}


def forward_graph(rast, params):
    """preprocess -> bin/sort -> forward of every view, captured in one HIP
    graph (the rendering half of the step, comparable in kind to a frame
    render time)."""
    import torch
    outputs = rast.new_outputs()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rast.preprocess(params)
        rast.bin_sort()
        rast.render_fwd(*outputs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rast.preprocess(params)
        rast.bin_sort()
        rast.render_fwd(*outputs)
    torch.cuda.synchronize()
    return g, outputs


def stage_times(rast, step, steps):
    """Average ms of each stage of the batched step, HIP events recorded on
    torch's current stream, which is the stream the library launches on."""
    import torch
    names = ("preprocess", "bin_sort", "raster_fwd", "l1_loss", "raster_bwd", "project_bwd")
    acc = {k: 0.0 for k in names}
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record()
        rast.preprocess(step.params)
        ev[1].record()
        rast.bin_sort()
        ev[2].record()
        rast.render_fwd(step.image, step.final_T, step.last)
        ev[3].record()
        rast.l1_loss(step.image, step.target, step.scale, step.dL, step.loss)
        ev[4].record()
        rast.raster_bwd(step.dL, step.final_T, step.last)
        ev[5].record()
        rast.project_bwd(step.params, step.grads, store=True)   # as the step runs it
        ev[6].record()
        torch.cuda.synchronize()
        for k, name in enumerate(names):
            acc[name] += ev[k].elapsed_time(ev[k + 1])
    return {k: v / steps for k, v in acc.items()}


def forward_stage_times(rast, params, outputs, steps):
    """Average ms of preprocess, bin/sort and raster forward (HIP events on
    torch's current stream, the library's stream)."""
    import torch
    names = ("preprocess", "bin_sort", "raster_fwd")
    acc = {k: 0.0 for k in names}
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        rast.preprocess(params)
        ev[1].record()
        rast.bin_sort()
        ev[2].record()
        rast.render_fwd(*outputs)
        ev[3].record()
        torch.cuda.synchronize()
        for k, name in enumerate(names):
            acc[name] += ev[k].elapsed_time(ev[k + 1])
    return {k: v / steps for k, v in acc.items()}


def gaussian_sh_times(scene, cams, cfg, steps):
    """Forward of the Gaussian-kernel + degree-3 SH comparison mode on the same
    scene and views: with the same scales (its 3-sigma support is 3x as wide
    as the Beta kernel's r < 1) and with scales / 3 (the same support)."""
    import torch
    from paper_2501_18630_amd import renderer, scenes
    n = scene["means"].shape[0]
    out = {}
    for name, factor in (("same_scales", 1.0), ("same_support", 1.0 / 3.0)):
        g = scenes.gaussian_sh(scene, seed=7, scale_factor=factor)
        params = renderer.to_device(g)
        gcfg = renderer.RasterConfig(tile_w=cfg.tile_w, tile_h=cfg.tile_h, batch=cfg.batch, kernel="gaussian_sh")
        rast = renderer.Rasterizer(cams, n, g["lobe_betas"].shape[1], gcfg, headroom=1.05)
        outputs = rast.forward(params)
        pairs = int(rast.counts[1].item())
        t = forward_stage_times(rast, params, outputs, steps)
        assert int(rast.overflow.item()) == 0
        out[name] = {k + "_ms": round(v, 4) for k, v in t.items()}
        out[name]["fwd_ms"] = round(sum(t.values()), 4)
        out[name]["pairs"] = pairs
        del rast, params, outputs
        torch.cuda.empty_cache()
    return out


def composite_loss_times(rast, step, steps, lam_ssim=0.2, lam_reg=0.01):
    """Average ms of the composite-loss kernels of Sec. 3.4 on the step's
    rendered images (the benchmark step itself uses L1): the photometric term
    with SSIM, and the regularisers."""
    import torch
    t_p = t_r = 0.0
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        rast.photometric_loss(step.image, step.target, lam_ssim, step.dL, step.loss)
        ev[1].record()
        rast.regularizer(step.params, lam_reg, lam_reg, step.grads, step.loss)
        ev[2].record()
        torch.cuda.synchronize()
        t_p += ev[0].elapsed_time(ev[1])
        t_r += ev[1].elapsed_time(ev[2])
    return t_p / steps, t_r / steps


def mcmc_times(params, n, m, steps, tau=0.005):
    """Average ms of the kernel-agnostic MCMC step of Sec. 3.4 over the scene
    (relocation of primitives with o <= tau, positional noise), on a copy of
    the parameters; not part of the benchmark step."""
    import torch
    from paper_2501_18630_amd import renderer
    mc = renderer.MCMC(n, m)
    g = torch.Generator(device="cuda").manual_seed(7)
    rand = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
    z = torch.randn(n, 3, device="cuda", generator=g)
    t_r = t_n = 0.0
    moved = 0
    for _ in range(steps):
        p = {k: v.clone() for k, v in params.items()}
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        cnt = mc.relocate(p, tau, rand)
        ev[1].record()
        mc.noise(p, z, 0.01, 5e4)
        ev[2].record()
        torch.cuda.synchronize()
        t_r += ev[0].elapsed_time(ev[1])
        t_n += ev[1].elapsed_time(ev[2])
        moved = int(cnt.item())
    return t_r / steps, t_n / steps, moved


def work_counts(rast, step):
    """Pair counts and evaluated / contributing (pixel, pair) counts of the
    last step, from the library's counting pass (outside the timed region)."""
    counts = {"pairs": int(rast.counts[1].item()), "visible": int(rast.counts[0].item())}
    counts.update(rast.stats(step.final_T, step.last))
    return counts


def atomic_count(rast, step):
    """Global float atomics one raster reverse pass issues (one per non-zero
    (tile, splat, value) sum), from the counting build on the step's last
    state; the projection reverse that follows clears the accumulator again.
    Outside the timed region."""
    import torch
    cnt = torch.zeros(1, dtype=torch.int64, device=rast.device)
    rast.raster_bwd(step.dL, step.final_T, step.last, atomics=cnt)
    rast.project_bwd(step.params, step.grads)
    return int(cnt.item())


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cams, n_pixels: int, n_pixels_1t: int, seed: int = 5):
    """The oracle, as it is, on bounded samples: fwd + bwd of random pixels of
    the first view (every splat of the scene is projected and depth-sorted for
    that view, then each sampled pixel is composited by brute force over all
    of them), on all the host threads OpenMP is given and on one thread."""
    import oracle
    cam = cams[0]
    rng = np.random.default_rng(seed)
    amax, teps = float(np.float32(0.99)), float(np.float32(1e-4))
    s64 = {k: np.ascontiguousarray(v, np.float64) for k, v in scene.items()}

    def run(k):
        pix = np.stack([rng.integers(0, cam["width"], k), rng.integers(0, cam["height"], k)], 1)
        dl = rng.standard_normal((k, 3))
        t0 = time.perf_counter()
        oracle.render(s64, cam, amax, teps, pixels=pix)
        oracle.render_bwd(s64, cam, amax, teps, dl, pixels=pix)
        return time.perf_counter() - t0

    want = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = oracle.set_threads(want)
    dt = run(n_pixels)
    oracle.set_threads(1)
    dt1 = run(n_pixels_1t)
    oracle.set_threads(cores)
    where = f"random pixels of view 0 ({cam['width']}x{cam['height']}) over all {scene['means'].shape[0]} splats"
    return {"value": n_pixels / dt / 1e6, "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"fwd+bwd of {n_pixels} {where}, {dt:.1f} s on {cores} threads",
            "single_thread": {"value": n_pixels_1t / dt1 / 1e6, "unit": "Mpix/s", "cores": 1,
                              "sample": f"fwd+bwd of {n_pixels_1t} {where}, {dt1:.1f} s"},
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(a multi-GPU run would shard the views across GPUs)"}))
        sys.exit(2)
    import torch
    from paper_2501_18630_amd import renderer, scenes

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        if args.copy_calibration == "full":
            dst = torch.empty_like(src)
            dst.copy_(src)
            moved = {"read_bytes": src.numel() * 4, "write_bytes": src.numel() * 4}
        else:
            half = src.view(-1, 16)[:, :8]   # 32 B of each 64 B line
            dst = torch.empty(half.shape, dtype=torch.float32, device="cuda")
            dst.copy_(half)
            moved = {"read_bytes": half.numel() * 4, "lines_touched_bytes": src.numel() * 4,
                     "write_bytes": dst.numel() * 4}
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": args.copy_calibration, **moved}))
        return

    t0 = time.perf_counter()
    scene, cams = scenes.CONFIGS[args.config]()
    n, m = scene["means"].shape[0], scene["lobe_betas"].shape[1]
    log(f"scene: config {args.config}, {n} splats, {m} lobes, {len(cams)} views "
        f"({time.perf_counter() - t0:.1f} s)")
    params = renderer.to_device(scene)
    targets = [scenes.target_image(c["height"], c["width"], seed=1 + v) for v, c in enumerate(cams)]
    target_flat = torch.as_tensor(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    X = sum(c["width"] * c["height"] for c in cams)
    if args.tile == "auto":
        from paper_2501_18630_amd import autotune
        t0 = time.perf_counter()
        cfg = autotune.tune(cams, params, target_flat, log=log)
        log(f"autotuned: {cfg.tile_w}x{cfg.tile_h} batch {cfg.batch} ({time.perf_counter() - t0:.1f} s)")
        torch.cuda.empty_cache()
    else:
        tw, th = (int(x) for x in args.tile.split("x"))
        cfg = renderer.RasterConfig(tile_w=tw, tile_h=th, batch=args.batch)
    tw, th = cfg.tile_w, cfg.tile_h

    rast = renderer.Rasterizer(cams, n, m, cfg)
    step = renderer.TrainStep(rast, params, target_flat, headroom=1.1, use_graph=True)
    for _ in range(args.warmup):
        step.run()
    torch.cuda.reset_peak_memory_stats()
    t_batched = timed(step.run, args.steps)
    peak_mem = torch.cuda.max_memory_allocated()
    free_b, total_b = torch.cuda.mem_get_info()   # hipMemGetInfo, with every buffer of the step held
    assert not step.overflowed()
    log(f"batched: {t_batched * 1e3:.3f} ms/step")
    if args.step_only:
        print(json.dumps({"ms_per_step": round(t_batched * 1e3, 4), "steps": args.steps,
                          "config": f"config{args.config}, tile {tw}x{th}, batch {cfg.batch}"}), flush=True)
        return
    dist = step_distribution(step.run, args.repeats)
    log(f"batched step over {args.repeats} replays: {dist}")
    fwd_g, fwd_out = forward_graph(rast, params)
    for _ in range(args.warmup):
        fwd_g.replay()
    fwd_dist = step_distribution(fwd_g.replay, args.repeats)
    assert int(rast.overflow.item()) == 0
    log(f"batched forward over {args.repeats} replays: {fwd_dist}")
    del fwd_g, fwd_out

    per_view = None
    if not args.no_per_view:
        steps_v = []
        off = 0
        for v, c in enumerate(cams):
            npx = c["width"] * c["height"]
            r = renderer.Rasterizer([c], n, m, cfg)
            steps_v.append(renderer.TrainStep(r, params, target_flat[3 * off:3 * (off + npx)], headroom=1.1,
                                              use_graph=False))
            off += npx

        def run_views():
            for s in steps_v:
                s.run()

        for _ in range(args.warmup):
            run_views()
        t_pv = timed(run_views, args.steps)
        per_view = X / t_pv / 1e6
        log(f"per-view: {t_pv * 1e3:.3f} ms/step")
        del steps_v

    st = stage_times(rast, step, max(3, args.steps // 2))
    log("stages (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in st.items()))
    wc = work_counts(rast, step)
    log(f"work: {wc}")
    n_atomics = atomic_count(rast, step)
    log(f"raster reverse: {n_atomics} global float atomics per pass")
    t_photo, t_reg = composite_loss_times(rast, step, max(3, args.steps // 2))
    log(f"composite loss (ms): photometric {t_photo:.3f}, regularisers {t_reg:.3f}")
    t_reloc, t_noise, n_moved = mcmc_times(params, n, m, 3)
    log(f"mcmc (ms): relocate {t_reloc:.3f} ({n_moved} moved), noise {t_noise:.3f}")
    gsh = gaussian_sh_times(scene, cams, cfg, 3)
    gsh["beta_fwd_ms"] = round(st["preprocess"] + st["bin_sort"] + st["raster_fwd"], 4)
    log(f"gaussian+SH forward (ms): {gsh}")

    mpix = X / t_batched / 1e6
    q_floats = 15 + 6 * m
    sb = step_bytes(q_floats, n, wc["visible"], wc["pairs"], X)
    # dominant kernel: the raster reverse pass; ALU-bound (support tests plus
    # the reverse arithmetic of contributing pairs), priced against FP32 peak
    bwd_flops = wc["bwd_evaluated"] * FLOP_TEST + wc["contributing"] * FLOP_BWD_CONTRIB
    bwd_ops = (wc["bwd_evaluated"] - wc["contributing"]) * OPS_BWD_REJECT + wc["contributing"] * OPS_BWD_CONTRIB
    t_bwd = st["raster_bwd"] * 1e-3
    achieved = bwd_ops / t_bwd / 1e12
    achieved_flop = bwd_flops / t_bwd / 1e12
    fwd_flops = wc["fwd_evaluated"] * FLOP_TEST + wc["contributing"] * FLOP_FWD_CONTRIB
    result = {
        "metric": "fwd+bwd Mpix/s, batched vs per-view, 1 MI355X, img err<=1e-5 vs FP64",
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_batched * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"config{args.config}: {len(cams)} views (sum {X} px), {n} splats, "
                               f"{m} lobes, tile {tw}x{th}, batch {cfg.batch}"
                               f"{' (autotuned)' if args.tile == 'auto' else ''}, batched + hipGraph",
                   "views": len(cams), "pixels": X, "splats": n, "lobes": m},
        "step_ms": dist,
        "forward": {"value": round(X / (fwd_dist["median_ms"] * 1e-3) / 1e6, 3), "unit": "Mpix/s",
                    "ms": fwd_dist, "what": "preprocess -> bin/sort -> raster forward of every view, one HIP graph"},
        "peak_device_memory_GiB": round(peak_mem / 2**30, 2),
        "device_memory_used_GiB": round((total_b - free_b) / 2**30, 2),
        "per_view_value": round(per_view, 3) if per_view else None,
        "batched_speedup": round(mpix / per_view, 3) if per_view else None,
        "roofline": {"kernel": "raster_bwd_kernel", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(f"config {args.config}, tile {tw}x{th}, batch {cfg.batch}"),
                     "ms_per_launch": round(st["raster_bwd"], 4),
                     "counting": f"{OPS_BWD_REJECT} operations per rejected support test, {OPS_BWD_CONTRIB} per "
                                 "pair with r^2 < 1 (each add, multiply, FMA, compare or transcendental is one)",
                     "ops_per_launch": bwd_ops,
                     "peak_basis": "published FP32 vector peak (packed FP32, FMA = 2)",
                     "frac_of_issue_peak": round(achieved / LANE_OPS_PEAK_T, 4),
                     "issue_peak": {"value": round(LANE_OPS_PEAK_T, 2), "unit": "T lane-ops/s",
                                    "basis": "non-packed FP32 issue: 256 CUs x 64 lanes x 2.4 GHz"},
                     "flop_count": {"flops_per_launch": bwd_flops, "achieved_TFLOPs": round(achieved_flop, 3),
                                    "counting": f"FMA = 2: {FLOP_TEST} per support test, {FLOP_BWD_CONTRIB} more "
                                                "per pair with r^2 < 1",
                                    "frac_of_157.3": round(achieved_flop / FP32_VECTOR_PEAK_TFLOPS, 4),
                                    "frac_of_78.6_non_packed": round(achieved_flop / (2 * LANE_OPS_PEAK_T), 4)}},
        "step_hbm": {"algorithmic_bytes": sb, "achieved_GBs": round(sb / t_batched / 1e9, 1),
                     "peak_GBs": HBM_PEAK_GBS, "frac": round(sb / t_batched / 1e9 / HBM_PEAK_GBS, 4)},
        "raster_fwd_tflops": round(fwd_flops / (st["raster_fwd"] * 1e-3) / 1e12, 3),
        "stage_ms": {k: round(v, 4) for k, v in st.items()},
        # not in the step: the composite loss of the paper's training (lambda_SSIM = 0.2)
        "composite_loss": {"photometric_ms": round(t_photo, 4), "regularizer_ms": round(t_reg, 4),
                           "photometric_GBs": round(12 * 3 * X / (t_photo * 1e-3) / 1e9, 1)},
        # not in the step: the MCMC step of Sec. 3.4 over all splats (dead: o <= 0.005)
        "mcmc": {"relocate_ms": round(t_reloc, 4), "noise_ms": round(t_noise, 4), "relocated": n_moved},
        "gaussian_sh_forward": gsh,
        "work": wc,
        "global_atomics": {"per_raster_bwd": n_atomics,
                           "per_s": round(n_atomics / (st["raster_bwd"] * 1e-3), 1),
                           "bytes_added": 4 * n_atomics},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene, cams, args.cpu_sample_pixels, args.cpu_sample_pixels_1t)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
