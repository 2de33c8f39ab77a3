"""Autotuner for the raster launch shape: tile shape x LDS batch depth.

For a given set of views and scene size it times the whole graph-captured
training step (preprocess -> bin/sort -> forward -> L1 -> backward) for every
built (tile_w, tile_h, batch), then re-times the few fastest with more steps,
in alternating order, and keeps the fastest of those.  A warm-up run of the
first shape precedes the sweep so that the first shapes timed are not
charged for clock ramp-up.  Results are cached in a
JSON file keyed by the GPU architecture, the HIP runtime and library
versions, the view resolutions and the splat and lobe counts, so a workload
is tuned once per machine type and software stack.

    cfg = autotune.tune(cams, params, target)      # RasterConfig
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import renderer

CANDIDATES = [(16, 16), (16, 8), (8, 8), (32, 8), (32, 16)]
BATCHES = [64, 128, 256]
CACHE = os.environ.get("DBS_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "dbs_autotune.json"))


def workload_key(cams, n: int, m: int) -> str:
    """GPU architecture, HIP runtime and library versions (a new compiler or
    kernel build can move the optimum), splat and lobe counts, resolutions."""
    from . import _lib
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    res = ",".join(f"{c['width']}x{c['height']}" for c in cams)
    lib = _lib.load().dbs_version().decode()
    return f"{arch}|hip {torch.version.hip}|{lib}|{n}|{m}|{res}"


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path: str, cache: dict):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(cams, params, target, cfg: renderer.RasterConfig, steps: int = 3, warmup: int = 1) -> float:
    """Seconds per graph-replayed training step for one launch shape."""
    n = params["means"].shape[0]
    m = params["lobe_betas"].shape[1]
    rast = renderer.Rasterizer(cams, n, m, cfg)
    step = renderer.TrainStep(rast, params, target, headroom=1.1, use_graph=True)
    for _ in range(warmup):
        step.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if step.overflowed():
        dt = float("inf")
    del step, rast
    return dt


def tune(cams, params, target, candidates=None, batches=None, cache_path: str | None = CACHE,
         steps: int = 3, refine: int = 3, log=None) -> renderer.RasterConfig:
    """Fastest RasterConfig for this workload (cached)."""
    n = params["means"].shape[0]
    m = params["lobe_betas"].shape[1]
    key = workload_key(cams, n, m)
    cache = _load_cache(cache_path) if cache_path else {}
    if key in cache:
        e = cache[key]
        return renderer.RasterConfig(tile_w=e["tile_w"], tile_h=e["tile_h"], batch=e["batch"])
    shapes = [(tw, th, b) for tw, th in candidates or CANDIDATES for b in batches or BATCHES]
    tw, th, b = shapes[0]
    time_config(cams, params, target, renderer.RasterConfig(tile_w=tw, tile_h=th, batch=b), steps=4 * steps)
    table = []
    for tw, th, b in shapes:
        t = time_config(cams, params, target, renderer.RasterConfig(tile_w=tw, tile_h=th, batch=b), steps=steps)
        table.append({"tile_w": tw, "tile_h": th, "batch": b, "ms": round(t * 1e3, 4)})
        if log:
            log(f"autotune {tw}x{th} batch {b}: {t * 1e3:.3f} ms")
    # second round over the fastest few: best of two longer runs each
    finalists = sorted(table, key=lambda e: e["ms"])[:refine]
    best, best_t = None, float("inf")
    for rnd in range(2):
        for e in (finalists if rnd == 0 else finalists[::-1]):
            cfg = renderer.RasterConfig(tile_w=e["tile_w"], tile_h=e["tile_h"], batch=e["batch"])
            t = time_config(cams, params, target, cfg, steps=4 * steps)
            e["refined_ms"] = round(min(t * 1e3, e.get("refined_ms", float("inf"))), 4)
            if log:
                log(f"autotune refine {cfg.tile_w}x{cfg.tile_h} batch {cfg.batch}: {t * 1e3:.3f} ms")
            if t < best_t:
                best, best_t = cfg, t
    if cache_path:
        cache[key] = {"tile_w": best.tile_w, "tile_h": best.tile_h, "batch": best.batch,
                      "ms": round(best_t * 1e3, 4), "table": table}
        _save_cache(cache_path, cache)
    return best
