"""Batched path at the benchmark's sizes and launch configuration (batched,
persistent, 16x16 tiles, batch 256): graph replay equals eager; configs 2, 3
and 4 against the oracle -- every record's pixel box, depth key and tile
count bit-exact against the oracle's FP64 projection, whole-view tile lists
bit-exact against the oracle's binning of its own boxes, sampled pixels and
a 64x64 crop at the far corner of a 1920x1080 view within 1e-5, and
crop-restricted gradients (config 3 through the accumulating reverse call,
config 4 through the gradient store and summed over two views).  Needs an
MI355X."""
import numpy as np
import pytest

from paper_2501_18630_amd import scenes
from gpu_helpers import AMAX, TEPS, PARAMS, assert_grads_close, assert_image_close, hw3

pytestmark = pytest.mark.gpu


def _scene64(s):
    """The scene widened once to FP64 (exact), so that the oracle's per-view
    calls do not convert it again."""
    return {k: np.ascontiguousarray(v, np.float64) for k, v in s.items()}


class Run:
    """One batched forward of a configuration, kept for the tests of the module."""

    def __init__(self, s, cams):
        from gpu_helpers import gpu_render
        self.s, self.cams = s, cams
        self.s64 = _scene64(s)
        self.n = s["means"].shape[0]
        self.out = gpu_render(s, cams)
        self.rast = self.out["rast"]


@pytest.fixture(scope="module")
def c2():
    return Run(*scenes.config2())


@pytest.fixture(scope="module")
def c3():
    return Run(*scenes.config3())


@pytest.fixture(scope="module")
def c4():
    import torch
    torch.cuda.reset_peak_memory_stats()
    r = Run(*scenes.config4())
    print(f"config 4: peak device memory {torch.cuda.max_memory_allocated() / 2**30:.1f} GiB")
    return r


def _pixels(rng, w, h, k):
    return np.stack([rng.integers(0, w, k), rng.integers(0, h, k)], 1).astype(np.int32)


def _touching(p, x0, y0, w, h):
    """Splats whose FP64 pixel box (the oracle's) meets [x0, x0+w) x [y0, y0+h):
    no other splat has r^2 < 1 at any pixel centre of the rectangle."""
    bb = p["bbox"]
    return np.where((p["valid"] == 1) & (bb[:, 0] <= bb[:, 1]) & (bb[:, 2] <= bb[:, 3]) &
                    (bb[:, 0] <= x0 + w - 1) & (bb[:, 1] >= x0) & (bb[:, 2] <= y0 + h - 1) & (bb[:, 3] >= y0))[0]


def test_graph_replay_equals_eager():
    import torch
    from paper_2501_18630_amd import renderer
    s = scenes.uniform_box_scene(3000, [-2, -2, 2], [2, 2, 8], m=2, seed=31)
    cams = [scenes.look_at_camera(p, w, h) for p, (w, h) in
            zip([[0, 0, -9.0], [4.0, 1.0, -7.0], [-3.0, 3.0, -6.0]], [(96, 64), (80, 80), (65, 97)])]
    params = renderer.to_device(s)
    targets = torch.as_tensor(np.random.default_rng(2).uniform(0, 1, 3 * sum(
        c["width"] * c["height"] for c in cams)).astype(np.float32)).cuda()
    eager = renderer.TrainStep(renderer.Rasterizer(cams, 3000, 2), params, targets, use_graph=False)
    eager.run()
    torch.cuda.synchronize()
    ref_img = eager.image.clone()
    ref_g = {k: v.clone() for k, v in eager.grads.items()}
    graph = renderer.TrainStep(renderer.Rasterizer(cams, 3000, 2), params, targets, use_graph=True)
    for rep in range(4):
        graph.run()
        # eager work on the same stream between replays
        scratch = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert not graph.overflowed()
        assert torch.equal(graph.image, ref_img), rep
        for k in PARAMS:
            torch.testing.assert_close(graph.grads[k], ref_g[k], rtol=1e-5, atol=1e-8)
        del scratch


def test_graph_overflow_is_reported():
    import torch
    from paper_2501_18630_amd import renderer
    s = scenes.uniform_box_scene(2000, [-2, -2, 2], [2, 2, 8], m=2, seed=32)
    cams = [scenes.camera(64, 48, f=64.0)]
    params = renderer.to_device(s)
    target = torch.zeros(3 * 64 * 48, device="cuda")
    step = renderer.TrainStep(renderer.Rasterizer(cams, 2000, 2), params, target, headroom=1.0)
    step.run()
    assert not step.overflowed()
    params["scales"].mul_(3.0)  # larger supports -> more pairs than captured capacity
    step.run()
    torch.cuda.synchronize()
    assert step.overflowed()
    assert torch.all(step.final_T == 1.0)


# ---------------------------------------------------------------- per record, every view

def _check_records(oracle, run, views):
    """Box, depth key and tile count of every record of the views, bit-exact
    against the oracle's FP64 projection rounded once."""
    rec = run.rast.records()
    n = run.n
    for v in views:
        p = oracle.project(run.s64, run.cams[v])
        sl = slice(v * n, (v + 1) * n)
        nt = rec["ntiles"][sl].cpu().numpy()
        bb = rec["bbox"][sl].cpu().numpy().astype(np.int32)
        dk = rec["depth"][sl].cpu().numpy().view(np.uint32)
        pb = p["bbox"]
        valid = p["valid"] == 1
        live = valid & (pb[:, 0] <= pb[:, 1]) & (pb[:, 2] <= pb[:, 3])
        assert live.sum() > 1000, v
        np.testing.assert_array_equal(nt > 0, live, err_msg=f"view {v}: visibility")
        np.testing.assert_array_equal(bb[live], pb[live], err_msg=f"view {v}: pixel boxes")
        np.testing.assert_array_equal(dk[valid], p["depth_key"][valid], err_msg=f"view {v}: depth keys")
        ref_nt = (pb[:, 1] // 16 - pb[:, 0] // 16 + 1) * (pb[:, 3] // 16 - pb[:, 2] // 16 + 1)
        np.testing.assert_array_equal(nt[live], ref_nt[live], err_msg=f"view {v}: tile counts")


def test_records_bit_exact_config2(oracle, c2):
    _check_records(oracle, c2, range(len(c2.cams)))


def test_records_bit_exact_config3(oracle, c3):
    _check_records(oracle, c3, range(len(c3.cams)))


@pytest.mark.parametrize("half", [0, 1])
def test_records_bit_exact_config4(oracle, c4, half):
    _check_records(oracle, c4, range(16 * half, 16 * half + 16))


# ---------------------------------------------------------------- whole-view tile lists

def _check_view_bins(oracle, run, v):
    """Every tile list of view v against the oracle's binning of its own FP64
    boxes and depth keys (end to end), vectorised over the view's pairs."""
    n = run.n
    cam = run.cams[v]
    b = run.rast.bins_arrays()
    toff = run.rast.tile_offsets()
    p = oracle.project(run.s64, cam)
    start, ids = oracle.bin_pairs(p["valid"], p["bbox"], p["depth_key"], cam["width"], cam["height"], 16, 16)
    nt = start.size - 1
    assert nt == int(toff[v + 1] - toff[v]) and ids.size > 10000
    rng = b["tile_range"][int(toff[v]):int(toff[v]) + nt].cpu().numpy().astype(np.int64)
    nonempty = start[1:] > start[:-1]
    np.testing.assert_array_equal(rng[:, 1] > rng[:, 0], nonempty, err_msg=f"view {v}: non-empty tiles")
    off = int(rng[nonempty, 0].min())
    np.testing.assert_array_equal(rng[nonempty, 0] - off, start[:-1][nonempty], err_msg=f"view {v}: starts")
    np.testing.assert_array_equal(rng[nonempty, 1] - off, start[1:][nonempty], err_msg=f"view {v}: ends")
    got = b["pair_rec"][off:off + ids.size].cpu().numpy().astype(np.int64) - v * n
    np.testing.assert_array_equal(got, ids, err_msg=f"view {v}: pair lists")


@pytest.mark.parametrize("cfg_views", [(2, (0,)), (3, (0, 7, 15)), (4, (0, 16, 31))], ids=["c2", "c3", "c4"])
def test_view_bins_bit_exact_end_to_end(oracle, request, cfg_views):
    which, views = cfg_views
    run = request.getfixturevalue(f"c{which}")
    for v in views:
        _check_view_bins(oracle, run, v)


# ---------------------------------------------------------------- images

@pytest.mark.parametrize("which", [2, 3, 4])
def test_fullsize_sampled_pixels(oracle, request, which):
    """Sampled pixels of the full-size forward against the oracle (brute force
    over every splat)."""
    run = request.getfixturevalue(f"c{which}")
    views = {2: [0], 3: [0, 7, 15], 4: [0, 16, 31]}[which]
    rng = np.random.default_rng(11 + which)
    for v in views:
        cam = run.cams[v]
        pix = _pixels(rng, cam["width"], cam["height"], 48 if which < 4 else 32)
        ref = oracle.render(run.s64, cam, float(AMAX), float(TEPS), pixels=pix)
        gpu = run.out["images"][v][:, pix[:, 1], pix[:, 0]].T
        assert_image_close(gpu, ref["rgb"], ref["T"], ref["T_prev"])


@pytest.mark.parametrize("which", [3, 4])
def test_far_corner_crop(oracle, request, which):
    """The bottom-right 64x64 corner of the first 1920x1080 view: pixels whose
    centres lie furthest from the principal point, where screen coordinates
    are largest, against the oracle over every splat that reaches the crop."""
    run = request.getfixturevalue(f"c{which}")
    v = next(i for i, c in enumerate(run.cams) if (c["width"], c["height"]) == (1920, 1080))
    cam = run.cams[v]
    x0, y0, w = 1920 - 64, 1080 - 64, 64
    p = oracle.project(run.s64, cam)
    near = _touching(p, x0, y0, w, w)
    assert near.size > 50
    ref = oracle.render(scenes.subset(run.s64, near), cam, float(AMAX), float(TEPS),
                        pixels=oracle.crop_pixels(x0, y0, w, w))
    assert np.count_nonzero(ref["T"] < 0.5) > 100
    gpu = hw3(run.out["images"][v][:, y0:y0 + w, x0:x0 + w])
    err = assert_image_close(gpu, ref["rgb"], ref["T"], ref["T_prev"])
    print(f"config {which} view {v} far-corner crop: max image error {err:.2e}")


def test_fullsize_sampled_tiles_bit_exact(oracle, c3):
    """Sampled tiles against the oracle's binning of the GPU's own boxes."""
    s, cams, n, rast = c3.s, c3.cams, c3.n, c3.rast
    rec = {k: v.cpu().numpy() for k, v in rast.records().items()}
    b = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in rast.bins_arrays().items()}
    toff = rast.tile_offsets()
    rng = np.random.default_rng(12)
    for v in (0, 5, 15):
        cam = cams[v]
        sl = slice(v * n, (v + 1) * n)
        nt = int(toff[v + 1] - toff[v])
        tiles = rng.integers(0, nt, 6)
        st, ids = oracle.bin_tiles((rec["ntiles"][sl] > 0).astype(np.int32), rec["bbox"][sl].astype(np.int32),
                                   rec["depth"][sl].view(np.uint32), cam["width"], 16, 16, tiles)
        for r, t in enumerate(tiles):
            lo, hi = b["tile_range"][toff[v] + t]
            got = b["pair_rec"][lo:hi].astype(np.int64) - v * n
            np.testing.assert_array_equal(got, ids[st[r]:st[r + 1]])


# ---------------------------------------------------------------- gradients

def _crop_grads(oracle, run, crops, dls):
    """Oracle gradient of sum_views <dL_v, image_v> with dL_v non-zero only on
    the crops [(view, x0, y0, w)]: per crop over the splats that reach it,
    summed over the crops.  Returns (near ids, grads, error scale, contribution
    scale) for the union of those splats."""
    parts = []
    for v, x0, y0, w in crops:
        cam = run.cams[v]
        p = oracle.project(run.s64, cam)
        near = _touching(p, x0, y0, w, w)
        assert near.size > 50
        g, a, c = oracle.render_bwd(scenes.subset(run.s64, near), cam, float(AMAX), float(TEPS),
                                    hw3(dls[v][:, y0:y0 + w, x0:x0 + w]),
                                    pixels=oracle.crop_pixels(x0, y0, w, w), want_abs=True, want_contrib=True)
        parts.append((near, g, a, c))
    union = np.unique(np.concatenate([pp[0] for pp in parts]))
    pos = {int(i): k for k, i in enumerate(union)}
    G, A, Cs = ({k: np.zeros((union.size,) + np.asarray(run.s[k]).shape[1:]) for k in PARAMS} for _ in range(3))
    for near, g, a, c in parts:
        idx = np.array([pos[int(i)] for i in near])
        for k in PARAMS:
            np.add.at(G[k], idx, g[k])
            np.add.at(A[k], idx, a[k])
            np.add.at(Cs[k], idx, c[k])
    return union, G, A, Cs


def _report_scales(tag, g, g_ref, a_ref, c_ref):
    """Worst |g - g_ref| / tol under the error scale the tests use and under
    the per-pixel contribution scale, printed for the record."""
    w_a = w_c = 0.0
    for k in PARAMS:
        d = np.abs(g[k] - g_ref[k])
        w_a = max(w_a, float((d / (1e-3 * np.abs(g_ref[k]) + 1e-5 * a_ref[k] + 1e-12)).max()))
        w_c = max(w_c, float((d / (1e-3 * np.abs(g_ref[k]) + 1e-5 * c_ref[k] + 1e-12)).max()))
    print(f"{tag}: worst |dg|/tol = {w_a:.3f} (error scale), {w_c:.3f} (contribution scale)")


def test_fullsize_crop_gradient_batched(oracle, c3):
    """Batched backward over all 16 views (accumulating call) with dL/dimage
    non-zero only on a 48x48 crop of one view: the gradient of every splat
    matches the oracle on that crop (splats that cannot reach it get exactly
    zero)."""
    import torch
    run = c3
    v0, x0, y0, w = 3, 300, 200, 48
    dls = [np.zeros((3, c["height"], c["width"]), np.float32) for c in run.cams]
    dls[v0][:, y0:y0 + w, x0:x0 + w] = np.random.default_rng(13).standard_normal((3, w, w))
    out, rast = run.out, run.rast
    dl = torch.cat([torch.as_tensor(d).reshape(-1) for d in dls]).cuda()
    grads = {k: torch.zeros_like(out["params"][k]) for k in PARAMS}
    rast.backward(out["params"], dl, out["T_t"], out["last_t"], grads)
    g = {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAMS}
    near, g_ref, a_ref, c_ref = _crop_grads(oracle, run, [(v0, x0, y0, w)], dls)
    mine = {k: g[k][near] for k in PARAMS}
    _report_scales("config 3 crop gradient", mine, g_ref, a_ref, c_ref)
    assert_grads_close(mine, g_ref, a_ref)
    far = np.setdiff1d(np.arange(run.n), near)
    for k in PARAMS:
        assert not np.any(g[k][far]), k


def test_config2_crop_gradient(oracle, c2):
    """Config 2 (one 1600x1064 view, 1.5 M clustered splats): dL/dimage
    non-zero on a 48x48 crop at the image centre, where the clusters overlap
    most; every splat that reaches the crop matches the oracle, every other
    one gets exactly zero."""
    import torch
    run = c2
    cam = run.cams[0]
    x0, y0, w = cam["width"] // 2 - 24, cam["height"] // 2 - 24, 48
    dls = [np.zeros((3, cam["height"], cam["width"]), np.float32)]
    dls[0][:, y0:y0 + w, x0:x0 + w] = np.random.default_rng(29).standard_normal((3, w, w))
    out, rast = run.out, run.rast
    dl = torch.as_tensor(dls[0]).reshape(-1).cuda()
    grads = {k: torch.zeros_like(out["params"][k]) for k in PARAMS}
    rast.backward(out["params"], dl, out["T_t"], out["last_t"], grads)
    g = {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAMS}
    near, g_ref, a_ref, c_ref = _crop_grads(oracle, run, [(0, x0, y0, w)], dls)
    assert near.size > 100
    mine = {k: g[k][near] for k in PARAMS}
    _report_scales("config 2 crop gradient", mine, g_ref, a_ref, c_ref)
    assert_grads_close(mine, g_ref, a_ref)
    far = np.setdiff1d(np.arange(run.n), near)
    for k in PARAMS:
        assert not np.any(g[k][far]), k


def test_config4_crop_gradient_store(oracle, c4):
    """Config 4's training-step reverse pass: the gradient store over all 32
    views, with dL/dimage non-zero on 48x48 crops of two views, so that a
    splat reaching both crops sums its two views' gradients.  Every element is
    written (buffers filled with NaN beforehand); splats reaching a crop match
    the oracle's gradient summed over the crops, every other splat gets
    exactly zero."""
    import torch
    run = c4
    big = [i for i, c in enumerate(run.cams) if c["width"] >= 1280]
    va, vb = big[0], big[-1]
    rng = np.random.default_rng(41)
    crops = []
    for v in (va, vb):
        cam = run.cams[v]
        crops.append((v, int(rng.integers(cam["width"] // 4, cam["width"] // 2)),
                      int(rng.integers(cam["height"] // 4, cam["height"] // 2)), 48))
    dls = [np.zeros((3, c["height"], c["width"]), np.float32) for c in run.cams]
    for v, x0, y0, w in crops:
        dls[v][:, y0:y0 + w, x0:x0 + w] = rng.standard_normal((3, w, w))
    out, rast = run.out, run.rast
    dl = torch.cat([torch.as_tensor(d).reshape(-1) for d in dls]).cuda()
    grads = {k: torch.full_like(out["params"][k], float("nan")) for k in PARAMS}
    rast.backward(out["params"], dl, out["T_t"], out["last_t"], grads, store=True)
    g = {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAMS}
    for k in PARAMS:
        assert np.all(np.isfinite(g[k])), k
    near, g_ref, a_ref, c_ref = _crop_grads(oracle, run, crops, dls)
    assert near.size > 200
    mine = {k: g[k][near] for k in PARAMS}
    _report_scales("config 4 two-view crop gradient (store)", mine, g_ref, a_ref, c_ref)
    assert_grads_close(mine, g_ref, a_ref)
    far = np.setdiff1d(np.arange(run.n), near)
    for k in PARAMS:
        assert not np.any(g[k][far]), k


def test_fullsize_gaussian_sh_sampled_pixels(oracle, c3):
    """The Gaussian + SH comparison mode at config 3's size, as the benchmark
    runs it (same scales: 3-sigma supports, ~340 M pairs); sampled pixels of
    two views against the oracle's comparison mode."""
    from gpu_helpers import gpu_render
    from paper_2501_18630_amd import renderer
    s, cams = c3.s, c3.cams
    g = scenes.gaussian_sh(s, seed=7, scale_factor=1.0)
    out = gpu_render(g, cams, renderer.RasterConfig(kernel="gaussian_sh"))
    rng = np.random.default_rng(13)
    for v in (0, 15):
        cam = cams[v]
        pix = _pixels(rng, cam["width"], cam["height"], 32)
        ref = oracle.render(g, cam, float(AMAX), float(TEPS), pixels=pix)
        gpu = out["images"][v][:, pix[:, 1], pix[:, 0]].T
        assert_image_close(gpu, ref["rgb"], ref["T"], ref["T_prev"])
