"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
binding and bring results to numpy; compare with the oracle."""
from __future__ import annotations

import numpy as np

AMAX = np.float32(0.99)
TEPS = np.float32(1e-4)
PARAMS = ("means", "scales", "quats", "opacities", "betas", "diffuse",
          "lobe_angles", "lobe_colors", "lobe_betas")


def gpu_render(scene, cams, cfg=None, grads_from=None):
    """Forward (and optionally backward with dL/dimage = grads_from, a list of
    [3,H,W] arrays per view) of the HIP path.  Returns a dict of numpy arrays."""
    import torch
    from paper_2501_18630_amd import renderer
    n = scene["means"].shape[0]
    m = scene["lobe_betas"].shape[1]
    rast = renderer.Rasterizer(cams, n, m, cfg)
    params = renderer.to_device(scene)
    image, T, last = rast.forward(params)
    out = dict(rast=rast, params=params, image_t=image, T_t=T, last_t=last)
    out["images"] = [im.cpu().numpy() for im in rast.split_image(image)]
    out["T"] = [t.cpu().numpy() for t in rast.split_pixels(T)]
    out["last"] = [t.cpu().numpy() for t in rast.split_pixels(last)]
    # last position -> splat id (or -1)
    b = rast.bins_arrays()
    pair_rec = b["pair_rec"].cpu().numpy().astype(np.int64)
    out["last_id"] = []
    for v, lv in enumerate(out["last"]):
        ids = np.full(lv.shape, -1, np.int64)
        ok = lv >= 0
        ids[ok] = pair_rec[lv[ok]] - v * n
        out["last_id"].append(ids)
    if grads_from is not None:
        dl = torch.cat([torch.as_tensor(np.ascontiguousarray(g, np.float32)).reshape(-1) for g in grads_from]).cuda()
        grads = {k: torch.zeros_like(params[k]) for k in PARAMS}
        rast.backward(params, dl, T, last, grads)
        out["grads"] = {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAMS}
    torch.cuda.synchronize()
    return out


def oracle_view(oracle, scene, cam, pixels=None):
    return oracle.render(scene, cam, float(AMAX), float(TEPS), pixels=pixels)


def straddle_mask(ref_T, ref_T_prev, teps=float(TEPS), rel=1e-5):
    """Pixels whose FP64 transmittance is within `rel` of t_eps at the stopping
    step (or just above it at the end): the FP32 path may legitimately stop one
    splat earlier or later there."""
    return (np.abs(ref_T / teps - 1) < rel) | (np.abs(ref_T_prev / teps - 1) < rel)


def assert_image_close(gpu_img_hw3, ref_rgb, ref_T, ref_T_prev, atol=1e-5):
    flag = straddle_mask(ref_T, ref_T_prev)
    err = np.abs(gpu_img_hw3 - ref_rgb).max(axis=1)
    bad = (err > atol) & ~flag
    assert not bad.any(), f"max err {err[~flag].max():.3e} at {np.argmax(np.where(flag, 0, err))}, " \
                          f"{bad.sum()} pixels over {atol}"
    return err.max() if err.size else 0.0


def assert_grads_close(g, g_ref, a_ref, rtol=1e-3, atol_abs=1e-5, names=PARAMS):
    """Per element |g - g_ref| <= rtol |g_ref| + atol_abs * A_ref, where A_ref is
    the oracle's error scale sum_pixels sum_j |J_pj| |s_j| (the FP32 sums of
    screen-space adjoints s_j carry an error proportional to sum |s_j|, which
    the chain J maps to the parameters); plus a per-tensor relative L2 check."""
    for k in names:
        d = np.abs(g[k] - g_ref[k])
        tol = rtol * np.abs(g_ref[k]) + atol_abs * a_ref[k] + 1e-12
        bad = d > tol
        assert not bad.any(), (k, int(bad.sum()), float((d / tol).max()),
                               g[k].reshape(-1)[np.argmax((d / tol).reshape(-1))],
                               g_ref[k].reshape(-1)[np.argmax((d / tol).reshape(-1))])
        nrm = np.linalg.norm(g_ref[k])
        if nrm > 0:
            assert np.linalg.norm(g[k] - g_ref[k]) <= rtol * nrm + 1e-12, k


def hw3(img_3hw):
    return np.transpose(img_3hw, (1, 2, 0)).reshape(-1, 3)
