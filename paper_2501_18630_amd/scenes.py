"""Seeded synthetic scenes and cameras shaped like the paper's workloads.

This module only draws inputs.  It holds none of the rasterizer's
arithmetic, so both the HIP path and the CPU oracle can consume what it
produces.  Everything is numpy ``default_rng`` (PCG64) with fixed seeds:
splats seed 0, target image seed 1, camera rig seed 2, resolution draws
seed 3.

A scene is a dict of float32 arrays following the primitive of Sec. 3.2,
Eq. (4) and the Spherical Beta features of Sec. 3.3, Eq. (8):

    means [N,3]  scales [N,3] (activated)  quats [N,4] (w,x,y,z)
    opacities [N] (activated)  betas [N] (raw b)  diffuse [N,3] (c0)
    lobe_angles [N,M,2] (theta, phi)  lobe_colors [N,M,3]  lobe_betas [N,M] (raw)

A camera is a dict: viewmat [3,4] (world->camera [R|t], OpenCV axes),
fx, fy, cx, cy, width, height, near, background [3].

The paper's workloads (Mip-NeRF 360 scenes, Sec. 4) are not available; the
distributions below stand in for them with the primitive counts (1.5 M to
6 M), lobe counts (2 or 4) and opacity spread the paper reports.
"""
from __future__ import annotations

import numpy as np

RESOLUTIONS = ((640, 480), (1024, 768), (1280, 720), (1600, 1064), (1920, 1080))


def _unit_rows(rng: np.random.Generator, n: int, d: int) -> np.ndarray:
    v = rng.standard_normal((n, d))
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    bad = nrm[:, 0] < 1e-12
    while bad.any():  # redraw degenerate directions (probability ~0)
        v[bad] = rng.standard_normal((int(bad.sum()), d))
        nrm = np.linalg.norm(v, axis=1, keepdims=True)
        bad = nrm[:, 0] < 1e-12
    return v / nrm


def _sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def _lobes(rng: np.random.Generator, n: int, m: int, b_std: float):
    d = _unit_rows(rng, n * m, 3).reshape(n, m, 3)
    theta = np.arccos(np.clip(d[..., 2], -1.0, 1.0))
    phi = np.arctan2(d[..., 1], d[..., 0])
    angles = np.stack([theta, phi], axis=-1)
    colors = rng.uniform(0.0, 0.5, size=(n, m, 3))
    betas = rng.normal(0.0, b_std, size=(n, m))
    return angles, colors, betas


def _pack(means, scales, quats, opac, betas, diffuse, angles, lcol, lb) -> dict:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(means=f(means), scales=f(scales), quats=f(quats), opacities=f(opac),
                betas=f(betas), diffuse=f(diffuse), lobe_angles=f(angles),
                lobe_colors=f(lcol), lobe_betas=f(lb))


def uniform_box_scene(n: int, lo, hi, m: int = 2, seed: int = 0,
                      log_scale=(np.log(0.02), np.log(0.2)), opacity_std: float = 1.0,
                      b_std: float = 0.5, lobe_b_std: float = 0.5) -> dict:
    """Splats with centres uniform in the box [lo, hi] (configs 0 and 1)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), size=(n, 3))
    scales = np.exp(rng.uniform(log_scale[0], log_scale[1], size=(n, 3)))
    quats = _unit_rows(rng, n, 4)
    opac = _sigmoid(rng.normal(0.0, opacity_std, size=n))
    betas = rng.normal(0.0, b_std, size=n)
    diffuse = rng.uniform(0.0, 1.0, size=(n, 3))
    angles, lcol, lb = _lobes(rng, n, m, lobe_b_std)
    return _pack(means, scales, quats, opac, betas, diffuse, angles, lcol, lb)


def cluster_scene(n: int, m: int = 4, seed: int = 0, n_clusters: int = 64) -> dict:
    """Splats drawn from a mixture of anisotropic Gaussian clusters in
    [-10,10]^3 (configs 2-4): centres U[-8,8]^3, random orthonormal axes,
    per-axis std exp(U[ln .2, ln 2]), equal weights; samples outside the box
    are redrawn.  Scales exp(U[ln .005, ln .3]), opacity sigmoid(N(0,1.5)),
    b ~ N(0, 0.7), lobes as in config 0."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-8.0, 8.0, size=(n_clusters, 3))
    axes = np.empty((n_clusters, 3, 3))
    for c in range(n_clusters):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        axes[c] = q * np.sign(np.diag(r))[None, :]
    sig = np.exp(rng.uniform(np.log(0.2), np.log(2.0), size=(n_clusters, 3)))
    means = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        cid = rng.integers(0, n_clusters, size=todo.size)
        z = rng.standard_normal((todo.size, 3)) * sig[cid]
        p = centres[cid] + np.einsum("nij,nj->ni", axes[cid], z)
        ok = np.all(np.abs(p) <= 10.0, axis=1)
        means[todo[ok]] = p[ok]
        todo = todo[~ok]
    scales = np.exp(rng.uniform(np.log(0.005), np.log(0.3), size=(n, 3)))
    quats = _unit_rows(rng, n, 4)
    opac = _sigmoid(rng.normal(0.0, 1.5, size=n))
    betas = rng.normal(0.0, 0.7, size=n)
    diffuse = rng.uniform(0.0, 1.0, size=(n, 3))
    angles, lcol, lb = _lobes(rng, n, m, 0.5)
    return _pack(means, scales, quats, opac, betas, diffuse, angles, lcol, lb)


def camera(width: int, height: int, f: float | None = None, R=None, t=None,
           near: float = 0.2, background=(0.0, 0.0, 0.0)) -> dict:
    """Pinhole camera; principal point at the image centre, f = width by default."""
    R = np.eye(3) if R is None else np.asarray(R, np.float64)
    t = np.zeros(3) if t is None else np.asarray(t, np.float64)
    f = float(width) if f is None else float(f)
    vm = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    return dict(viewmat=vm, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0, width=int(width),
                height=int(height), near=float(near),
                background=np.asarray(background, np.float32).reshape(3))


def look_at_camera(position, width: int, height: int, **kw) -> dict:
    """Camera at `position` looking at the origin: forward = -p/|p|,
    right = forward x y (z if nearly parallel), down = forward x right."""
    p = np.asarray(position, np.float64)
    fwd = -p / np.linalg.norm(p)
    up = np.array([0.0, 1.0, 0.0])
    if abs(fwd @ up) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    return camera(width, height, R=R, t=-R @ p, **kw)


def sphere_rig(n_views: int, radius: float = 15.0, seed: int = 2, res_seed: int = 3):
    """Cameras on a sphere looking at the origin with resolutions drawn from
    {640x480, 1024x768, 1280x720, 1600x1064, 1920x1080}."""
    rng = np.random.default_rng(seed)
    pos = _unit_rows(rng, n_views, 3) * radius
    rr = np.random.default_rng(res_seed)
    pick = rr.integers(0, len(RESOLUTIONS), size=n_views)
    return [look_at_camera(pos[v], *RESOLUTIONS[pick[v]]) for v in range(n_views)]


def target_image(height: int, width: int, seed: int = 1) -> np.ndarray:
    """Seeded U[0,1] target, planar [3, H, W]."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


# --------------------------------------------------------------------------
# the five workloads

def config0():
    """1 view 64x64, f=64, 256 splats in [-1,1]^2 x [2,6], 2 lobes."""
    return uniform_box_scene(256, [-1, -1, 2], [1, 1, 6], m=2, seed=0), [camera(64, 64, f=64.0)]


def config1():
    """1 view 1024x768, f=1024, 100k splats in [-4,4]^2 x [2,12], 2 lobes."""
    return (uniform_box_scene(100_000, [-4, -4, 2], [4, 4, 12], m=2, seed=0),
            [camera(1024, 768, f=1024.0)])


def config2(n: int = 1_500_000):
    """1 view 1600x1064, camera at (0,0,-15) looking down +z, 1.5M clustered splats, 4 lobes."""
    return cluster_scene(n, m=4, seed=0), [camera(1600, 1064, t=[0.0, 0.0, 15.0])]


def config3(n: int = 3_000_000, n_views: int = 16):
    """16 mixed-resolution views on a radius-15 sphere, 3M clustered splats, 4 lobes."""
    return cluster_scene(n, m=4, seed=0), sphere_rig(n_views)


def config4(n: int = 6_000_000, n_views: int = 32):
    """32 mixed-resolution views, 6M clustered splats, 4 lobes."""
    return cluster_scene(n, m=4, seed=0), sphere_rig(n_views)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}


def gaussian_sh(scene: dict, seed: int = 7, scale_factor: float = 1.0) -> dict:
    """The scene as input of the Gaussian-kernel + SH comparison mode: the same
    centres, rotations and opacities, scales times `scale_factor` (1/3 puts
    the 3-sigma ellipse on the Beta kernel's support), and degree-3 SH
    coefficients [n, 16, 3]: DC ~ N(0, 0.6), higher orders ~ N(0, 0.15)."""
    rng = np.random.default_rng(seed)
    n = scene["means"].shape[0]
    sh = rng.normal(0.0, 0.15, size=(n, 16, 3))
    sh[:, 0, :] = rng.normal(0.0, 0.6, size=(n, 3))
    out = dict(scene)
    out["scales"] = np.ascontiguousarray(scene["scales"] * np.float32(scale_factor), dtype=np.float32)
    out["sh"] = np.ascontiguousarray(sh, dtype=np.float32)
    return out


def subset(scene: dict, idx) -> dict:
    """Rows `idx` of every array of a scene."""
    return {k: np.ascontiguousarray(v[idx]) for k, v in scene.items()}
