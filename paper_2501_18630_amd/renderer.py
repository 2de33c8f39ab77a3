"""Rasterizer front end over the C ABI of libdbs.

PyTorch provides device memory and streams; every step of the path runs in
the library's HIP kernels.

    rast = Rasterizer(cameras, n_splats, n_lobes)
    image, T, last = rast.forward(params)            # eager, sizes bins exactly
    rast.backward(params, dL_dimage, T, last, grads) # grads accumulate (+=)

`render(params, rast)` wraps the two in a torch.autograd.Function.
`TrainStep` captures preprocess -> bin/sort -> forward -> L1 loss -> backward
for a fixed scene size in one HIP graph (the batched multi-view step).

Parameters are a dict of contiguous float32 CUDA tensors (names as in
`_lib.PARAMS`); cameras are the dicts of `scenes.camera`.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import PARAMS, check


@dataclass
class RasterConfig:
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 256
    t_eps: float = 1e-4
    alpha_max: float = 0.99
    persistent: bool = True
    # decomposition render modes (forward only): "diffuse" / "specular" colour,
    # and primitives with b below / at-or-above b_split
    color: str = "full"
    b_range: str = "all"
    b_split: float = 0.0
    # "beta" (the method) or "gaussian_sh": the comparison mode with a
    # Gaussian kernel and degree-3 SH colour (forward only; params["sh"])
    kernel: str = "beta"

    def to_c(self) -> _lib.RasterCfg:
        flags = _lib.FLAG_PERSISTENT if self.persistent else 0
        flags |= {"full": 0, "diffuse": _lib.FLAG_DIFFUSE_ONLY, "specular": _lib.FLAG_SPECULAR_ONLY}[self.color]
        flags |= {"all": 0, "below": _lib.FLAG_B_BELOW, "above": _lib.FLAG_B_ABOVE}[self.b_range]
        flags |= {"beta": 0, "gaussian_sh": _lib.FLAG_GAUSSIAN_SH}[self.kernel]
        return _lib.RasterCfg(self.tile_w, self.tile_h, self.batch, self.t_eps, self.alpha_max, flags, self.b_split)


def make_cameras(cams) -> C.Array:
    arr = (_lib.Camera * len(cams))()
    for k, c in enumerate(cams):
        vm = np.asarray(c["viewmat"], np.float32).reshape(12)
        bg = np.asarray(c.get("background", (0, 0, 0)), np.float32).reshape(3)
        arr[k] = _lib.Camera((C.c_float * 12)(*vm), c["fx"], c["fy"], c["cx"], c["cy"], int(c["width"]),
                             int(c["height"]), c["near"], (C.c_float * 3)(*bg))
    return arr


def to_device(scene: dict, device="cuda") -> dict:
    """numpy scene -> dict of contiguous float32 tensors on `device`."""
    keys = PARAMS + (("sh",) if "sh" in scene else ())
    return {k: torch.as_tensor(np.ascontiguousarray(scene[k], np.float32), device=device).contiguous()
            for k in keys}


def _splats_c(params: dict, n: int, m: int) -> _lib.Splats:
    ptrs = []
    for k in PARAMS:
        t = params[k]
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
        ptrs.append(t.data_ptr() if t.numel() > 0 else None)
    return _lib.Splats(*ptrs, n, m)


def _grads_c(grads: dict) -> _lib.Grads:
    return _lib.Grads(*[grads[k].data_ptr() if grads[k].numel() > 0 else None for k in PARAMS])


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Rasterizer:
    """Buffers and calls for one set of views over a scene of n splats with m
    lobes.  One forward/backward pair at a time: forward() leaves the state
    backward() consumes."""

    def __init__(self, cams, n: int, m: int, cfg: RasterConfig | None = None, device="cuda",
                 pair_capacity: int = 0, headroom: float = 1.0):
        self.lib = _lib.load()
        self.cams = list(cams)
        self.cams_c = make_cameras(self.cams)
        self.V = len(self.cams)
        self.n, self.m = int(n), int(m)
        self.cfg = cfg or RasterConfig()
        self.cfg_c = self.cfg.to_c()
        # the same configuration with the gradient store flag (reverse calls that overwrite)
        self.cfg_store_c = self.cfg.to_c()
        self.cfg_store_c.flags |= _lib.FLAG_GRAD_STORE
        self.device = torch.device(device)
        self.headroom = headroom
        self.sizes = [(int(c["height"]), int(c["width"])) for c in self.cams]
        self.pix_off = np.concatenate([[0], np.cumsum([h * w for h, w in self.sizes])]).astype(np.int64)
        self.n_pixels = int(self.pix_off[-1])
        pb = self.lib.dbs_projected_bytes(self.n, self.V)
        if pb == 0:
            raise ValueError("invalid splat or view count")
        # zero-filled once: the reverse pass's accumulator lives in it
        self.projected = torch.zeros(pb, dtype=torch.uint8, device=self.device)
        self.counts = torch.zeros(2, dtype=torch.int64, device=self.device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.capacity = -1
        self.bins = None
        self.workspace = None
        self.ensure_capacity(pair_capacity)

    # ---- buffers ----
    def ensure_capacity(self, pairs: int):
        if pairs <= self.capacity:
            return
        cap = int(pairs)
        bb = self.lib.dbs_bins_bytes(cap, self.cams_c, self.V, C.byref(self.cfg_c))
        wb = self.lib.dbs_workspace_bytes(self.n, self.V, cap, self.cams_c, C.byref(self.cfg_c))
        if bb == 0 or wb == 0:
            raise ValueError("invalid camera or raster configuration")
        self.bins = None
        self.workspace = None
        self.bins = torch.empty(bb, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.capacity = cap

    def new_outputs(self):
        image = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=self.device)
        final_T = torch.empty(self.n_pixels, dtype=torch.float32, device=self.device)
        last = torch.empty(self.n_pixels, dtype=torch.int32, device=self.device)
        return image, final_T, last

    # ---- the four calls ----
    def preprocess(self, params: dict):
        sp = _splats_c(params, self.n, self.m)
        if self.cfg.kernel == "gaussian_sh":
            sh = params["sh"]
            if sh.dtype != torch.float32 or not sh.is_contiguous() or not sh.is_cuda or sh.numel() != 48 * self.n:
                raise ValueError("sh must be a contiguous float32 CUDA tensor of shape [n, 16, 3]")
            check("dbs_preprocess_gaussian_sh", self.lib.dbs_preprocess_gaussian_sh(
                C.byref(sp), C.c_void_p(sh.data_ptr()), self.cams_c, self.V, C.byref(self.cfg_c),
                C.c_void_p(self.projected.data_ptr()), self.projected.numel(),
                C.c_void_p(self.counts.data_ptr()), _stream()))
            return
        check("dbs_preprocess", self.lib.dbs_preprocess(
            C.byref(sp), self.cams_c, self.V, C.byref(self.cfg_c), C.c_void_p(self.projected.data_ptr()),
            self.projected.numel(), C.c_void_p(self.counts.data_ptr()), _stream()))

    def bin_sort(self):
        check("dbs_bin_sort", self.lib.dbs_bin_sort(
            C.c_void_p(self.projected.data_ptr()), self.cams_c, self.V, C.byref(self.cfg_c), self.n,
            self.capacity, C.c_void_p(self.bins.data_ptr()), self.bins.numel(),
            C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
            C.c_void_p(self.overflow.data_ptr()), _stream()))

    def render_fwd(self, image, final_T, last):
        check("dbs_render_fwd", self.lib.dbs_render_fwd(
            C.c_void_p(self.projected.data_ptr()), C.c_void_p(self.bins.data_ptr()), self.cams_c, self.V,
            C.byref(self.cfg_c), self.n, C.c_void_p(image.data_ptr()), C.c_void_p(final_T.data_ptr()),
            C.c_void_p(last.data_ptr()), _stream()))

    def render_bwd(self, params: dict, dL_dimage, final_T, last, grads: dict, store: bool = False):
        """Gradients added into `grads`, or written over them with store=True."""
        sp = _splats_c(params, self.n, self.m)
        gr = _grads_c(grads)
        cfg = self.cfg_store_c if store else self.cfg_c
        check("dbs_render_bwd", self.lib.dbs_render_bwd(
            C.byref(sp), C.c_void_p(self.projected.data_ptr()), C.c_void_p(self.bins.data_ptr()),
            self.cams_c, self.V, C.byref(cfg), C.c_void_p(final_T.data_ptr()),
            C.c_void_p(last.data_ptr()), C.c_void_p(dL_dimage.data_ptr()), C.byref(gr), _stream()))

    def raster_bwd(self, dL_dimage, final_T, last, atomics=None):
        """Raster reverse pass into the accumulator; with `atomics` (a device
        int64 tensor) the counting build runs and adds the number of global
        float atomics it issued."""
        if atomics is None:
            check("dbs_raster_bwd", self.lib.dbs_raster_bwd(
                C.c_void_p(self.projected.data_ptr()), C.c_void_p(self.bins.data_ptr()), self.cams_c, self.V,
                C.byref(self.cfg_c), self.n, C.c_void_p(final_T.data_ptr()), C.c_void_p(last.data_ptr()),
                C.c_void_p(dL_dimage.data_ptr()), _stream()))
        else:
            check("dbs_raster_bwd_count", self.lib.dbs_raster_bwd_count(
                C.c_void_p(self.projected.data_ptr()), C.c_void_p(self.bins.data_ptr()), self.cams_c, self.V,
                C.byref(self.cfg_c), self.n, C.c_void_p(final_T.data_ptr()), C.c_void_p(last.data_ptr()),
                C.c_void_p(dL_dimage.data_ptr()), C.c_void_p(atomics.data_ptr()), _stream()))

    def project_bwd(self, params: dict, grads: dict, store: bool = False):
        sp = _splats_c(params, self.n, self.m)
        gr = _grads_c(grads)
        cfg = self.cfg_store_c if store else self.cfg_c
        check("dbs_project_bwd", self.lib.dbs_project_bwd(
            C.byref(sp), C.c_void_p(self.projected.data_ptr()), self.cams_c, self.V, C.byref(cfg),
            C.byref(gr), _stream()))

    def stats(self, final_T, last) -> dict:
        """Evaluated / contributing (pixel, pair) counts of the last forward."""
        out = torch.zeros(5, dtype=torch.int64, device=self.device)
        check("dbs_render_stats", self.lib.dbs_render_stats(
            C.c_void_p(self.projected.data_ptr()), C.c_void_p(self.bins.data_ptr()), self.cams_c, self.V,
            C.byref(self.cfg_c), self.n, C.c_void_p(final_T.data_ptr()), C.c_void_p(last.data_ptr()),
            C.c_void_p(out.data_ptr()), _stream()))
        o = out.cpu().tolist()
        return {"bwd_evaluated": o[0], "contributing": o[1], "fwd_evaluated": o[2],
                "bwd_wave_steps": o[3], "bwd_wave_steps_active": o[4]}

    # ---- eager helpers ----
    def forward(self, params: dict, outputs=None):
        """preprocess, size the bins from the exact pair count (one host sync),
        bin/sort, composite.  Returns (image [3*sum HW], final_T, last_index)."""
        self.preprocess(params)
        k = int(self.counts[1].item())
        self.ensure_capacity(int(k * self.headroom) if self.headroom > 1 else k)
        self.bin_sort()
        image, final_T, last = outputs or self.new_outputs()
        self.render_fwd(image, final_T, last)
        return image, final_T, last

    def backward(self, params: dict, dL_dimage, final_T, last, grads: dict, store: bool = False):
        self.render_bwd(params, dL_dimage.contiguous(), final_T, last, grads, store=store)
        return grads

    def l1_loss(self, image, target, scale: float, dL_dimage, loss=None):
        check("dbs_l1_loss", self.lib.dbs_l1_loss(
            C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()), image.numel(), float(scale),
            C.c_void_p(dL_dimage.data_ptr()), C.c_void_p(loss.data_ptr()) if loss is not None else None,
            _stream()))

    def photometric_loss(self, image, target, lambda_ssim: float, dL_dimage, loss=None):
        """(1 - lambda) L1 + lambda (1 - SSIM), summed over views (Sec. 3.4);
        dL_dimage and loss are overwritten."""
        check("dbs_photometric_loss", self.lib.dbs_photometric_loss(
            C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()), self.cams_c, self.V,
            float(lambda_ssim), C.c_void_p(dL_dimage.data_ptr()),
            C.c_void_p(loss.data_ptr()) if loss is not None else None, _stream()))

    def regularizer(self, params: dict, lambda_o: float, lambda_s: float, grads: dict, loss=None):
        """lambda_o sum|o| + lambda_s sum|s| (Sec. 3.4): gradients added, loss incremented."""
        sp = _splats_c(params, self.n, self.m)
        gr = _grads_c(grads)
        check("dbs_regularizer", self.lib.dbs_regularizer(
            C.byref(sp), float(lambda_o), float(lambda_s), C.byref(gr),
            C.c_void_p(loss.data_ptr()) if loss is not None else None, _stream()))

    # ---- views of the flat buffers ----
    def split_image(self, image):
        """flat planar image -> list of [3, H, W] views."""
        return [image[3 * int(self.pix_off[v]):3 * int(self.pix_off[v + 1])].view(3, h, w)
                for v, (h, w) in enumerate(self.sizes)]

    def split_pixels(self, flat):
        """flat per-pixel buffer -> list of [H, W] views."""
        return [flat[int(self.pix_off[v]):int(self.pix_off[v + 1])].view(h, w)
                for v, (h, w) in enumerate(self.sizes)]

    # ---- introspection ----
    def records(self) -> dict:
        """Per-record arrays (record r = v n + i) viewed from `projected`."""
        ptrs = [C.c_void_p() for _ in range(5)]
        check("dbs_projected_layout", self.lib.dbs_projected_layout(
            C.c_void_p(self.projected.data_ptr()), self.n, self.V, *[C.byref(p) for p in ptrs]))
        base = self.projected.data_ptr()
        R = self.n * self.V

        def sl(p, nbytes):
            off = (p.value or base) - base
            return self.projected[off:off + nbytes]

        rec = sl(ptrs[0], 64 * R)
        f64 = rec.view(torch.float64).view(R, 8)
        f32 = rec.view(torch.float32).view(R, 16)
        return dict(centre=f64[:, 0:2], conic=f64[:, 2:5], opacity=f32[:, 10], beta=f32[:, 11],
                    color=f32[:, 12:15],
                    bbox=sl(ptrs[1], 8 * R).view(torch.int16).view(R, 4),
                    depth=sl(ptrs[2], 4 * R).view(torch.int32).view(R),
                    ntiles=sl(ptrs[3], 4 * R).view(torch.int32).view(R),
                    counts=sl(ptrs[4], 16).view(torch.int64).view(2))

    def state(self) -> dict:
        """Visibility bits [V, S] (int32 words), gradient mask [ceil(V/64), n]
        (int64 words) and accumulator lines [R, 16] (float32) in `projected`."""
        ptrs = [C.c_void_p() for _ in range(3)]
        check("dbs_projected_state", self.lib.dbs_projected_state(
            C.c_void_p(self.projected.data_ptr()), self.n, self.V, *[C.byref(p) for p in ptrs]))
        base = self.projected.data_ptr()
        R, S, W = self.n * self.V, (self.n + 4095) // 4096 * 128, (self.V + 63) // 64

        def sl(p, nbytes):
            off = p.value - base
            return self.projected[off:off + nbytes]

        return dict(visbits=sl(ptrs[0], 4 * self.V * S).view(torch.int32).view(self.V, S),
                    gradmask=sl(ptrs[1], 8 * W * self.n).view(torch.int64).view(W, self.n),
                    sgrad=sl(ptrs[2], 64 * R).view(torch.float32).view(R, 16))

    def bins_arrays(self) -> dict:
        ptrs = [C.c_void_p() for _ in range(3)]
        nt = C.c_int64()
        check("dbs_bins_layout", self.lib.dbs_bins_layout(
            C.c_void_p(self.bins.data_ptr()), self.capacity, self.cams_c, self.V, C.byref(self.cfg_c),
            *[C.byref(p) for p in ptrs], C.byref(nt)))
        base = self.bins.data_ptr()
        T = nt.value

        def sl(p, nbytes, dtype, shape):
            off = (p.value or base) - base
            return self.bins[off:off + nbytes].view(dtype).view(*shape)

        return dict(pair_rec=sl(ptrs[0], 4 * self.capacity, torch.int32, (self.capacity,)),
                    tile_range=sl(ptrs[1], 8 * T, torch.int32, (T, 2)),
                    tile_order=sl(ptrs[2], 4 * T, torch.int32, (T,)), n_tiles=T)

    def tile_offsets(self):
        """First global tile id of every view (host)."""
        tw, th = self.cfg.tile_w, self.cfg.tile_h
        nt = [((w + tw - 1) // tw) * ((h + th - 1) // th) for h, w in self.sizes]
        return np.concatenate([[0], np.cumsum(nt)]).astype(np.int64)


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast: Rasterizer, *tensors):
        params = dict(zip(PARAMS, tensors))
        image, final_T, last = rast.forward(params)
        ctx.rast = rast
        ctx.save_for_backward(*tensors, final_T, last)
        ctx.mark_non_differentiable(final_T, last)
        return image, final_T, last

    @staticmethod
    def backward(ctx, g_image, g_T, g_last):
        saved = ctx.saved_tensors
        params = dict(zip(PARAMS, saved[:len(PARAMS)]))
        final_T, last = saved[len(PARAMS)], saved[len(PARAMS) + 1]
        grads = {k: torch.empty_like(params[k]) for k in PARAMS}   # every element is stored
        ctx.rast.backward(params, g_image.contiguous(), final_T, last, grads, store=True)
        return (None, *[grads[k] for k in PARAMS])


def render(params: dict, rast: Rasterizer):
    """Differentiable render of all views: (image [3*sum HW], final_T, last_index)."""
    return _RenderFn.apply(rast, *[params[k] for k in PARAMS])


class MCMC:
    """Kernel-agnostic MCMC step of Sec. 3.4 on device parameter tensors
    (updated in place): relocation of dead primitives and positional noise.
    Random numbers are inputs: 32-bit uniforms for the draws, standard
    normals for the noise."""

    def __init__(self, n: int, m: int, device="cuda"):
        self.lib = _lib.load()
        self.n, self.m = int(n), int(m)
        wb = self.lib.dbs_mcmc_workspace_bytes(self.n)
        self.workspace = torch.empty(max(wb, 1), dtype=torch.uint8, device=device)
        self.relocated = torch.zeros(1, dtype=torch.int32, device=device)

    def relocate(self, params: dict, dead_opacity: float, rand):
        """rand: int32/uint32 tensor [n] of uniform bits.  Returns the device
        count of moved primitives (no host sync)."""
        sp = _splats_c(params, self.n, self.m)
        check("dbs_mcmc_relocate", self.lib.dbs_mcmc_relocate(
            C.byref(sp), float(dead_opacity), C.c_void_p(rand.data_ptr()), C.c_void_p(self.workspace.data_ptr()),
            self.workspace.numel(), C.c_void_p(self.relocated.data_ptr()), _stream()))
        return self.relocated

    def noise(self, params: dict, z, lr: float, lambda_eps: float, b_prime: float = float(np.log(25.0))):
        sp = _splats_c(params, self.n, self.m)
        check("dbs_mcmc_noise", self.lib.dbs_mcmc_noise(
            C.byref(sp), C.c_void_p(z.data_ptr()), float(lr), float(lambda_eps), float(b_prime), _stream()))


class TrainStep:
    """One fixed-size training step (forward, loss to a target, backward)
    over all views, captured once in a HIP graph and replayed.  The loss is
    L1 (mean over all channel-pixels) or, with `lambda_ssim` set, the
    composite loss of Sec. 3.4: per view (1 - lambda) L1 + lambda (1 - SSIM),
    plus lambda_o sum|o| + lambda_s sum|s|.

    The pair capacity is fixed at capture time from an eager run times
    `headroom`; a replay whose pair count exceeds it sets `overflow`, leaves
    every tile list empty, and `replay()` reports it so the caller can
    rebuild with a larger capacity."""

    def __init__(self, rast: Rasterizer, params: dict, target, headroom: float = 1.1, use_graph=True,
                 lambda_ssim: float | None = None, lambda_o: float = 0.0, lambda_s: float = 0.0):
        self.lambda_ssim, self.lambda_o, self.lambda_s = lambda_ssim, lambda_o, lambda_s
        self.rast = rast
        self.params = params
        self.target = target
        self.scale = 1.0 / float(target.numel())
        self.image, self.final_T, self.last = rast.new_outputs()
        self.dL = torch.empty_like(self.image)
        self.loss = torch.zeros(1, dtype=torch.float32, device=rast.device)
        self.grads = {k: torch.zeros_like(params[k]) for k in PARAMS}
        # eager sizing run
        rast.preprocess(params)
        k = int(rast.counts[1].item())
        rast.ensure_capacity(int(k * headroom) + 1024)
        self.graph = None
        if use_graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                self._body()  # warm up (first-use host work outside the capture)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._body()
            torch.cuda.synchronize()

    def _body(self):
        r = self.rast
        r.preprocess(self.params)
        r.bin_sort()
        r.render_fwd(self.image, self.final_T, self.last)
        if self.lambda_ssim is None:
            r.l1_loss(self.image, self.target, self.scale, self.dL, self.loss)
        else:
            r.photometric_loss(self.image, self.target, self.lambda_ssim, self.dL, self.loss)
        # the reverse pass writes every gradient element: no clearing needed
        r.render_bwd(self.params, self.dL, self.final_T, self.last, self.grads, store=True)
        if self.lambda_o or self.lambda_s:
            r.regularizer(self.params, self.lambda_o, self.lambda_s, self.grads, self.loss)

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self._body()

    def overflowed(self) -> bool:
        return bool(self.rast.overflow.item())
