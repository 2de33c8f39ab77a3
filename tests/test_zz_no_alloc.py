"""dbs_bin_sort_noalloc (the entry point for callers that cannot allocate)
produces the same tile lists, bit for bit, as dbs_bin_sort with a caller
workspace, on two calls in a row (the second on a smaller input, so that the
scratch still holds the first call's contents), and rejects inputs whose
scratch would exceed its fixed size.  Needs an MI355X."""
import ctypes as C

import numpy as np
import pytest

from paper_2501_18630_amd import scenes

pytestmark = pytest.mark.gpu


def _bins(rast):
    b = rast.bins_arrays()
    k = int(rast.counts[1].item())
    return (b["tile_range"].cpu().numpy().copy(), b["tile_order"].cpu().numpy().copy(),
            b["pair_rec"][:k].cpu().numpy().copy())


def _noalloc(rast):
    import torch
    from paper_2501_18630_amd import _lib
    from paper_2501_18630_amd.renderer import _stream
    rast.bins.fill_(0xAB)  # every byte the call must write is overwritten
    _lib.check("dbs_bin_sort_noalloc", rast.lib.dbs_bin_sort_noalloc(
        C.c_void_p(rast.projected.data_ptr()), rast.cams_c, rast.V, C.byref(rast.cfg_c), rast.n, rast.capacity,
        C.c_void_p(rast.bins.data_ptr()), rast.bins.numel(), C.c_void_p(rast.overflow.data_ptr()), _stream()))
    torch.cuda.synchronize()
    return int(rast.overflow.item())


def test_noalloc_bin_sort_matches_workspace_call():
    import torch
    from paper_2501_18630_amd import _lib, renderer
    # two calls in a row, the second on a smaller input
    for n, m, (w0, h0), second in ((60_000, 2, (256, 192), (200, 150)), (9_000, 1, (97, 61), None)):
        s = scenes.uniform_box_scene(n, (-3, -3, 2), (3, 3, 10), m=m, seed=n % 97)
        cams = [scenes.look_at_camera([0.5, -0.3, -6.0], w0, h0)]
        if second:
            cams.append(scenes.look_at_camera([-2.0, 1.0, -5.0], *second))
        rast = renderer.Rasterizer(cams, n, m)
        params = renderer.to_device(s)
        image, T, last = rast.forward(params)       # dbs_bin_sort with a caller workspace
        torch.cuda.synchronize()
        need = rast.lib.dbs_workspace_bytes(n, rast.V, rast.capacity, rast.cams_c, C.byref(rast.cfg_c))
        assert 0 < need <= _lib.NOALLOC_SCRATCH_BYTES
        assert int(rast.overflow.item()) == 0 and int(rast.counts[1].item()) > 1000
        ref = _bins(rast)
        ref_img = image.clone()
        assert _noalloc(rast) == 0
        got = _bins(rast)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        rast.render_fwd(image, T, last)
        torch.cuda.synchronize()
        assert torch.equal(image, ref_img)


def test_noalloc_bin_sort_rejects_oversize():
    import torch
    from paper_2501_18630_amd import _lib, renderer
    from paper_2501_18630_amd.renderer import _stream
    cams = [scenes.camera(1920, 1080)]
    n = 3_000_000
    cams_c = renderer.make_cameras(cams)
    cfg = renderer.RasterConfig().to_c()
    lib = _lib.load()
    cap = 20_000_000
    assert lib.dbs_workspace_bytes(n, 1, cap, cams_c, C.byref(cfg)) > _lib.NOALLOC_SCRATCH_BYTES
    bb = lib.dbs_bins_bytes(cap, cams_c, 1, C.byref(cfg))
    projected = torch.zeros(lib.dbs_projected_bytes(n, 1), dtype=torch.uint8, device="cuda")
    bins = torch.zeros(bb, dtype=torch.uint8, device="cuda")
    st = lib.dbs_bin_sort_noalloc(C.c_void_p(projected.data_ptr()), cams_c, 1, C.byref(cfg), n, cap,
                                  C.c_void_p(bins.data_ptr()), bb, None, _stream())
    assert st == _lib.ERR_CAPACITY
