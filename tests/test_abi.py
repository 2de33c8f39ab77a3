"""The C ABI library loads and exports every function include/dbs.h declares
(CPU only: no compute call is made)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dbs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dbs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2501_18630_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2501_18630_amd import build
        build.build()
    return _lib.load()


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    from paper_2501_18630_amd import _lib
    assert set(_lib.EXPORTS) == set(names)


def test_host_only_queries(lib):
    import ctypes as C
    from paper_2501_18630_amd import _lib, renderer, scenes
    assert lib.dbs_version().decode().endswith("gfx950")
    assert lib.dbs_status_string(_lib.ERR_CAPACITY).decode() == "buffer too small"
    cfg = _lib.RasterCfg()
    lib.dbs_default_cfg(C.byref(cfg))
    assert (cfg.tile_w, cfg.tile_h, cfg.batch, cfg.flags) == (16, 16, 256, _lib.FLAG_PERSISTENT)
    assert abs(cfg.t_eps - 1e-4) < 1e-9 and abs(cfg.alpha_max - 0.99) < 1e-7
    cams = renderer.make_cameras([scenes.camera(64, 48), scenes.camera(100, 30)])
    assert lib.dbs_projected_bytes(1000, 2) > 2 * 1000 * 64
    nb = lib.dbs_bins_bytes(5000, cams, 2, C.byref(cfg))
    assert nb >= 5000 * 4 + (4 * 3 + 7 * 2) * 12
    assert lib.dbs_workspace_bytes(1000, 2, 5000, cams, C.byref(cfg)) > 0
    # invalid arguments are rejected before anything touches a device
    assert lib.dbs_projected_bytes(-1, 1) == 0
    bad = _lib.RasterCfg(12, 16, 256, 1e-4, 0.99, 0)
    assert lib.dbs_bins_bytes(10, cams, 2, C.byref(bad)) == 0
    bad = _lib.RasterCfg(16, 16, 256, 1e-4, 1.0, 0)
    assert lib.dbs_workspace_bytes(10, 2, 10, cams, C.byref(bad)) == 0
    assert lib.dbs_preprocess(None, cams, 2, C.byref(cfg), None, 0, None, None) == _lib.ERR_INVALID_ARGUMENT
    sp = _lib.Splats(*([None] * 9), 10, 9)
    assert lib.dbs_preprocess(C.byref(sp), cams, 2, C.byref(cfg), None, 0, None, None) == _lib.ERR_UNSUPPORTED
    sp = _lib.Splats(*([None] * 9), 10, 2)
    assert lib.dbs_preprocess(C.byref(sp), cams, 2, C.byref(cfg), None, 0, None, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dbs_bin_sort(None, cams, 2, C.byref(cfg), 10, 10, None, 0, None, 0, None, None) \
        == _lib.ERR_INVALID_ARGUMENT
    assert lib.dbs_l1_loss(None, None, -1, 1.0, None, None, None) == _lib.ERR_INVALID_ARGUMENT
    # decomposition modes: exclusive pairs are rejected, single modes accepted
    for flags, ok in ((_lib.FLAG_DIFFUSE_ONLY, True), (_lib.FLAG_B_ABOVE | _lib.FLAG_SPECULAR_ONLY, True),
                      (_lib.FLAG_DIFFUSE_ONLY | _lib.FLAG_SPECULAR_ONLY, False),
                      (_lib.FLAG_B_BELOW | _lib.FLAG_B_ABOVE, False), (128, False), (_lib.FLAG_GRAD_STORE, True),
                      (_lib.FLAG_GAUSSIAN_SH, True), (_lib.FLAG_GAUSSIAN_SH | _lib.FLAG_DIFFUSE_ONLY, False),
                      (_lib.FLAG_GAUSSIAN_SH | _lib.FLAG_B_BELOW, False)):
        c2 = _lib.RasterCfg(16, 16, 256, 1e-4, 0.99, _lib.FLAG_PERSISTENT | flags, 0.5)
        assert (lib.dbs_bins_bytes(10, cams, 2, C.byref(c2)) > 0) == ok, flags
    # the Gaussian + SH comparison mode: its own preprocess, which needs the flag and the coefficients
    gcfg = _lib.RasterCfg(16, 16, 256, 1e-4, 0.99, _lib.FLAG_PERSISTENT | _lib.FLAG_GAUSSIAN_SH, 0.0)
    sp = _lib.Splats(*([None] * 9), 10, 0)
    assert lib.dbs_preprocess_gaussian_sh(C.byref(sp), None, cams, 2, C.byref(gcfg), None, 0, None, None) \
        == _lib.ERR_INVALID_ARGUMENT
    sp = _lib.Splats(*([None] * 9), 0, 0)
    assert lib.dbs_preprocess_gaussian_sh(C.byref(sp), None, cams, 2, C.byref(cfg), None, 0, None, None) \
        == _lib.ERR_INVALID_ARGUMENT
    assert lib.dbs_preprocess(C.byref(sp), cams, 2, C.byref(gcfg), None, 0, None, None) == _lib.ERR_INVALID_ARGUMENT
    c2 = _lib.RasterCfg(16, 16, 256, 1e-4, 0.99, _lib.FLAG_PERSISTENT, float("nan"))
    assert lib.dbs_bins_bytes(10, cams, 2, C.byref(c2)) == 0
    # loss and MCMC entry points validate before touching a device
    assert lib.dbs_photometric_loss(None, None, cams, 2, 0.2, None, None, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dbs_mcmc_workspace_bytes(1000) >= 1000 * 20
    sp = _lib.Splats(*([None] * 9), 10, 2)
    assert lib.dbs_mcmc_noise(C.byref(sp), None, 0.1, 1.0, 3.2, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dbs_mcmc_relocate(C.byref(sp), 0.005, None, None, 0, None, None) == _lib.ERR_INVALID_ARGUMENT


def test_no_cpu_fallback_when_library_missing(tmp_path):
    from paper_2501_18630_amd import _lib
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))


def test_raster_config_flags():
    """Host-side mapping of the Python configuration onto dbs_raster_cfg flags."""
    from paper_2501_18630_amd import _lib, renderer
    assert renderer.RasterConfig().to_c().flags == _lib.FLAG_PERSISTENT
    c = renderer.RasterConfig(kernel="gaussian_sh", persistent=False).to_c()
    assert c.flags == _lib.FLAG_GAUSSIAN_SH
    c = renderer.RasterConfig(color="diffuse", b_range="above", b_split=0.25).to_c()
    assert c.flags == _lib.FLAG_PERSISTENT | _lib.FLAG_DIFFUSE_ONLY | _lib.FLAG_B_ABOVE
    assert abs(c.b_split - 0.25) < 1e-7
    with pytest.raises(KeyError):
        renderer.RasterConfig(kernel="gaussian").to_c()
