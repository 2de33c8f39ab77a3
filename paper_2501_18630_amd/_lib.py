"""ctypes binding of libdbs.so (the C ABI declared in include/dbs.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels of the library.  There is no CPU fallback: if the library is not
built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbs.so")

OK, ERR_INVALID_ARGUMENT, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED = range(5)
MAX_LOBES = 8
MAX_VIEWS = 1024
NOALLOC_SCRATCH_BYTES = 64 << 20
FLAG_PERSISTENT = 1
FLAG_DIFFUSE_ONLY = 2
FLAG_SPECULAR_ONLY = 4
FLAG_B_BELOW = 8
FLAG_B_ABOVE = 16
FLAG_GAUSSIAN_SH = 32
FLAG_GRAD_STORE = 64

PARAMS = ("means", "scales", "quats", "opacities", "betas", "diffuse",
          "lobe_angles", "lobe_colors", "lobe_betas")

EXPORTS = ("dbs_default_cfg", "dbs_projected_bytes", "dbs_bins_bytes", "dbs_workspace_bytes",
           "dbs_preprocess", "dbs_preprocess_gaussian_sh", "dbs_bin_sort", "dbs_bin_sort_noalloc", "dbs_render_fwd", "dbs_render_bwd", "dbs_l1_loss",
           "dbs_photometric_loss", "dbs_regularizer", "dbs_mcmc_workspace_bytes", "dbs_mcmc_relocate",
           "dbs_mcmc_noise",
           "dbs_raster_bwd", "dbs_raster_bwd_count", "dbs_project_bwd", "dbs_render_stats",
           "dbs_projected_layout", "dbs_projected_state", "dbs_bins_layout", "dbs_status_string", "dbs_version")


class DbsError(RuntimeError):
    def __init__(self, call: str, status: int, msg: str):
        super().__init__(f"{call} failed: {msg} (status {status})")
        self.status = status


class Splats(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in PARAMS] + [("n", C.c_int64), ("m", C.c_int32)]


class Grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in PARAMS]


class Camera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("near_plane", C.c_float), ("background", C.c_float * 3)]


class RasterCfg(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("batch", C.c_int32),
                ("t_eps", C.c_float), ("alpha_max", C.c_float), ("flags", C.c_uint32), ("b_split", C.c_float)]


_lib = None


def _declare(lib):
    P, I64, I32, SZ = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    lib.dbs_default_cfg.argtypes = [P]
    lib.dbs_default_cfg.restype = None
    lib.dbs_projected_bytes.argtypes = [I64, I32]
    lib.dbs_projected_bytes.restype = SZ
    lib.dbs_bins_bytes.argtypes = [I64, P, I32, P]
    lib.dbs_bins_bytes.restype = SZ
    lib.dbs_workspace_bytes.argtypes = [I64, I32, I64, P, P]
    lib.dbs_workspace_bytes.restype = SZ
    lib.dbs_preprocess.argtypes = [P, P, I32, P, P, SZ, P, P]
    lib.dbs_preprocess_gaussian_sh.argtypes = [P, P, P, I32, P, P, SZ, P, P]
    lib.dbs_bin_sort.argtypes = [P, P, I32, P, I64, I64, P, SZ, P, SZ, P, P]
    lib.dbs_bin_sort_noalloc.argtypes = [P, P, I32, P, I64, I64, P, SZ, P, P]
    lib.dbs_render_fwd.argtypes = [P, P, P, I32, P, I64, P, P, P, P]
    lib.dbs_render_bwd.argtypes = [P, P, P, P, I32, P, P, P, P, P, P]
    lib.dbs_raster_bwd.argtypes = [P, P, P, I32, P, I64, P, P, P, P]
    lib.dbs_raster_bwd_count.argtypes = [P, P, P, I32, P, I64, P, P, P, P, P]
    lib.dbs_project_bwd.argtypes = [P, P, P, I32, P, P, P]
    lib.dbs_render_stats.argtypes = [P, P, P, I32, P, I64, P, P, P, P]
    lib.dbs_l1_loss.argtypes = [P, P, I64, C.c_float, P, P, P]
    lib.dbs_photometric_loss.argtypes = [P, P, P, I32, C.c_float, P, P, P]
    lib.dbs_regularizer.argtypes = [P, C.c_float, C.c_float, P, P, P]
    lib.dbs_mcmc_workspace_bytes.argtypes = [I64]
    lib.dbs_mcmc_workspace_bytes.restype = SZ
    lib.dbs_mcmc_relocate.argtypes = [P, C.c_float, P, P, SZ, P, P]
    lib.dbs_mcmc_noise.argtypes = [P, P, C.c_float, C.c_float, C.c_float, P]
    lib.dbs_projected_layout.argtypes = [P, I64, I32] + [C.POINTER(C.c_void_p)] * 5
    lib.dbs_projected_state.argtypes = [P, I64, I32] + [C.POINTER(C.c_void_p)] * 3
    lib.dbs_bins_layout.argtypes = [P, I64, P, I32, P] + [C.POINTER(C.c_void_p)] * 3 + [C.POINTER(C.c_int64)]
    for f in ("dbs_preprocess", "dbs_preprocess_gaussian_sh", "dbs_bin_sort", "dbs_bin_sort_noalloc", "dbs_render_fwd", "dbs_render_bwd", "dbs_l1_loss",
              "dbs_photometric_loss", "dbs_regularizer", "dbs_mcmc_workspace_bytes", "dbs_mcmc_relocate",
           "dbs_mcmc_noise", "dbs_raster_bwd", "dbs_raster_bwd_count", "dbs_project_bwd", "dbs_render_stats",
              "dbs_projected_layout", "dbs_projected_state", "dbs_bins_layout"):
        getattr(lib, f).restype = C.c_int
    lib.dbs_status_string.argtypes = [C.c_int]
    lib.dbs_status_string.restype = C.c_char_p
    lib.dbs_version.argtypes = []
    lib.dbs_version.restype = C.c_char_p


def load(path: str | None = None):
    """Load libdbs.so.  torch is imported first so that the library binds to
    the HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    import torch  # noqa: F401  (brings in libamdhip64 before the library)
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is not built; run `python -m paper_2501_18630_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(p)
    _declare(lib)
    if path is None:
        _lib = lib
    return lib


def check(call: str, status: int):
    if status != OK:
        msg = load().dbs_status_string(status).decode()
        raise DbsError(call, status, msg)
