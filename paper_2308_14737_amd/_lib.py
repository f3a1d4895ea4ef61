"""ctypes binding of the C ABI in include/fmb.h (argument marshalling only).

The shared library libfmb.so is built in-tree by `paper_2308_14737_amd.build`.  If it
is missing, importing this module raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfmb.so")

FMB_OK = 0
STATUS = {0: "FMB_OK", 1: "FMB_ERR_INVALID_ARG", 2: "FMB_ERR_SHAPE", 3: "FMB_ERR_HIP",
          4: "FMB_ERR_OOM", 5: "FMB_ERR_CAPTURE", 6: "FMB_ERR_STATE"}

# name -> (restype, argtypes); mirrors include/fmb.h
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float
_int = ctypes.c_int
SIGNATURES = {
    "fmb_abi_version": (_int, []),
    "fmb_last_error": (ctypes.c_char_p, []),
    "fmb_scene_create": (_int, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _f32]),
    "fmb_scene_rebind": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "fmb_scene_destroy": (_int, [_vp]),
    "fmb_set_cameras": (_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fmb_set_rays": (_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fmb_num_rays": (_i64, [_vp]),
    "fmb_set_colors": (_int, [_vp, _vp, _vp]),
    "fmb_set_flow_pose2": (_int, [_vp, _vp, _vp, _vp]),
    "fmb_set_model": (_int, [_vp, _vp, _i32]),
    "fmb_set_config": (_int, [_vp, _vp, _i32, _i32, _i32, _i32]),
    "fmb_split_statistic": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fmb_prune_mask": (_int, [_i32, _vp, _f32, _vp]),
    "fmb_split_mask": (_int, [_i32, _vp, _f32, _vp]),
    "fmb_split_gaussians": (_int, [_i32] + [_vp] * 10),
    "fmb_render": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fmb_backward": (_int, [_vp] + [_vp] * 13 + [_vp]),
    "fmb_backward_noalloc": (_int, [_vp] + [_vp] * 13 + [_vp]),
    "fmb_batch_create": (_int, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp]),
    "fmb_batch_destroy": (_int, [_vp]),
    "fmb_batch_num_rays": (_i64, [_vp]),
    "fmb_batch_ray_offset": (_i64, [_vp, _i32]),
    "fmb_batch_gauss_offset": (_i64, [_vp, _i32]),
    "fmb_batch_forward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fmb_batch_forward_loss": (_int, [_vp] + [_vp] * 6 + [_vp, _vp, _f32, _vp, _vp, _vp]),
    "fmb_batch_backward": (_int, [_vp] + [_vp] * 13 + [_vp]),
    "fmb_batch_capture": (_int, [_vp] + [_vp] * 16 + [_vp]),
    "fmb_batch_graph_launch": (_int, [_vp, _i32, _vp]),
    "fmb_autotune": (_int, [_vp, _vp] + [_vp] * 16 + [ctypes.c_char_p, _vp]),
    "fmb_loss_grad": (_int, [_i64] + [_vp] * 8 + [_f32, _f32, _i32, _i32, _f32] + [_vp] * 5 + [_vp]),
    "fmb_validate": (_int, [_vp, ctypes.POINTER(_i32), _vp]),
    "fmb_get_config": (_int, [_vp, _vp, ctypes.POINTER(_i32)]),
    "fmb_timing_enable": (_int, [_int]),
    "fmb_kernel_times": (_int, [ctypes.POINTER(ctypes.c_double), _int]),
}

_lib = None


class FmbError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libfmb.so (built by `python -m paper_2308_14737_amd.build`)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python -m paper_2308_14737_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int, where: str):
    if code != FMB_OK:
        msg = load().fmb_last_error()
        raise FmbError(code, where, msg.decode() if msg else "")


def call(name: str, *args):
    lib = load()
    rc = getattr(lib, name)(*args)
    if SIGNATURES[name][0] is _int:
        check(rc, name)
    return rc
