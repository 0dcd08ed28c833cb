"""ctypes mirror of include/sgs.h and loader of the in-tree libsgs.so.

Argument marshalling only: every step of the rasterizer runs in the HIP
library.  There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgs.so")

P = C.c_void_p


class Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("_pad", C.c_int32),
                ("mean", P), ("log_scale", P), ("quat", P), ("skew", P),
                ("opa_logit", P), ("opa2_logit", P), ("opa_dir", P), ("sh", P)]


class ParamsGrad(C.Structure):
    _fields_ = [("mean", P), ("log_scale", P), ("quat", P), ("skew", P),
                ("opa_logit", P), ("opa2_logit", P), ("opa_dir", P), ("sh", P),
                ("densify_uv", P), ("densify_z", P), ("densify_count", P)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("w2c", C.c_float * 12), ("campos", C.c_float * 3), ("near_z", C.c_float),
                ("bg", C.c_float * 3), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("tile_base", C.c_int32), ("pix_base", C.c_int64)]


class Options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("filter_s", C.c_float),
                ("compensate", C.c_int32), ("guard", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("sort_mode", C.c_int32),
                ("blend_batch", C.c_int32), ("split_tiles", C.c_int32), ("depth_digit_bits", C.c_int32),
                ("blend_lists", C.c_int32)]


class Geom(C.Structure):
    _fields_ = [("rec", P), ("depth", P), ("rect", P), ("tiles", P), ("block_off", P), ("rows", P),
                ("enhanced", C.c_int32), ("_pad", C.c_int32)]


class GeomGrad(C.Structure):
    _fields_ = [("rec", P)]


class Schedule(C.Structure):
    _fields_ = [("tile_order", P), ("work_counter", P)]


class DensifyOptions(C.Structure):
    _fields_ = [("tau_uv", C.c_float), ("tau_z", C.c_float), ("dense_scale", C.c_float),
                ("split_shrink", C.c_float)]


class DensifyOut(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("mean", P), ("log_scale", P), ("quat", P), ("skew", P),
                ("opa_logit", P), ("opa2_logit", P), ("opa_dir", P), ("sh", P), ("parent", P)]


class AdamGroup(C.Structure):
    _fields_ = [("param", P), ("grad", P), ("m1", P), ("m2", P), ("n", C.c_int64), ("lr", C.c_float),
                ("_pad", C.c_int32)]


ADAM_MAX_GROUPS = 16

STRUCTS = [Params, ParamsGrad, Camera, Options, Geom, GeomGrad, Schedule, AdamGroup, DensifyOptions,
           DensifyOut]

# bytes of the fixed per-device scratch of sgs_bin_sort_noalloc (SGS_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20

STATUS = {0: "SGS_OK", 1: "SGS_EINVAL", 2: "SGS_ECAPACITY", 3: "SGS_EHIP", 4: "SGS_EUNSUPPORTED"}

# name -> (restype, argtypes)
SIGNATURES = {
    "sgs_default_options": (None, [C.POINTER(Options)]),
    "sgs_struct_size": (C.c_size_t, [C.c_int32]),
    "sgs_status_string": (C.c_char_p, [C.c_int]),
    "sgs_camera_from_gl": (C.c_int, [C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_double,
                                     C.c_double, C.c_float, C.POINTER(C.c_float), C.POINTER(Camera)]),
    "sgs_camera_layout": (C.c_int, [C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sgs_geom_rec_floats": (C.c_int64, [C.c_int64, C.c_int32]),
    "sgs_geom_block_entries": (C.c_int64, [C.c_int64, C.c_int32]),
    "sgs_bin_sort_scratch_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64, C.POINTER(Options)]),
    "sgs_bin_sort_mode": (C.c_int32, [C.POINTER(Options), C.c_int64, P, C.c_int32, C.c_int32]),
    "sgs_preprocess": (C.c_int, [C.POINTER(Params), C.POINTER(Camera), P, C.c_int32,
                                 C.POINTER(Options), C.POINTER(Geom), P]),
    "sgs_bin_sort": (C.c_int, [C.POINTER(Geom), C.c_int64, C.POINTER(Camera), P, C.c_int32,
                               C.POINTER(Options), C.c_int64, P, P, P, P, C.POINTER(Schedule), P,
                               C.c_size_t, P]),
    "sgs_bin_sort_noalloc": (C.c_int, [C.POINTER(Geom), C.c_int64, C.POINTER(Camera), P, C.c_int32,
                                       C.POINTER(Options), C.c_int64, P, P, P, P, C.POINTER(Schedule), P]),
    "sgs_render_fwd": (C.c_int, [C.POINTER(Geom), C.c_int64, P, C.c_int64, P, C.POINTER(Schedule),
                                 C.POINTER(Camera), P, C.c_int32, C.c_int32, C.POINTER(Options), P, P, P,
                                 P, P, C.c_int64, P]),
    "sgs_default_densify_options": (None, [C.POINTER(DensifyOptions)]),
    "sgs_densify_scratch_words": (C.c_int64, [C.c_int64]),
    "sgs_densify": (C.c_int, [C.POINTER(Params), P, P, P, C.POINTER(DensifyOptions), P, C.POINTER(DensifyOut), P,
                              P, P]),
    "sgs_adam_step": (C.c_int, [C.POINTER(AdamGroup), C.c_int32, P, C.c_float, C.c_float, C.c_float, P]),
    "sgs_render_bwd": (C.c_int, [C.POINTER(Params), C.POINTER(Geom), C.c_int64, P, C.c_int64, P,
                                 C.POINTER(Schedule), C.POINTER(Camera), P, C.c_int32, C.POINTER(Options),
                                 P, P, P, C.c_int64, C.POINTER(GeomGrad), C.POINTER(ParamsGrad), P]),
}

_lib = None


class SgsError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")
        self.code = code


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads libsgs.so (built by paper_2605_18334_amd.build) and checks the
    ctypes struct mirrors against the library's own sizeof."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2605_18334_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    for i, s in enumerate(STRUCTS):
        if lib.sgs_struct_size(i) != C.sizeof(s):
            raise RuntimeError(f"ABI mismatch for {s.__name__}: C {lib.sgs_struct_size(i)} vs ctypes {C.sizeof(s)}")
    _lib = lib
    return lib


def check(fn: str, code: int) -> None:
    if code != 0:
        raise SgsError(fn, code)


def default_options(**over) -> Options:
    o = Options()
    load().sgs_default_options(C.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o
