"""ctypes declarations of the C ABI in include/nedf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnedf.so")

MAX_OBJECTS = 32
W2L_FLOATS = 16

NEDF_OK = 0
STATUS = {0: "OK", 1: "NULL", 2: "SHAPE", 3: "DTYPE", 4: "ALIGN", 5: "WORKSPACE", 6: "CAPACITY",
          7: "HIP", 8: "UNSUPPORTED"}
DTYPES = {"f32": 0, "bf16": 1, "fp8": 2, "fp8mx": 3}
FIELDS = {"sphere": 0, "slab": 1, "mlp": 2}
SIGMA_MODES = {"softplus": 0, "softplus_masked": 1, "sdf": 2}
IN_KINDS = {"xyz": 0, "pluecker": 1, "points16": 2}
OPS = {"march": 0, "infer": 1, "shade": 2, "shadow": 3}
TUNE_KERNELS = {"march": 0, "nedf": 1, "slabs": 2}


class MlpShape(C.Structure):
    _fields_ = [("in_kind", C.c_int32), ("enc_L", C.c_int32), ("width", C.c_int32),
                ("n_hidden", C.c_int32), ("n_out", C.c_int32), ("rgb_width", C.c_int32),
                ("dir_L", C.c_int32)]


class Mlp(C.Structure):
    _fields_ = [("shape", MlpShape), ("dtype", C.c_int32), ("blob", C.c_void_p)]


class Object(C.Structure):
    _fields_ = [("field", C.c_int32), ("sigma_mode", C.c_int32), ("bound", C.c_float),
                ("param", C.c_float * 6), ("density", Mlp), ("nedf", Mlp)]


class Scene(C.Structure):
    _fields_ = [("n_objects", C.c_int32), ("objects", C.POINTER(Object)), ("n_inst", C.c_int32),
                ("inst_object", C.c_void_p), ("inst_w2l", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("at", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class Rays(C.Structure):
    _fields_ = [("kind", C.c_int32), ("camera", Camera), ("origins", C.c_void_p), ("dirs", C.c_void_p),
                ("n", C.c_int64)]


class MarchOpts(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("clip_to_bound", C.c_int32), ("t_near", C.c_float),
                ("t_far", C.c_float), ("hit_threshold", C.c_float), ("dtype", C.c_int32)]


class InferOpts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("p_lo", C.c_float), ("p_hi", C.c_float), ("refine_steps", C.c_int32),
                ("refine_h", C.c_float), ("march", MarchOpts)]


class ShadeOpts(C.Structure):
    _fields_ = [("K", C.c_int32), ("h", C.c_float), ("clear_rgb", C.c_float * 3), ("dtype", C.c_int32),
                ("rs_sigma", C.c_float), ("rs_samples", C.c_int32)]


class ShadowOpts(C.Structure):
    _fields_ = [("eps", C.c_float), ("beta", C.c_float), ("method", C.c_int32), ("infer", InferOpts),
                ("directional_mask", C.c_uint32), ("dir_distance", C.c_float)]


class TrainOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("w_hit", C.c_float), ("bound", C.c_float)]


TUNE_MAX = 8


class TuneReport(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("dtype", C.c_int32), ("n_candidates", C.c_int32),
                ("candidate", C.c_int32 * TUNE_MAX), ("ms", C.c_float * TUNE_MAX), ("chosen", C.c_int32)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("nedf_version", C.c_char_p, []),
    ("nedf_last_error", C.c_char_p, []),
    ("nedf_status_string", C.c_char_p, [C.c_int32]),
    ("nedf_mlp_packed_bytes", C.c_size_t, [C.POINTER(MlpShape), C.c_int32]),
    ("nedf_pack_mlp", C.c_int32, [C.POINTER(MlpShape), C.c_int32, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_size_t]),
    ("nedf_compose_transforms", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("nedf_workspace_size", C.c_size_t, [C.c_int32, C.POINTER(Scene), C.POINTER(Rays), C.c_int64]),
    ("nedf_check_status", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("nedf_profile_enable", C.c_int32, [C.c_int32]),
    ("nedf_profile_read", C.c_int32, [C.c_int32, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]),
    ("nedf_ws_counters", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    ("nedf_infer_depth_id", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.POINTER(InferOpts), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nedf_infer_depth_id_static", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.POINTER(InferOpts),
                                               C.c_void_p, C.c_void_p, C.c_void_p]),
    ("nedf_static_scratch_bytes", C.c_size_t, []),
    ("nedf_infer_keys", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.POINTER(InferOpts), C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nedf_compose_keys", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.POINTER(InferOpts),
                                      C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.c_void_p]),
    ("nedf_shade_deferred", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.c_void_p, C.c_void_p,
                                        C.POINTER(ShadeOpts), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nedf_shadow", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, C.POINTER(ShadowOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_size_t, C.c_void_p]),
    ("nedf_train_state_bytes", C.c_size_t, [C.POINTER(MlpShape)]),
    ("nedf_train_workspace_size", C.c_size_t, [C.POINTER(MlpShape), C.c_int32]),
    ("nedf_train_init", C.c_int32, [C.POINTER(MlpShape), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    ("nedf_train_step", C.c_int32, [C.POINTER(MlpShape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int32, C.POINTER(TrainOpts), C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    ("nedf_train_export", C.c_int32, [C.POINTER(MlpShape), C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_void_p), C.c_void_p]),
    ("nedf_fp8_calibrate_workspace_size", C.c_size_t, [C.POINTER(MlpShape), C.c_int32]),
    ("nedf_fp8_calibrate", C.c_int32, [C.POINTER(MlpShape), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                       C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                       C.c_void_p]),
    ("nedf_march_depth", C.c_int32, [C.POINTER(Scene), C.POINTER(Rays), C.POINTER(MarchOpts), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nedf_tune_candidates", C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("nedf_tune_get", C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    ("nedf_tune_set", C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    ("nedf_autotune", C.c_int32, [C.c_int32, C.c_int32, C.POINTER(Scene), C.POINTER(Rays), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                                  C.POINTER(TuneReport)]),
]

_lib = None


class NedfError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({message})")
        self.status = status


def load() -> C.CDLL:
    """Load libnedf.so (built by paper_2308_04669_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_04669_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != NEDF_OK:
        msg = load().nedf_last_error().decode(errors="replace")
        raise NedfError(status, where, msg)
