"""ctypes declarations of the C ABI in include/eag.h (argument marshalling
only; every computation runs in the HIP library)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeag.so")

EAG_OK = 0
EAG_NOT_READY = 1
STATUS_NAMES = {0: "EAG_OK", 1: "EAG_NOT_READY", -1: "EAG_ERR_INVALID_ARGUMENT", -2: "EAG_ERR_WORKSPACE_TOO_SMALL",
                -3: "EAG_ERR_OUT_OF_BUDGET", -4: "EAG_ERR_DEVICE", -5: "EAG_ERR_CANCELLED",
                -6: "EAG_ERR_UNKNOWN_TICKET", -7: "EAG_ERR_INTERNAL"}

JITTER, ADDITIVE_EMISSION, DETACH_BOUNCE = 1, 2, 4
EDIT_SET_RADIANCE, EDIT_SCALE_RADIANCE, EDIT_SET_ALBEDO, EDIT_SET_EMISSIVE, EDIT_TRANSFORM = 1, 2, 3, 4, 5
FWD_PIXEL_FLOATS = 28
STAGE0_FLOATS = 8
ACCUM_SCALE = 4294967296.0

vp = C.c_void_p
fp = C.POINTER(C.c_float)


class Surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", vp), ("rot", vp), ("scale", vp), ("opacity", vp), ("albedo", vp),
                ("radiance", vp), ("emissive", vp)]


class SurfelGrads(C.Structure):
    _fields_ = [("pos", vp), ("rot", vp), ("scale", vp), ("opacity", vp), ("albedo", vp), ("radiance", vp)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3), ("vfov_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class TraceParams(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("rr_start", C.c_int32), ("tau_E", C.c_float),
                ("T_min", C.c_float), ("t_min", C.c_float), ("k_sigma", C.c_float), ("depth_quantum", C.c_float),
                ("kbuf", C.c_int32), ("camera_id", C.c_uint32), ("seed", C.c_uint64), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


class BvhInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("max_depth", C.c_int32), ("root", C.c_int32), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3), ("nodes", vp), ("records", vp), ("perm", vp), ("nodes4", vp),
                ("n_nodes4", C.c_int32), ("depth4", C.c_int32)]


class Edit(C.Structure):
    _fields_ = [("kind", C.c_int32), ("idx", vp), ("count", C.c_int64), ("value", C.c_float * 12)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class SurfelsOut(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", vp), ("rot", vp), ("scale", vp), ("opacity", vp), ("albedo", vp),
                ("radiance", vp), ("emissive", vp)]


class SurfelAttrs(C.Structure):
    _fields_ = [("n", C.c_int64), ("albedo", vp), ("radiance", vp), ("emissive", vp)]


class ServerConfig(C.Structure):
    _fields_ = [("arena", vp), ("arena_bytes", C.c_size_t), ("max_live_requests", C.c_int32),
                ("paths_per_launch", C.c_int64), ("stream", vp)]


class Request(C.Structure):
    _fields_ = [("cam", Camera), ("params", TraceParams), ("out_rgb", vp)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("scene_version", C.c_uint32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("paths", C.c_uint64)]


P = C.POINTER
SIGNATURES = {
    "eag_last_error": (C.c_char_p, []),
    "eag_abi_version": (C.c_uint32, []),
    "eag_default_params": (None, [P(TraceParams)]),
    "eag_bvh_bytes": (C.c_size_t, [C.c_int64]),
    "eag_build_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "eag_build_bvh": (C.c_int, [P(Surfels), vp, C.c_size_t, vp, C.c_size_t, vp, P(vp)]),
    "eag_refit_bvh": (C.c_int, [vp, P(Surfels), vp, C.c_size_t, vp]),
    "eag_bvh_get_info": (C.c_int, [vp, P(BvhInfo)]),
    "eag_bvh_destroy": (None, [vp]),
    "eag_trace_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "eag_trace_rays": (C.c_int, [vp, P(Surfels), P(TraceParams), C.c_int64, vp, vp, vp, vp, vp, C.c_int32, vp, vp,
                                 C.c_size_t, vp]),
    "eag_init": (C.c_int, []),
    "eag_trace_rays_noalloc": (C.c_int, [vp, P(Surfels), P(TraceParams), C.c_int64, vp, vp, vp, vp, vp, C.c_int32,
                                         vp, vp]),
    "eag_fwd_state_floats": (C.c_int64, [P(Camera), C.c_int32, P(TraceParams)]),
    "eag_render_workspace_bytes": (C.c_size_t, [C.c_int64, P(Camera), C.c_int32, P(TraceParams)]),
    "eag_backward_workspace_bytes": (C.c_size_t, [C.c_int64, P(Camera), C.c_int32, P(TraceParams)]),
    "eag_render_single_bounce": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, vp,
                                           C.c_size_t, vp]),
    "eag_single_bounce_backward": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp,
                                             P(SurfelGrads), vp, C.c_size_t, vp]),
    "eag_path_trace_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "eag_path_trace": (C.c_int, [vp, P(Surfels), P(Camera), P(TraceParams), C.c_uint32, C.c_uint32, vp, vp, vp,
                                 C.c_size_t, vp]),
    "eag_accum_resolve": (C.c_int, [vp, C.c_int64, C.c_int32, vp, vp]),
    "eag_emitters_bytes": (C.c_size_t, [C.c_int64]),
    "eag_emitters_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "eag_build_emitters": (C.c_int, [P(Surfels), P(TraceParams), C.c_float, vp, C.c_size_t, vp, C.c_size_t, vp,
                                     P(vp)]),
    "eag_emitters_get_info": (C.c_int, [vp, P(C.c_int64), P(C.c_double), P(C.c_int32)]),
    "eag_emitters_destroy": (None, [vp]),
    "eag_path_trace_mis_workspace_bytes": (C.c_size_t, [C.c_int64, P(Camera), P(TraceParams)]),
    "eag_path_trace_mis": (C.c_int, [vp, P(Surfels), vp, P(Camera), P(TraceParams), C.c_uint32, C.c_uint32, vp, vp,
                                     vp, C.c_size_t, vp]),
    "eag_apply_edit": (C.c_int, [P(Edit), P(SurfelAttrs), vp]),
    "eag_select_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "eag_select_box": (C.c_int, [P(Surfels), P(C.c_float), P(C.c_float), vp, vp, vp, C.c_size_t, vp]),
    "eag_move_surfels": (C.c_int, [P(SurfelsOut), vp, C.c_int64, P(C.c_float), P(C.c_float), P(C.c_float), vp]),
    "eag_delete_surfels": (C.c_int, [P(SurfelsOut), vp, C.c_int64, vp]),
    "eag_duplicate_surfels": (C.c_int, [P(Surfels), vp, C.c_int64, P(SurfelsOut), P(C.c_float), P(C.c_float),
                                        P(C.c_float), vp]),
    "eag_bvh_sah_cost": (C.c_int, [vp, vp, vp, C.c_size_t, vp]),
    "eag_stage0_workspace_bytes": (C.c_size_t, [C.c_int64, P(Camera), C.c_int32]),
    "eag_render_stage0": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, vp, C.c_size_t,
                                    vp]),
    "eag_stage0_loss_workspace_bytes": (C.c_size_t, [P(Camera), C.c_int32]),
    "eag_stage0_loss": (C.c_int, [vp, vp, vp, vp, P(Camera), C.c_int32, P(TraceParams), P(C.c_float), vp, vp, vp,
                                  C.c_size_t, vp]),
    "eag_stage0_backward": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, P(SurfelGrads),
                                      vp, vp, C.c_size_t, vp]),
    "eag_bake_workspace_bytes": (C.c_size_t, [C.c_int64, P(Camera), C.c_int32]),
    "eag_render_zero_bounce": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, C.c_size_t,
                                         vp]),
    "eag_zero_bounce_backward": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, vp,
                                           C.c_size_t, vp]),
    "eag_bake_loss": (C.c_int, [vp, vp, C.c_int64, vp, vp, vp]),
    "eag_adam_step": (C.c_int, [vp, vp, vp, vp, C.c_int64, P(Adam), C.c_int32, vp]),
    "eag_bake_step": (C.c_int, [vp, P(Surfels), P(Camera), C.c_int32, P(TraceParams), vp, vp, vp, vp, P(Adam),
                                C.c_int32, vp, vp, C.c_size_t, vp]),
    "eag_serve_arena_bytes": (C.c_size_t, [C.c_int64, C.c_int32, C.c_size_t]),
    "eag_serve_create": (C.c_int, [P(Surfels), P(ServerConfig), P(vp)]),
    "eag_serve_submit": (C.c_int, [vp, P(Request), P(C.c_uint64)]),
    "eag_serve_edit": (C.c_int, [vp, P(Edit), P(C.c_uint64)]),
    "eag_serve_poll": (C.c_int, [vp, C.c_uint64, P(Result)]),
    "eag_serve_cancel": (C.c_int, [vp, C.c_uint64]),
    "eag_serve_destroy": (C.c_int, [vp]),
}

_lib = None


def load():
    """Load libeag.so (after torch, so that both share one HIP runtime).
    Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_23065_amd.build` "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    missing = []
    for name, (res, args) in SIGNATURES.items():
        try:
            f = getattr(lib, name)
        except AttributeError:
            missing.append(name)
            continue
        f.restype = res
        f.argtypes = args
    lib.missing_symbols = missing
    _lib = lib
    return lib


class EagError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status < 0:
        raise EagError(status, load().eag_last_error().decode())
    return status
