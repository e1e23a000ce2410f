"""ctypes mirror of include/misslam.h and the loader of libmisslam.so.

Argument marshalling only; no computation happens in Python.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmisslam.so")

OK, EINVAL, ESHAPE, EWORKSPACE, EHIP, ECAPACITY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FLAG_NONSPD_BLOCK, FLAG_PCG_BREAKDOWN, FLAG_NONFINITE, FLAG_FRAME_REJECT, FLAG_GRAPH_OVERFLOW = 1, 2, 4, 8, 16
FLAG_SYNC_TIMEOUT = 32
WEIGHT_GAUSS, WEIGHT_LINEAR = 0, 1
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
LAUNCH_PLAIN, LAUNCH_COOPERATIVE, LAUNCH_KERNELS = 0, 1, 2
SOLVE_TEXTBOOK, SOLVE_PIPELINED = 0, 1
MAX_K, MAX_PCG, MAX_ROW, MAX_LIST, SOLVE_ROWS = 8, 64, 32, 2048, 16
MAX_KEYPOINTS = 1 << 24
NOALLOC_SCRATCH_BYTES = 96 << 20

c_float_p = ctypes.POINTER(ctypes.c_float)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("T", ctypes.c_float * 3)]


class Points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("px", ctypes.c_void_p), ("py", ctypes.c_void_p), ("pz", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p), ("nz", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("stamp", ctypes.c_void_p), ("stable", ctypes.c_void_p)]


class Nodes(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("gx", ctypes.c_void_p), ("gy", ctypes.c_void_p), ("gz", ctypes.c_void_p),
                ("params", ctypes.c_void_p)]


class Graph(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("bsr_cap", ctypes.c_int32),
                ("knn_idx", ctypes.c_void_p), ("knn_w", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("list_ptr", ctypes.c_void_p), ("list_pts", ctypes.c_void_p), ("list_key", ctypes.c_void_p),
                ("info", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("weight_kind", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("w_rot", ctypes.c_float), ("w_reg", ctypes.c_float), ("w_data", ctypes.c_float),
                ("eps_d", ctypes.c_double), ("cos_eps_n", ctypes.c_double), ("lambda_", ctypes.c_float),
                ("gn_iters", ctypes.c_int32), ("pcg_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("reject_threshold", ctypes.c_float),
                ("solve_launch", ctypes.c_int32), ("sync_spin_limit", ctypes.c_int32),
                ("solve_form", ctypes.c_int32), ("asm_waves", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("e_data", ctypes.c_double), ("e_rot", ctypes.c_double), ("e_reg", ctypes.c_double),
                ("pcg_resid", ctypes.c_double * (MAX_PCG + 1)), ("n_valid", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("pcg_iters_done", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("e_corr", ctypes.c_double), ("lm_e", ctypes.c_double), ("lm_e_trial", ctypes.c_double),
                ("lm_lambda", ctypes.c_float), ("lm_accepted", ctypes.c_int32), ("e_pose_r", ctypes.c_double),
                ("e_pose_p", ctypes.c_double)]


class PoseWeights(ctypes.Structure):
    _fields_ = [("w_r", ctypes.c_float), ("w_p", ctypes.c_float)]


class LMParams(ctypes.Structure):
    _fields_ = [("lambda0", ctypes.c_float), ("up", ctypes.c_float), ("down", ctypes.c_float),
                ("lambda_min", ctypes.c_float), ("lambda_max", ctypes.c_float)]


class Keypoints(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("w_corr", ctypes.c_float), ("point", ctypes.c_void_p),
                ("target", ctypes.c_void_p)]


class FuseParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("cos_delta", ctypes.c_double), ("w_max", ctypes.c_float),
                ("frame", ctypes.c_int32)]


class GrowParams(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_float), ("node_spacing", ctypes.c_float), ("tau_weight", ctypes.c_float),
                ("tau_time", ctypes.c_int32), ("frame", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("points", Points), ("nodes", Nodes), ("graph", Graph), ("depth", ctypes.c_void_p),
                ("camera", Camera), ("pose", Pose), ("report", ctypes.c_void_p)]


P = ctypes.POINTER
vp = ctypes.c_void_p
st = ctypes.c_int32

# symbol -> (restype, argtypes); every function declared in include/misslam.h
SIGNATURES = {
    "misslam_default_params": (None, [P(Params)]),
    "misslam_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "misslam_last_hip_error": (ctypes.c_int32, []),
    "misslam_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  P(Params)]),
    "misslam_normal_map": (st, [vp, P(Camera), vp, vp]),
    "misslam_build_graph": (st, [P(Points), P(Nodes), P(Params), P(Graph), vp, ctypes.c_size_t, vp]),
    "misslam_warp": (st, [P(Points), P(Nodes), P(Graph), P(Pose), vp, vp, vp]),
    "misslam_build_normal_eq": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params), vp, vp, vp,
                                     vp, vp, ctypes.c_size_t, vp]),
    "misslam_pcg_solve": (st, [P(Graph), ctypes.c_int32, vp, vp, P(Params), vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_gn_register": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params), vp, vp, vp,
                                 ctypes.c_size_t, vp]),
    "misslam_gn_register_keypoints": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params),
                                           P(Keypoints), vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_gn_register_noalloc": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params), vp, vp,
                                         vp]),
    "misslam_default_lm_params": (None, [P(LMParams)]),
    "misslam_joint_register": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(PoseWeights),
                                    P(Keypoints), P(Params), vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_lm_register": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params), P(Keypoints),
                                 P(LMParams), vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_fuse_color": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(FuseParams), vp, vp,
                                ctypes.c_int64, vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_grow_color": (st, [P(Points), P(Nodes), vp, vp, vp, P(Camera), P(Pose), P(GrowParams), vp, vp,
                                ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]),
    "misslam_fuse": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(FuseParams), vp, vp, vp,
                          ctypes.c_size_t, vp]),
    "misslam_energy_vjp": (st, [P(Points), P(Nodes), P(Graph), vp, P(Camera), P(Pose), P(Params), vp, vp, vp, vp,
                                vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "misslam_grow_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "misslam_grow": (st, [P(Points), P(Nodes), vp, vp, vp, P(Camera), P(Pose), P(GrowParams), vp, vp,
                          ctypes.c_size_t, vp]),
    "misslam_batch_create": (st, [P(Problem), ctypes.c_int32, P(Params), ctypes.c_int32, P(vp)]),
    "misslam_batch_workspace_bytes": (ctypes.c_size_t, [vp]),
    "misslam_batch_register": (st, [vp, vp, ctypes.c_size_t, vp]),
    "misslam_batch_tile": (ctypes.c_int32, [vp]),
    "misslam_batch_asm_waves": (ctypes.c_int32, [vp]),
    "misslam_probe_mfma_bf16": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int64),
                                                 vp]),
    "misslam_batch_destroy": (None, [vp]),
    "misslam_profile_enable": (ctypes.c_int32, [ctypes.c_int32]),
    "misslam_profile_get": (st, [ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int64)]),
    "misslam_profile_reset": (None, []),
}

_lib = None


def load(path=LIB_PATH):
    """Loads the built library (fails loudly if it is missing) and declares every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1803_02009_amd.build.build() (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MisslamError(RuntimeError):
    def __init__(self, fn, status):
        lib = load()
        msg = lib.misslam_status_string(status).decode()
        extra = f" (hipError {lib.misslam_last_hip_error()})" if status == EHIP else ""
        super().__init__(f"{fn} returned {status}: {msg}{extra}")
        self.status = status


def check(fn, status):
    if status != OK:
        raise MisslamError(fn, status)
