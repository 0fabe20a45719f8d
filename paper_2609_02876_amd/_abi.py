"""ctypes mirror of ``include/ensode.h`` and loader of ``libensode.so``.

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing this module does not touch the GPU.
"""
import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libensode.so")

# return codes
ENS_OK, ENS_EINVAL, ENS_EUNSUPPORTED, ENS_ENOSPACE, ENS_EHIP = 0, -1, -2, -3, -4
# lane status
LANE_OK, LANE_MAX_STEPS, LANE_DT_UNDERFLOW, LANE_NONFINITE, LANE_NOSPACE = 0, 1, 2, 3, 4
# systems / methods / dtypes / losses
SYS_LORENZ, SYS_VDP, SYS_ROBERTSON, SYS_HIRES, SYS_LV_UDE, SYS_LINEAR = 1, 2, 3, 4, 5, 6
TSIT5, VERN7, RODAS4, ROS23 = 1, 2, 3, 4
F64, F32 = 1, 2
LOSS_SUMSQ, LOSS_MSE_TARGET, LOSS_COTANGENT = 0, 1, 2
MAX_SAVE = 64

SYSTEMS = {"lorenz": (SYS_LORENZ, 3, 3), "vdp": (SYS_VDP, 2, 1),
           "robertson": (SYS_ROBERTSON, 3, 3), "hires": (SYS_HIRES, 8, 12),
           "ude": (SYS_LV_UDE, 2, 1218),
           "linear": (SYS_LINEAR, 2, 2)}
METHODS = {"tsit5": TSIT5, "vern7": VERN7, "rodas4": RODAS4, "ros23": ROS23}


class Problem(C.Structure):
    _fields_ = [("system", C.c_int32), ("method", C.c_int32), ("dtype", C.c_int32),
                ("dim", C.c_int32), ("nparams", C.c_int32), ("params_shared", C.c_int32)]


class Ivp(C.Structure):
    _fields_ = [("n", C.c_int64), ("y0", C.c_void_p), ("params", C.c_void_p),
                ("t0", C.c_double), ("t1", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("h0", C.c_double), ("max_steps", C.c_int64),
                ("n_save", C.c_int32), ("save_times", C.POINTER(C.c_double)),
                ("dense", C.c_int32)]


class TapeCfg(C.Structure):
    _fields_ = [("pool", C.c_void_p), ("pool_bytes", C.c_size_t), ("ckpt_every", C.c_int32),
                ("steps_per_traj", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("n", C.c_int64),
                ("system", C.c_int32), ("method", C.c_int32), ("dtype", C.c_int32),
                ("dim", C.c_int32), ("nparams", C.c_int32), ("params_shared", C.c_int32),
                ("n_save", C.c_int32), ("page_steps", C.c_int32), ("rec_bytes", C.c_int32),
                ("n_pages", C.c_int64), ("page_bytes", C.c_int64),
                ("static_pages", C.c_int32), ("ckpt_every", C.c_int32),
                ("t0", C.c_double), ("t1", C.c_double),
                ("pool", C.c_void_p), ("pool_bytes", C.c_size_t),
                ("steps", C.c_void_p), ("n_trial", C.c_void_p), ("first_page", C.c_void_p),
                ("last_page", C.c_void_p), ("status", C.c_void_p), ("save_idx", C.c_void_p),
                ("save_dt", C.c_void_p), ("save_times", C.c_void_p), ("y_final", C.c_void_p),
                ("links", C.c_void_p), ("counters", C.c_void_p), ("pages", C.c_void_p),
                ("save_base", C.c_void_p), ("dense", C.c_int32), ("save_base_hi", C.c_void_p),
                ("save_h", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("overflow_pages_used", C.c_ulonglong), ("steps_accepted", C.c_ulonglong),
                ("trials", C.c_ulonglong), ("side_steps", C.c_ulonglong)]


class Loss(C.Structure):
    _fields_ = [("kind", C.c_int32), ("data", C.c_void_p), ("scale", C.c_double)]


class Job(C.Structure):
    _fields_ = [("prob", Problem), ("ivp", Ivp), ("loss", Loss), ("steps_hint", C.c_int64),
                ("y_save", C.c_void_p), ("lane_status", C.c_void_p), ("grad_params", C.c_void_p),
                ("grad_y0", C.c_void_p), ("loss_out", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("retried", C.c_int64), ("running", C.c_int64), ("waiting", C.c_int64),
                ("lanes_completed", C.c_int64), ("p50_latency_s", C.c_double),
                ("p99_latency_s", C.c_double), ("mean_latency_s", C.c_double),
                ("busy_s", C.c_double), ("throughput", C.c_double),
                ("pool_in_use", C.c_size_t), ("pool_peak", C.c_size_t),
                ("pool_arena", C.c_size_t)]


JOB_WAITING, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, -1

STATIC_WORKSPACE_BYTES = 64 << 20   # ENS_STATIC_WORKSPACE_BYTES

EXPORTS = ("ensemble_solve", "ensemble_record_bytes", "ensemble_record",
           "ensemble_replay_mesh", "ensemble_refresh", "ensemble_mesh_export",
           "ensemble_adjoint", "ensemble_adjoint_static",
           "ensemble_adjoint_workspace_bytes", "ensemble_jvp", "ensemble_system_register",
           "ensemble_record_stats",
           "ensemble_server_create", "ensemble_server_submit", "ensemble_server_progress",
           "ensemble_server_poll", "ensemble_server_wait", "ensemble_server_drain",
           "ensemble_server_stats", "ensemble_server_destroy",
           "ensemble_last_error")

_lib = None


def load(build_if_missing=True):
    """Load the in-tree HIP library (building it once if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIB_PATH} is not built")
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P, V, Ptr = C.POINTER(Problem), C.POINTER(Ivp), C.c_void_p
    lib.ensemble_solve.argtypes = [P, V, Ptr, Ptr, Ptr]
    lib.ensemble_record_bytes.argtypes = [P, V, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
    lib.ensemble_record.argtypes = [P, V, C.POINTER(TapeCfg), C.POINTER(Record), Ptr, Ptr, Ptr]
    lib.ensemble_replay_mesh.argtypes = [P, V, C.POINTER(TapeCfg), Ptr, Ptr, C.c_int64,
                                         C.POINTER(Record), Ptr, Ptr, Ptr]
    lib.ensemble_refresh.argtypes = [P, V, C.POINTER(TapeCfg), Ptr, Ptr, C.c_int64, C.c_double,
                                     C.POINTER(Record), Ptr, Ptr, Ptr, Ptr]
    lib.ensemble_mesh_export.argtypes = [C.POINTER(Record), Ptr, Ptr, C.c_int64, Ptr]
    lib.ensemble_adjoint.argtypes = [P, V, C.POINTER(Record), C.POINTER(Loss), Ptr, Ptr, Ptr,
                                     Ptr, C.c_size_t, Ptr]
    lib.ensemble_adjoint_static.argtypes = [P, V, C.POINTER(Record), C.POINTER(Loss), Ptr, Ptr,
                                            Ptr, Ptr]
    lib.ensemble_adjoint_workspace_bytes.argtypes = [C.POINTER(Record), C.POINTER(C.c_size_t)]
    lib.ensemble_jvp.argtypes = [P, V, C.POINTER(Record), Ptr, Ptr, C.POINTER(Loss), Ptr, Ptr,
                                 Ptr]
    lib.ensemble_system_register.argtypes = [C.c_char_p, C.c_int32, C.c_int32, C.c_int32,
                                             C.POINTER(C.c_int32)]
    lib.ensemble_record_stats.argtypes = [C.POINTER(Record), C.POINTER(Stats), Ptr]
    S = C.c_void_p
    lib.ensemble_server_create.argtypes = [Ptr, C.c_size_t, C.c_int32, C.POINTER(S)]
    lib.ensemble_server_submit.argtypes = [S, C.POINTER(Job), C.POINTER(C.c_int64)]
    lib.ensemble_server_progress.argtypes = [S, C.POINTER(C.c_int32)]
    lib.ensemble_server_poll.argtypes = [S, C.c_int64, C.POINTER(C.c_int32)]
    lib.ensemble_server_wait.argtypes = [S, C.c_int64]
    lib.ensemble_server_drain.argtypes = [S]
    lib.ensemble_server_stats.argtypes = [S, C.POINTER(ServerStats)]
    lib.ensemble_server_destroy.argtypes = [S]
    lib.ensemble_last_error.argtypes = []
    lib.ensemble_last_error.restype = C.c_char_p
    for f in EXPORTS[:-1]:
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class EnsembleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ensode error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != ENS_OK:
        raise EnsembleError(rc, load().ensemble_last_error().decode())
    return rc
