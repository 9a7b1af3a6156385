"""ctypes declarations of the librf C ABI (include/rf.h)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librf.so")

RF_OK = 0
RF_EINVAL = -1
RF_ESHAPE = -2
RF_ERANGE = -3
RF_EWORKSPACE = -4
RF_EHIP = -5
RF_EUNSUPPORTED = -6
RF_CF32 = 0
RF_CF16 = 1
RF_OP_IMAGE = 1
RF_OP_SEARCH = 2
RF_OP_SEGMENT = 3
RF_OP_SEGMENT_STEPS = 4

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_dp = ctypes.POINTER(ctypes.c_double)
c_ip = ctypes.POINTER(ctypes.c_int32)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("nint", c_i32), ("nbl", c_i32), ("nchan", c_i32), ("npol", c_i32),
        ("vis_dtype", c_i32),
        ("tint_s", ctypes.c_double),
        ("freq_ghz", c_dp), ("uvw_m", c_dp), ("dm", c_dp),
        ("ndm", c_i32),
        ("width", c_ip),
        ("nwidth", c_i32),
        ("npix", c_i32),
        ("du", ctypes.c_double), ("dv", ctypes.c_double), ("kdm", ctypes.c_double),
        ("threshold", ctypes.c_float),
        ("t_begin", c_i32), ("t_end", c_i32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_images", c_i64), ("n_valid", c_i32), ("n_dropped", c_i32), ("n_cells", c_i32),
        ("n_rows", c_i32), ("max_delay", c_i32), ("npix", c_i32), ("table_bytes", c_size),
        ("lanes", c_i32), ("m_budget_mb", c_i32),
    ]


class ImageTag(ctypes.Structure):
    _fields_ = [("dm_idx", c_i32), ("width_idx", c_i32), ("t_int", c_i32)]


class ImageStats(ctypes.Structure):
    _fields_ = [("peak", ctypes.c_float), ("sigma", ctypes.c_float), ("snr", ctypes.c_float),
                ("x", c_i32), ("y", c_i32)]


class Candidate(ctypes.Structure):
    _fields_ = [("dm_idx", c_i32), ("width_idx", c_i32), ("t_int", c_i32), ("x", c_i32),
                ("y", c_i32), ("snr", ctypes.c_float), ("peak", ctypes.c_float),
                ("sigma", ctypes.c_float)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("concurrent", c_i32), ("sample", c_i32), ("ms", ctypes.c_double * 8),
                ("launches", c_i64 * 8)]


KERNEL_KINDS = ["drs", "rows", "cols", "select", "fallback", "grid"]


class ServeTimes(ctypes.Structure):
    _fields_ = [("released_s", ctypes.c_double), ("started_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("latency_s", ctypes.c_double)]

class Mock(ctypes.Structure):
    _fields_ = [("dm", ctypes.c_double), ("t0", ctypes.c_double), ("width", ctypes.c_double),
                ("l", ctypes.c_double), ("m", ctypes.c_double), ("amp", ctypes.c_double)]


assert ctypes.sizeof(Mock) == 48
assert ctypes.sizeof(Candidate) == 32
assert ctypes.sizeof(ImageStats) == 20
assert ctypes.sizeof(ImageTag) == 12

# name -> (restype, argtypes)
SIGNATURES = {
    "rf_status_string": (ctypes.c_char_p, [c_i32]),
    "rf_plan_table_bytes": (c_i32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(c_size)]),
    "rf_plan_create": (c_i32, [ctypes.POINTER(PlanDesc), c_vp, c_size, c_vp, ctypes.POINTER(c_vp)]),
    "rf_plan_destroy": (c_i32, [c_vp]),
    "rf_plan_query": (c_i32, [c_vp, ctypes.POINTER(PlanInfo)]),
    "rf_get_delays": (c_i32, [c_vp, c_vp]),
    "rf_get_cells": (c_i32, [c_vp, c_vp]),
    "rf_workspace_bytes": (c_i32, [c_vp, c_i32, c_i64, ctypes.POINTER(c_size)]),
    "rf_dedisperse": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "rf_resample": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_vp, c_vp]),
    "rf_grid": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp]),
    "rf_image": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_size, c_vp]),
    "rf_image_static": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp]),
    "rf_image_static_max_bytes": (c_i32, [ctypes.POINTER(c_size)]),
    "rf_search": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_size, c_vp]),
    "rf_search_segment": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rf_search_segment_begin": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_size, c_vp,
                                        ctypes.POINTER(c_vp)]),
    "rf_search_segment_end": (c_i32, [c_vp]),
    "rf_search_segment_steps": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rf_search_segment_profile": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_size, c_vp,
                                          ctypes.POINTER(KernelTimes)]),
    "rf_server_request_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_size)]),
    "rf_server_create": (c_i32, [c_vp, c_size, c_i32, ctypes.POINTER(c_vp)]),
    "rf_server_submit": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, ctypes.POINTER(c_i64)]),
    "rf_server_wait": (c_i32, [c_vp, c_i64, c_vp, c_i32, ctypes.POINTER(c_i32),
                               ctypes.POINTER(ServeTimes)]),
    "rf_server_destroy": (c_i32, [c_vp]),
    "rf_plan_set_tuning": (c_i32, [c_vp, c_i32, c_i32]),
    "rf_subtract_mean": (c_i32, [c_vp, c_vp, c_vp]),
    "rf_inject": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_vp, c_vp]),
    "rf_noise": (c_i32, [c_vp, ctypes.c_uint64, ctypes.c_uint32, c_i64, c_vp, c_vp]),
    "rf_periodic_workspace_bytes": (c_i32, [c_vp, ctypes.POINTER(c_size)]),
    "rf_search_periodic": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rf_products_workspace_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_size)]),
    "rf_candidate_products": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp,
                                      c_size, c_vp]),
    "rf_select_tier": (c_i32, [c_vp, c_i32, ctypes.c_float, c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "rf_batch_workspace_bytes": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_size)]),
    "rf_batch_create": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_size, c_i32,
                                ctypes.POINTER(c_vp)]),
    "rf_batch_graph_nodes": (c_i32, [c_vp, ctypes.POINTER(c_size)]),
    "rf_batch_run": (c_i32, [c_vp, c_vp]),
    "rf_batch_destroy": (c_i32, [c_vp]),
}

_lib = None


class RFError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def load():
    """Load librf.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1802_03084_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(status):
    try:
        return load().rf_status_string(status).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "status"


def check(status, where):
    if status != RF_OK:
        raise RFError(status, where)
