"""ctypes binding of libdgd.so (the C interface declared in include/dgd.h).

Argument marshalling only: every step of the method runs in the HIP library.
The library must have been built (``paper_2502_09714_amd.build.build()``);
importing this module on a machine without it raises ImportError.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgd.so")

DGD_OK = 0
STATUS = {0: "DGD_OK", -1: "DGD_EINVAL", -2: "DGD_ENOMEM", -3: "DGD_EDEVICE",
          -4: "DGD_ESTATE", -5: "DGD_ENUMERIC"}
FP64, FP32, BF16 = 0, 1, 2
PREDICT_CK, PREDICT_PICARD = 0, 1

_lib = None

c_dp = ctypes.POINTER(ctypes.c_double)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_i8p = ctypes.POINTER(ctypes.c_int8)
c_ip = ctypes.POINTER(ctypes.c_int)
H = ctypes.c_void_p

_SIGS = {
    "dgd_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(H)]),
    "dgd_destroy": (ctypes.c_int, [H]),
    "dgd_last_error": (ctypes.c_char_p, [H]),
    "dgd_sizes": (ctypes.c_int, [H, c_ip, c_ip, c_ip, c_ip]),
    "dgd_set_mesh": (ctypes.c_int, [H, ctypes.c_int64, c_dp, ctypes.c_int64, c_i64p, c_i8p, c_i64p]),
    "dgd_set_material": (ctypes.c_int, [H, c_dp, c_dp, c_dp, c_dp, c_dp, c_dp]),
    "dgd_set_material_ivm": (ctypes.c_int, [H, c_dp, c_dp, c_dp, c_dp, c_dp]),
    "dgd_set_params": (ctypes.c_int, [H, ctypes.c_double, ctypes.c_double]),
    "dgd_get_quadrature_points": (ctypes.c_int, [H, ctypes.c_int64, ctypes.c_int64, c_dp]),
    "dgd_set_state_from_points": (ctypes.c_int, [H, ctypes.c_int64, ctypes.c_int64, c_dp]),
    "dgd_set_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int]),
    "dgd_get_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int]),
    "dgd_get_point_values": (ctypes.c_int, [H, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int]),
    "dgd_set_time": (ctypes.c_int, [H, ctypes.c_double]),
    "dgd_get_time": (ctypes.c_int, [H, c_dp]),
    "dgd_set_predictor": (ctypes.c_int, [H, ctypes.c_int, ctypes.c_int]),
    "dgd_set_clusters": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_double]),
    "dgd_make_clusters": (ctypes.c_int, [H, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, c_dp]),
    "dgd_step_lts": (ctypes.c_int, [H, ctypes.c_int64]),
    "dgd_set_point_sources": (ctypes.c_int, [H, ctypes.c_int, c_dp, c_dp, c_dp, c_dp, ctypes.c_int]),
    "dgd_set_receivers": (ctypes.c_int, [H, ctypes.c_int, c_dp]),
    "dgd_step": (ctypes.c_int, [H, ctypes.c_int64]),
    "dgd_set_check_interval": (ctypes.c_int, [H, ctypes.c_int64]),
    "dgd_synchronize": (ctypes.c_int, [H]),
    "dgd_get_seismograms": (ctypes.c_int, [H, c_dp, c_i64p]),
    "dgd_num_seismogram_steps": (ctypes.c_int, [H, c_i64p]),
    "dgd_clear_seismograms": (ctypes.c_int, [H]),
    "dgd_energy": (ctypes.c_int, [H, c_dp]),
    "dgd_energy_noalloc": (ctypes.c_int, [H, ctypes.c_void_p]),
    "dgd_wavespeed_change": (ctypes.c_int, [H, c_dp]),
    "dgd_get_time_point_states": (ctypes.c_int, [H, c_dp]),
    "dgd_set_profiling": (ctypes.c_int, [H, ctypes.c_int]),
    "dgd_get_kernel_times": (ctypes.c_int, [H, c_dp, c_i64p]),
    "dgd_adjoint_step": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "dgd_adjoint_step_host": (ctypes.c_int, [H, c_dp, c_dp, c_dp, c_dp]),
    "dgd_forward_checkpointed": (ctypes.c_int, [H, ctypes.c_int64, ctypes.c_int64]),
    "dgd_backward": (ctypes.c_int, [H, c_dp, c_dp, c_dp, c_dp]),
    "dgd_tape_id": (ctypes.c_int, [H, c_i64p]),
    "dgd_release_tape": (ctypes.c_int, [H]),
}
NUM_KERNEL_CLASSES = 10


def lib():
    """Load libdgd.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2502_09714_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class DGDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
