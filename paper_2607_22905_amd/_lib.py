"""ctypes declarations of the C-ABI in include/algmortar.h (marshalling only)."""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ALGMORTAR_LIB", os.path.join(HERE, "libalgmortar.so"))

AM_OK = 0
STATUS_NAMES = {
    0: "AM_OK", -1: "AM_ERR_ARG", -2: "AM_ERR_NOT_SYMMETRIC", -3: "AM_ERR_POSITIVE_COUPLING",
    -4: "AM_ERR_NOT_SPD", -5: "AM_ERR_NO_CONVERGENCE", -6: "AM_ERR_BREAKDOWN", -7: "AM_ERR_HIP",
    -8: "AM_ERR_OOM", -9: "AM_ERR_UNSUPPORTED",
}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
MORTAR = {"interface": 0, "edge": 1}
AM_FLAG_NO_GRAPH = 1
AM_FLAG_SEPARATE_IFACE = 2
AM_FLAG_DENSE_IFACE = 4
AM_FLAG_INEXACT_IFACE = 8
AM_FLAG_BF16_PRODUCTS = 16


class AmCsr(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p), ("col_idx", c_void_p),
                ("val", c_void_p), ("values_on_device", c_int32)]


class AmOptions(ctypes.Structure):
    _fields_ = [("local_prec", c_int32), ("mortar", c_int32), ("max_nrhs", c_int32),
                ("device", c_int32), ("flags", c_uint32)]


class AmInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("converged", c_int32), ("rel_res", c_double),
                ("true_rel_res", c_double), ("solve_ms", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AmFaces(ctypes.Structure):
    _fields_ = [("n_faces", c_int64), ("k", c_void_p), ("l", c_void_p), ("gk", c_void_p),
                ("gl", c_void_p), ("pD", c_void_p)]


class AlgMortarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))


_SIGS = {
    "am_partition_blocks": [c_int32] * 6 + [c_void_p, POINTER(c_int32)],
    "am_partition_bisect": [POINTER(AmCsr), c_int32, c_int32, c_uint64, c_void_p, POINTER(c_int32)],
    "am_structure_sizes": [POINTER(AmCsr), c_void_p, c_int32, c_int32, POINTER(c_int64), POINTER(c_int64)],
    "am_structure": [POINTER(AmCsr), c_void_p, c_int32, c_int32] + [c_void_p] * 6,
    "am_interface_nd": [POINTER(AmCsr), c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                        POINTER(c_int32), POINTER(c_int64)],
    "algmortar_setup": [POINTER(AmCsr), c_void_p, c_int32, POINTER(AmOptions), c_void_p, POINTER(c_void_p)],
    "algmortar_apply": [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p],
    "algmortar_apply_static": [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p],
    "algmortar_local_solve": [c_void_p, c_void_p, c_void_p, c_void_p],
    "algmortar_set_smoother": [c_void_p, c_void_p, c_int32, c_int32, c_void_p],
    "algmortar_set_inexact": [c_void_p, c_double, c_int32],
    "algmortar_update_values": [c_void_p, POINTER(AmCsr), c_void_p],
    "algmortar_pcg": [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_double, c_int32, c_void_p, c_void_p],
    "algmortar_interfaces": [c_void_p] * 7,
    "algmortar_sizes": [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)],
    "algmortar_export_interface": [c_void_p, c_int32, c_void_p],
    "algmortar_export_mbf": [c_void_p, c_int64, c_int32, c_void_p],
    "algmortar_destroy": [c_void_p],
    "am_tpfa_create": [POINTER(AmFaces), c_int64, c_int32, POINTER(c_void_p), POINTER(c_int64)],
    "am_tpfa_pattern": [c_void_p, c_void_p, c_void_p],
    "am_tpfa_assemble": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "algmortar_adjoint_grad": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                               c_void_p, c_void_p, c_void_p, c_void_p],
    "am_tpfa_face_grad": [c_void_p] * 6,
    "am_tpfa_destroy": [c_void_p],
    "algmortar_time_kernel": [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_double)],
    "algmortar_tile_choice": [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_double)],
    "algmortar_pcg_profile": [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_double, c_int32, c_void_p,
                              POINTER(c_double), POINTER(c_int64), c_void_p],
}

_lib = None


def load():
    """Load libalgmortar.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_22905_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int32
    lib.algmortar_last_error.argtypes = [c_void_p]
    lib.algmortar_last_error.restype = c_char_p
    _lib = lib
    return lib


def check(status, handle=None):
    if status != AM_OK:
        msg = load().algmortar_last_error(handle)
        raise AlgMortarError(status, msg.decode() if msg else "")
