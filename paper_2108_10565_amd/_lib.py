"""ctypes binding of ``libstp.so`` (the C ABI declared in include/stp.h).

Argument marshalling only: every step of the predictor runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.
The binding raises if the library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstp.so")

STP_OK = 0
STATUS_NAMES = {0: "STP_OK", -1: "STP_EINVAL", -2: "STP_EDEGREE", -3: "STP_ENOTUPPER",
                -4: "STP_ESINGULAR", -5: "STP_ENOMEM", -6: "STP_EHIP", -7: "STP_EWORKSPACE",
                -8: "STP_ENONFINITE"}
STP_FP64 = 0
STP_FP32_REFINE = 1
STP_FLAG_REFERENCE_KERNEL = 1
STP_FLAG_MFMA_FLOAT_CHAIN = 2
MAX_DEGREE = 7
EXPORTED = ("stp_create", "stp_destroy", "stp_workspace_size", "stp_predict", "stp_validate",
            "stp_reference_matrices", "stp_flops", "stp_batched_workspace_size",
            "stp_predict_batched", "stp_graph_create", "stp_graph_launch", "stp_graph_destroy",
            "stp_measure_peaks", "stp_static_scratch_bytes", "stp_predict_static",
            "stp_staged_workspace_size", "stp_graph_create_staged",
            "stp_workspace_size_nq", "stp_predict_nq", "stp_validate_nq",
            "stp_basis_eval", "stp_reference_mass", "stp_corrector_tables_size", "stp_corrector_tables",
            "stp_upwind_split", "stp_face_operators", "stp_correct",
            "stp_check_inputs", "stp_status_string", "stp_last_error")


class StpBatch(ctypes.Structure):
    """struct stp_batch of include/stp.h."""
    _fields_ = [("degree", ctypes.c_int), ("n_elements", ctypes.c_int64), ("dt", ctypes.c_double),
                ("star", ctypes.c_void_p), ("E", ctypes.c_void_p), ("Q0", ctypes.c_void_p),
                ("Q", ctypes.c_void_p), ("Qint", ctypes.c_void_p)]


class StpPeaks(ctypes.Structure):
    """struct stp_peaks of include/stp.h."""
    _fields_ = [("fp64_valu_tflops", ctypes.c_double), ("fp32_valu_tflops", ctypes.c_double),
                ("fp64_mfma_tflops", ctypes.c_double), ("hbm_copy_gbs", ctypes.c_double),
                ("hbm_write_gbs", ctypes.c_double)]


_lib = None


class StpError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{name}: {detail}" if detail else name)


def load(path: str = LIB_PATH):
    """Load libstp.so (once) and declare the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python paper_2108_10565_amd/build.py)")
    lib = ctypes.CDLL(path)
    vp, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.stp_create.argtypes = [ctypes.POINTER(vp)]
    lib.stp_destroy.argtypes = [vp]
    lib.stp_workspace_size.argtypes = [vp, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(sz)]
    lib.stp_predict.argtypes = [vp, vp, ctypes.c_int, i64, dbl, vp, vp, vp, vp, vp,
                                ctypes.c_int, ctypes.c_int, vp, sz, ctypes.c_uint]
    lib.stp_validate.argtypes = [vp, vp, ctypes.c_int, i64, dbl, vp, vp, vp]
    lib.stp_check_inputs.argtypes = [vp, vp]
    lib.stp_workspace_size_nq.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(sz)]
    lib.stp_predict_nq.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64, dbl, vp, vp, vp, vp, vp,
                                   ctypes.c_int, ctypes.c_int, vp, sz, ctypes.c_uint]
    lib.stp_validate_nq.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64, dbl, vp, vp, vp]
    lib.stp_basis_eval.argtypes = [ctypes.c_int, i64, vp, vp]
    lib.stp_reference_mass.argtypes = [ctypes.c_int, vp]
    lib.stp_corrector_tables_size.argtypes = [ctypes.c_int]
    lib.stp_corrector_tables_size.restype = sz
    lib.stp_corrector_tables.argtypes = [ctypes.c_int, vp]
    lib.stp_upwind_split.argtypes = [ctypes.c_int, vp, vp, vp]
    lib.stp_face_operators.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, vp]
    lib.stp_correct.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.stp_static_scratch_bytes.argtypes = []
    lib.stp_static_scratch_bytes.restype = sz
    lib.stp_predict_static.argtypes = [vp, vp, ctypes.c_int, i64, dbl, vp, vp, vp, vp, vp,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    lib.stp_reference_matrices.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.stp_flops.argtypes = [ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    pb = ctypes.POINTER(StpBatch)
    lib.stp_batched_workspace_size.argtypes = [vp, ctypes.c_int, pb, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(sz)]
    lib.stp_predict_batched.argtypes = [vp, vp, ctypes.c_int, pb, ctypes.c_int, ctypes.c_int, vp, sz,
                                        ctypes.c_uint]
    lib.stp_graph_create.argtypes = [vp, vp, ctypes.c_int, pb, ctypes.c_int, ctypes.c_int, vp, sz,
                                     ctypes.c_uint, ctypes.POINTER(vp)]
    lib.stp_staged_workspace_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), pb, ctypes.c_int,
                                              ctypes.c_int, ctypes.POINTER(sz)]
    lib.stp_graph_create_staged.argtypes = [vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), pb, ctypes.c_int,
                                            ctypes.c_int, vp, sz, ctypes.c_uint, ctypes.POINTER(vp)]
    lib.stp_graph_launch.argtypes = [vp, vp]
    lib.stp_graph_destroy.argtypes = [vp]
    lib.stp_measure_peaks.argtypes = [vp, vp, vp, sz, ctypes.POINTER(StpPeaks)]
    lib.stp_status_string.argtypes = [ctypes.c_int]
    lib.stp_status_string.restype = ctypes.c_char_p
    lib.stp_last_error.argtypes = [vp]
    lib.stp_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("stp_status_string", "stp_last_error", "stp_static_scratch_bytes",
                        "stp_corrector_tables_size"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class Handle:
    """Owns one stp_handle."""

    def __init__(self):
        self.lib = load()
        self.ptr = ctypes.c_void_p()
        self.check(self.lib.stp_create(ctypes.byref(self.ptr)))

    def check(self, status: int):
        if status != STP_OK:
            detail = self.lib.stp_last_error(self.ptr).decode() if self.ptr else ""
            raise StpError(status, detail)

    def close(self):
        if self.ptr:
            self.lib.stp_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
