"""Python entry points with the same names as the C ABI (include/stp.h)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

_handle = None


def _h():
    global _handle
    if _handle is None:
        _handle = _lib.Handle()
    return _handle


def n_modes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


_PREC = {"fp64": _lib.STP_FP64, "fp32_refine": _lib.STP_FP32_REFINE}


def workspace_size(degree: int, n: int, precision: str = "fp64", refine_steps: int = 1, nq: int = 13) -> int:
    h = _h()
    out = ctypes.c_size_t()
    h.check(h.lib.stp_workspace_size_nq(h.ptr, nq, degree, n, _PREC[precision], refine_steps,
                                        ctypes.byref(out)))
    return out.value


def predict(Q0, star, E, dt: float, degree: int, precision: str = "fp64", refine_steps: int = 1,
            Q=None, Qint=None, with_qint: bool = True, reference_kernel: bool = False,
            stream=None, mfma_float_chain: bool = False, workspace=None):
    """Space-time DOFs Q [n,nq,B,T] and time-integrated DOFs Qint [n,nq,B].

    Q0 [n,nq,B], star [n,3,nq,nq], E [n,nq,nq]: float64, contiguous, on the
    same cuda device; nq = 13 (poroelastic) or 6 (damped Maxwell), taken
    from Q0 (stp_predict_nq).  Outputs are allocated here unless passed in.  The call
    is asynchronous on ``stream`` (default: torch's current stream).
    ``mfma_float_chain`` selects the matrix-core float32 chain
    (STP_FLAG_MFMA_FLOAT_CHAIN) for precision="fp32_refine".  ``workspace``
    (a contiguous uint8 cuda tensor of at least workspace_size() bytes)
    is used instead of allocating one, so that a call with Q, Qint and
    workspace passed in allocates nothing."""
    import torch
    h = _h()
    n = _check_inputs(Q0, star, E, degree)
    nq = int(Q0.shape[1])
    B, T = n_modes(degree), degree + 1
    if Q is None:
        Q = torch.empty((n, nq, B, T), dtype=torch.float64, device=Q0.device)
    if Qint is None and with_qint:
        Qint = torch.empty((n, nq, B), dtype=torch.float64, device=Q0.device)
    if workspace is not None:
        if workspace.dtype != torch.uint8 or not workspace.is_contiguous() or workspace.device != Q0.device:
            raise ValueError("workspace: expected a contiguous uint8 tensor on the device of Q0")
        work, ws = workspace, workspace.numel()
    else:
        ws = workspace_size(degree, n, precision, refine_steps, nq)
        work = torch.empty(ws, dtype=torch.uint8, device=Q0.device) if ws else None
    if stream is None:
        stream = torch.cuda.current_stream(Q0.device)
    flags = (_lib.STP_FLAG_REFERENCE_KERNEL if reference_kernel else 0) | \
        (_lib.STP_FLAG_MFMA_FLOAT_CHAIN if mfma_float_chain else 0)
    h.check(h.lib.stp_predict_nq(h.ptr, ctypes.c_void_p(stream.cuda_stream), nq, degree, n, float(dt),
                                 _ptr(star), _ptr(E), _ptr(Q0), _ptr(Q), _ptr(Qint), _PREC[precision],
                                 refine_steps, _ptr(work), ws, flags))
    return Q, Qint


def static_scratch_bytes() -> int:
    """stp_static_scratch_bytes: size of the library's per-device scratch."""
    return int(_lib.load().stp_static_scratch_bytes())


def predict_static(Q0, star, E, dt: float, degree: int, Q, Qint=None, precision: str = "fp64",
                   refine_steps: int = 1, reference_kernel: bool = False, stream=None):
    """stp_predict_static: as predict(), into the caller's Q (and Qint, may be
    None), with no workspace: the library's per-device scratch is used and
    nothing is allocated here or in the library."""
    import torch
    h = _h()
    n = _check_inputs(Q0, star, E, degree)
    if stream is None:
        stream = torch.cuda.current_stream(Q0.device)
    flags = _lib.STP_FLAG_REFERENCE_KERNEL if reference_kernel else 0
    h.check(h.lib.stp_predict_static(h.ptr, ctypes.c_void_p(stream.cuda_stream), degree, n, float(dt),
                                     _ptr(star), _ptr(E), _ptr(Q0), _ptr(Q), _ptr(Qint), _PREC[precision],
                                     refine_steps, flags))
    return Q, Qint


def _check_inputs(Q0, star, E, degree):
    import torch
    n = int(Q0.shape[0])
    nq = int(Q0.shape[1]) if Q0.dim() == 3 else 13
    B = n_modes(degree)
    for name, t, shape in (("Q0", Q0, (n, nq, B)), ("star", star, (n, 3, nq, nq)), ("E", E, (n, nq, nq))):
        if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: expected contiguous cuda float64 {shape}, got "
                             f"{tuple(t.shape)} {t.dtype} cuda={t.is_cuda}")
    return n


def _batch_array(batches, with_qint=True):
    """Allocates missing outputs and fills a ctypes stp_batch array.

    ``batches``: list of dicts with keys degree, dt, Q0, star, E and
    optionally Q, Qint (outputs written in place)."""
    import torch
    arr = (_lib.StpBatch * max(len(batches), 1))()
    for i, b in enumerate(batches):
        N = int(b["degree"])
        n = _check_inputs(b["Q0"], b["star"], b["E"], N)
        if b["Q0"].shape[1] != 13:
            raise ValueError("batched calls and graphs take the 13-quantity system")
        if b.get("Q") is None:
            b["Q"] = torch.empty((n, 13, n_modes(N), N + 1), dtype=torch.float64, device=b["Q0"].device)
        if b.get("Qint") is None and with_qint:
            b["Qint"] = torch.empty((n, 13, n_modes(N)), dtype=torch.float64, device=b["Q0"].device)
        arr[i] = _lib.StpBatch(N, n, float(b["dt"]), b["star"].data_ptr(), b["E"].data_ptr(),
                               b["Q0"].data_ptr(), b["Q"].data_ptr(),
                               b["Qint"].data_ptr() if b.get("Qint") is not None else 0)
    return arr


def _batched_workspace(arr, count, precision, refine_steps, device):
    import torch
    h = _h()
    out = ctypes.c_size_t()
    h.check(h.lib.stp_batched_workspace_size(h.ptr, count, arr, _PREC[precision], refine_steps,
                                             ctypes.byref(out)))
    return torch.empty(out.value, dtype=torch.uint8, device=device) if out.value else None


def predict_batched(batches, precision: str = "fp64", refine_steps: int = 1, with_qint: bool = True,
                    reference_kernel: bool = False, stream=None):
    """stp_predict_batched: every batch (dict with degree, dt, Q0, star, E and
    optional Q, Qint) predicted in order on one stream; returns the batches
    with their Q and Qint filled in."""
    import torch
    h = _h()
    if not batches:
        return batches
    arr = _batch_array(batches, with_qint)
    dev = batches[0]["Q0"].device
    work = _batched_workspace(arr, len(batches), precision, refine_steps, dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    flags = _lib.STP_FLAG_REFERENCE_KERNEL if reference_kernel else 0
    h.check(h.lib.stp_predict_batched(h.ptr, ctypes.c_void_p(stream.cuda_stream), len(batches), arr,
                                      _PREC[precision], refine_steps, _ptr(work),
                                      work.numel() if work is not None else 0, flags))
    return batches


class Graph:
    """stp_graph_create / stp_graph_launch / stp_graph_destroy: the launches
    of one stp_predict_batched call captured once on ``capture_stream`` (a
    non-default torch stream; a new one if None) and replayed by launch().
    With ``stages`` (list of batch counts, summing to len(batches)),
    stp_graph_create_staged: the batches of one stage run on parallel graph
    branches.  Keeps the batches' tensors and the workspace alive."""

    def __init__(self, batches, precision: str = "fp64", refine_steps: int = 1, with_qint: bool = True,
                 reference_kernel: bool = False, capture_stream=None, stages=None):
        import torch
        self._h = _h()
        self.batches = batches
        self._arr = _batch_array(batches, with_qint)
        dev = batches[0]["Q0"].device if batches else torch.device("cuda")
        flags = _lib.STP_FLAG_REFERENCE_KERNEL if reference_kernel else 0
        self.ptr = ctypes.c_void_p()
        self._stream = capture_stream if capture_stream is not None else torch.cuda.Stream(dev)
        if stages is None:
            self._work = _batched_workspace(self._arr, len(batches), precision, refine_steps, dev)
            torch.cuda.current_stream(dev).synchronize()
            self._h.check(self._h.lib.stp_graph_create(
                self._h.ptr, ctypes.c_void_p(self._stream.cuda_stream), len(batches), self._arr,
                _PREC[precision], refine_steps, _ptr(self._work),
                self._work.numel() if self._work is not None else 0, flags, ctypes.byref(self.ptr)))
        else:
            if sum(stages) != len(batches):
                raise ValueError("stages must sum to the number of batches")
            self._stages = (ctypes.c_int * max(len(stages), 1))(*stages)
            out = ctypes.c_size_t()
            self._h.check(self._h.lib.stp_staged_workspace_size(self._h.ptr, len(stages), self._stages, self._arr,
                                                                _PREC[precision], refine_steps, ctypes.byref(out)))
            self._work = torch.empty(out.value, dtype=torch.uint8, device=dev) if out.value else None
            torch.cuda.current_stream(dev).synchronize()
            self._h.check(self._h.lib.stp_graph_create_staged(
                self._h.ptr, ctypes.c_void_p(self._stream.cuda_stream), len(stages), self._stages, self._arr,
                _PREC[precision], refine_steps, _ptr(self._work), out.value, flags, ctypes.byref(self.ptr)))

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        st = self._h.lib.stp_graph_launch(self.ptr, ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.STP_OK:
            raise _lib.StpError(st, "stp_graph_launch")

    def close(self):
        if self.ptr:
            self._h.lib.stp_graph_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks(scratch_bytes: int = 2 << 30, stream=None) -> dict:
    """stp_measure_peaks: measured FP64/FP32 VALU and FP64 MFMA FMA rates
    (TFLOP/s) and HBM copy / write bandwidth (GB/s) of the current device."""
    import torch
    h = _h()
    scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    out = _lib.StpPeaks()
    h.check(h.lib.stp_measure_peaks(h.ptr, ctypes.c_void_p(stream.cuda_stream), _ptr(scratch), scratch_bytes,
                                    ctypes.byref(out)))
    del scratch
    return {name: getattr(out, name) for name, _ in _lib.StpPeaks._fields_}


def validate(Q0, star, E, dt: float, degree: int, stream=None) -> None:
    """Data checks of stp_validate; raises StpError on failure (synchronises)."""
    import torch
    h = _h()
    if stream is None:
        stream = torch.cuda.current_stream(Q0.device)
    h.check(h.lib.stp_validate_nq(h.ptr, ctypes.c_void_p(stream.cuda_stream), int(Q0.shape[1]), degree,
                                  int(Q0.shape[0]), float(dt), _ptr(star), _ptr(E), _ptr(Q0)))


def check_inputs(stream=None) -> None:
    """stp_check_inputs: takes the device's report of inputs the prediction
    kernels met and could not take (dt E_pp >= 0.5, E not upper triangular)
    since the last check; raises StpError (ESINGULAR / ENOTUPPER) if there
    were any.  Synchronises ``stream`` (default: torch's current stream)."""
    import torch
    h = _h()
    if stream is None:
        stream = torch.cuda.current_stream()
    h.check(h.lib.stp_check_inputs(h.ptr, ctypes.c_void_p(stream.cuda_stream)))


def reference_matrices(degree: int):
    """(Z [T,T], Sinv_w [T], Khat [3,B,B]) as the library computes them (host)."""
    h = _h()
    B, T = n_modes(degree), degree + 1
    Z = np.zeros((T, T)); s = np.zeros(T); K = np.zeros((3, B, B))
    h.check(h.lib.stp_reference_matrices(h.ptr, degree, Z.ctypes.data_as(ctypes.c_void_p),
                                         s.ctypes.data_as(ctypes.c_void_p),
                                         K.ctypes.data_as(ctypes.c_void_p)))
    return Z, s, K


def flops(degree: int):
    """(paper upper bound of Algorithm 3, FLOP executed by the fused kernel) per element."""
    lib = _lib.load()
    a, b = ctypes.c_double(), ctypes.c_double()
    st = lib.stp_flops(degree, ctypes.byref(a), ctypes.byref(b))
    if st != 0:
        raise _lib.StpError(st)
    return a.value, b.value


# ---- corrector (one ADER-DG step) --------------------------------------------

def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def basis_eval(degree: int, xi):
    """stp_basis_eval: basis values [npts, B] at reference points xi [npts, 3]."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.empty((xi.shape[0], n_modes(degree)))
    st = _lib.load().stp_basis_eval(degree, xi.shape[0], _np_ptr(xi), _np_ptr(out))
    if st != 0:
        raise _lib.StpError(st)
    return out


def reference_mass(degree: int):
    out = np.empty(n_modes(degree))
    st = _lib.load().stp_reference_mass(degree, _np_ptr(out))
    if st != 0:
        raise _lib.StpError(st)
    return out


def corrector_tables(degree: int):
    """stp_corrector_tables: (V [3,B,B], Fl [4,B,B], Fn [4,4,6,B,B]) on the host."""
    lib = _lib.load()
    B = n_modes(degree)
    buf = np.empty(lib.stp_corrector_tables_size(degree))
    st = lib.stp_corrector_tables(degree, _np_ptr(buf))
    if st != 0:
        raise _lib.StpError(st)
    return buf


def upwind_split(An):
    An = np.ascontiguousarray(An, dtype=np.float64)
    ap, am = np.empty_like(An), np.empty_like(An)
    st = _lib.load().stp_upwind_split(An.shape[0], _np_ptr(An), _np_ptr(ap), _np_ptr(am))
    if st != 0:
        raise _lib.StpError(st, "stp_upwind_split")
    return ap, am


def face_operators(ABC, vertices):
    """stp_face_operators: (Gp, Gm) [n, 4, nq, nq] from the physical Jacobians
    ABC [n, 3, nq, nq] and the element corners [n, 4, 3] (host arrays)."""
    h = _h()
    ABC = np.ascontiguousarray(ABC, dtype=np.float64)
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    n, nq = ABC.shape[0], ABC.shape[-1]
    Gp = np.empty((n, 4, nq, nq))
    Gm = np.empty((n, 4, nq, nq))
    h.check(h.lib.stp_face_operators(h.ptr, nq, n, _np_ptr(ABC), _np_ptr(v), _np_ptr(Gp), _np_ptr(Gm)))
    return Gp, Gm


def correct(degree: int, tables, star, E, Gp, Gm, neighbor, nb_code, Qint, Q, stream=None):
    """stp_correct on device tensors; Q [n, nq, B] is updated in place."""
    import torch
    h = _h()
    n, nq = int(Q.shape[0]), int(Q.shape[1])
    if stream is None:
        stream = torch.cuda.current_stream(Q.device)
    for name, t, dt in (("neighbor", neighbor, torch.int32), ("nb_code", nb_code, torch.int32)):
        if t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name}: contiguous {dt} expected")
    h.check(h.lib.stp_correct(h.ptr, ctypes.c_void_p(stream.cuda_stream), nq, degree, n, _ptr(tables),
                              _ptr(star), _ptr(E), _ptr(Gp), _ptr(Gm), _ptr(neighbor), _ptr(nb_code),
                              _ptr(Qint), _ptr(Q)))
    return Q
