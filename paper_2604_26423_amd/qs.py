"""Thin Python binding of libqs (include/qs.h): argument marshalling only.

Every function keeps the C name and order of arguments.  Device buffers may be
passed as torch tensors (their data_ptr is used) or as integer addresses;
streams as torch streams, raw hipStream_t integers, or None for the current
torch stream.  A non-OK status raises QSError carrying the status and the
library's message.  The library must have been built (``python -m
paper_2604_26423_amd.build``); if it is missing every call fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

QS_OK, QS_ERR_ARG, QS_ERR_OOM, QS_ERR_HIP, QS_ERR_RANGE, QS_ERR_STATE = range(6)
QS_C64, QS_C128 = 0, 1
QS_SYM = 16          # complement-symmetric layout flag, OR'ed into the precision
QS_MAX_QUBITS_C64, QS_MAX_QUBITS_C128 = 34, 33
(QS_KIND_PASS, QS_KIND_PASS_PHASE, QS_KIND_ADJOINT, QS_KIND_EXPECT, QS_KIND_SAMPLE,
 QS_KIND_ELEMENTWISE, QS_KIND_REDUCE, QS_KIND_SMALL, QS_KIND_TURNAROUND, QS_KIND_HISTOGRAM,
 QS_KIND_COUNT) = range(11)
KIND_NAMES = ["pass", "pass_phase", "adjoint", "expect", "sample", "elementwise", "reduce", "small",
              "turnaround", "histogram"]
# kernel symbol behind each kind (kinds that share a kernel are timed together
# when compared with a profiler's per-kernel statistics)
KIND_KERNEL = {"pass": "pass_kernel", "pass_phase": "pass_kernel", "adjoint": "adjoint_kernel<reverse>",
               "turnaround": "adjoint_kernel<turnaround>", "expect": "expect_kernel",
               "elementwise": "elementwise", "sample": "sample_kernels", "reduce": "reduce_kernels",
               "small": "small_kernels", "histogram": "hist_kernel"}

# every symbol the public headers declare
EXPORTS = ["qs_last_error", "qs_version", "qs_state_bytes", "qs_alloc", "qs_free", "qs_state_ptr",
           "qs_set_stream", "qs_init_plus", "qs_cost_diagonal", "qs_cost_diagonal_sym", "qs_apply_cost_layer", "qs_apply_mixer",
           "qs_forward", "qs_expect", "qs_sample", "qs_cost_histogram", "qs_layout_index", "qs_get_amplitudes",
           "qs_set_amplitudes", "qs_adjoint_grad", "qs_adjoint_grad_store", "qs_adjoint_ckpt_bytes",
           "qs_profile", "qs_profile_read",
           "qs_plan_check", "qs_batch_plan_check", "qs_batch_create", "qs_batch_info", "qs_batch_forward_grad",
           "qs_batch_free", "qs_noise_create", "qs_noise_info", "qs_noise_run", "qs_noise_free",
           "qs_bandwidth_probe", "qs_cost_diagonal_noalloc", "qs_debug_set_cut_mode"]
QS_BATCH_MAX_QUBITS = 30
QS_NOISE_MAX_QUBITS = 12
QS_NOISE_MAX_LAYERS = 4096


class QSCircuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("w_tenths", ctypes.c_void_p)]


(QS_PROBE_READ, QS_PROBE_WRITE, QS_PROBE_COPY, QS_PROBE_UPDATE, QS_PROBE_PHASE, QS_PROBE_TILE,
 QS_PROBE_WINDOW_VALU, QS_PROBE_WINDOW_MFMA) = range(8)
PROBE_KINDS = {"read": QS_PROBE_READ, "write": QS_PROBE_WRITE, "copy": QS_PROBE_COPY, "update": QS_PROBE_UPDATE,
               "phase": QS_PROBE_PHASE, "tile": QS_PROBE_TILE, "window_valu": QS_PROBE_WINDOW_VALU,
               "window_mfma": QS_PROBE_WINDOW_MFMA}
PROBE_WINDOW_U = 0.25   # u = tan(theta / 2) of the window probes
QS_PROBE_NT_LOAD, QS_PROBE_NT_STORE = 1, 2


class QSProbe(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("flags", ctypes.c_int), ("wg_per_cu", ctypes.c_int),
                ("unroll", ctypes.c_int), ("n", ctypes.c_int), ("c", ctypes.c_int), ("q0", ctypes.c_int),
                ("swizzle", ctypes.c_int), ("windows", ctypes.c_int)]


class QSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libqs status {status}: {message}")
        self.status = status


_lib = None
_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)


def lib() -> ctypes.CDLL:
    """Load libqs.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libqs.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_2604_26423_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl, u64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t,
                                  ctypes.c_double, ctypes.c_uint64)
    sig = {
        "qs_last_error": ([], ctypes.c_char_p),
        "qs_version": ([], ctypes.c_char_p),
        "qs_state_bytes": ([i32, i32], sz),
        "qs_alloc": ([i32, i32, vp, sz, vp, ctypes.POINTER(vp)], i32),
        "qs_free": ([vp], i32),
        "qs_state_ptr": ([vp, ctypes.POINTER(vp)], i32),
        "qs_set_stream": ([vp, vp], i32),
        "qs_init_plus": ([vp], i32),
        "qs_cost_diagonal": ([i32, vp, vp, _c_i64_p, _c_i32_p, vp], i32),
        "qs_cost_diagonal_noalloc": ([i32, vp, vp, _c_i64_p, _c_i32_p, vp], i32),
        "qs_cost_diagonal_sym": ([i32, vp, vp, _c_i64_p, _c_i32_p, vp], i32),
        "qs_apply_cost_layer": ([vp, vp, i64, dbl], i32),
        "qs_apply_mixer": ([vp, dbl], i32),
        "qs_forward": ([vp, vp, i64, i32, vp, vp, _c_dbl_p, _c_dbl_p], i32),
        "qs_expect": ([vp, vp, _c_dbl_p, _c_dbl_p], i32),
        "qs_sample": ([vp, u64, i64, vp, i32], i32),
        "qs_cost_histogram": ([vp, vp, i32, vp, i32], i32),
        "qs_layout_index": ([i64], i64),
        "qs_get_amplitudes": ([vp, i64, i64, vp, i32], i32),
        "qs_set_amplitudes": ([vp, i64, i64, vp, i32], i32),
        "qs_adjoint_grad": ([vp, vp, i64, i32, vp, vp, vp, sz, _c_dbl_p, vp, vp], i32),
        "qs_adjoint_grad_store": ([vp, vp, i64, i32, vp, vp, vp, sz, vp, sz, _c_dbl_p, vp, vp], i32),
        "qs_adjoint_ckpt_bytes": ([vp, i32, ctypes.POINTER(sz)], i32),
        "qs_profile": ([vp, i32], i32),
        "qs_profile_read": ([vp, i32, _c_i64_p, _c_dbl_p, _c_dbl_p], i32),
        "qs_plan_check": ([i32, i32, i32, ctypes.c_char_p, sz], i32),
        "qs_debug_set_cut_mode": ([vp, i32], i32),
        "qs_batch_plan_check": ([i32, vp, i32, ctypes.c_char_p, sz], i32),
        "qs_batch_create": ([i32, vp, i32, vp, ctypes.POINTER(vp)], i32),
        "qs_batch_info": ([vp, i32, _c_i64_p, _c_i32_p, ctypes.POINTER(vp), ctypes.POINTER(vp)], i32),
        "qs_batch_forward_grad": ([vp, vp, vp, vp, vp, vp], i32),
        "qs_batch_free": ([vp], i32),
        "qs_noise_create": ([i32, i32, vp, vp, ctypes.POINTER(vp)], i32),
        "qs_noise_info": ([vp, _c_i64_p, _c_i32_p], i32),
        "qs_noise_run": ([vp, i32, vp, vp, dbl, u64, i64, i64, vp, vp, vp, vp], i32),
        "qs_noise_free": ([vp], i32),
        "qs_bandwidth_probe": ([vp, vp, vp, sz, i32, vp, _c_dbl_p, _c_dbl_p], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int) -> None:
    if status != QS_OK:
        raise QSError(status, lib().qs_last_error().decode(errors="replace"))


def _ptr(x) -> Optional[int]:
    """Device address of a torch tensor, an integer address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _f64(a: Sequence[float]) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- wrappers
def qs_last_error() -> str:
    return lib().qs_last_error().decode(errors="replace")


def qs_version() -> str:
    return lib().qs_version().decode()


def qs_state_bytes(n: int, prec: int) -> int:
    return int(lib().qs_state_bytes(n, prec))


def qs_alloc(n: int, prec: int, dev_buf=None, buf_bytes: int = 0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().qs_alloc(n, prec, _ptr(dev_buf), buf_bytes, _stream(stream), ctypes.byref(h)))
    return h


def qs_free(s) -> None:
    _check(lib().qs_free(s))


def qs_state_ptr(s) -> int:
    p = ctypes.c_void_p()
    _check(lib().qs_state_ptr(s, ctypes.byref(p)))
    return int(p.value or 0)


def qs_set_stream(s, stream=None) -> None:
    _check(lib().qs_set_stream(s, _stream(stream)))


def qs_init_plus(s) -> None:
    _check(lib().qs_init_plus(s))


def qs_cost_diagonal(n: int, w_tenths, diag_dev, stream=None) -> tuple:
    """Returns (W_t, C_max in tenths)."""
    w = np.ascontiguousarray(np.asarray(w_tenths, dtype=np.int32))
    W, cm = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().qs_cost_diagonal(n, w.ctypes.data if w.size else None, _ptr(diag_dev), ctypes.byref(W),
                                  ctypes.byref(cm), _stream(stream)))
    return int(W.value), int(cm.value)


def qs_cost_diagonal_noalloc(n: int, w_tenths, diag_dev, stream=None) -> tuple:
    """qs_cost_diagonal with its scratch in the library's static device array
    (no device allocation); returns (W_t, C_max in tenths)."""
    w = np.ascontiguousarray(np.asarray(w_tenths, dtype=np.int32))
    W, cm = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().qs_cost_diagonal_noalloc(n, w.ctypes.data if w.size else None, _ptr(diag_dev), ctypes.byref(W),
                                          ctypes.byref(cm), _stream(stream)))
    return int(W.value), int(cm.value)


def qs_cost_diagonal_sym(n: int, w_tenths, diag_dev, stream=None) -> tuple:
    """Diagonal of the complement-symmetric layout (2^(n-1) entries, z order); returns (W_t, C_max)."""
    w = np.ascontiguousarray(np.asarray(w_tenths, dtype=np.int32))
    W, cm = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().qs_cost_diagonal_sym(n, w.ctypes.data if w.size else None, _ptr(diag_dev), ctypes.byref(W),
                                      ctypes.byref(cm), _stream(stream)))
    return int(W.value), int(cm.value)


def qs_apply_cost_layer(s, diag_dev, w_total_tenths: int, theta_zz: float) -> None:
    _check(lib().qs_apply_cost_layer(s, _ptr(diag_dev), int(w_total_tenths), float(theta_zz)))


def qs_apply_mixer(s, theta_x: float) -> None:
    _check(lib().qs_apply_mixer(s, float(theta_x)))


def qs_forward(s, diag_dev, w_total_tenths: int, theta_zz, theta_x, readout: bool = True):
    """Returns (exp_c, norm) when readout, else None."""
    tzz, tx = _f64(theta_zz), _f64(theta_x)
    if tzz.shape != tx.shape:
        raise ValueError("theta_zz and theta_x must have the same length")
    e, nrm = ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_forward(s, _ptr(diag_dev), int(w_total_tenths), len(tzz),
                            tzz.ctypes.data if len(tzz) else None, tx.ctypes.data if len(tx) else None,
                            ctypes.byref(e) if readout else None, ctypes.byref(nrm) if readout else None))
    return (e.value, nrm.value) if readout else None


def qs_expect(s, diag_dev) -> tuple:
    e, nrm = ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_expect(s, _ptr(diag_dev), ctypes.byref(e), ctypes.byref(nrm)))
    return e.value, nrm.value


def qs_sample(s, seed: int, shots: int, out=None) -> np.ndarray:
    """Shots to a new host array, or into a device tensor `out` (returned)."""
    if out is not None:
        _check(lib().qs_sample(s, int(seed), int(shots), _ptr(out), 1))
        return out
    host = np.empty(int(shots), dtype=np.uint64)
    _check(lib().qs_sample(s, int(seed), int(shots), host.ctypes.data if shots > 0 else None, 0))
    return host


def qs_layout_index(x: int) -> int:
    return int(lib().qs_layout_index(int(x)))


def layout_indices(x):
    """qs_layout_index for an integer array (the formula of include/qs.h)."""
    x = np.asarray(x, dtype=np.int64)
    y = x >> 13
    y = y ^ (y >> 9)
    y = y ^ (y >> 18)
    return x ^ ((y & 511) << 4)


def qs_get_amplitudes(s, first: int, count: int, out=None):
    """Amplitudes [first, first + count) in index order: into a device tensor
    `out` (returned), else a new host array of the state's complex type."""
    if out is not None:
        _check(lib().qs_get_amplitudes(s, int(first), int(count), _ptr(out), 1))
        return out
    raise ValueError("pass a device tensor or use qs_get_amplitudes_host")


def qs_get_amplitudes_host(s, first: int, count: int, dtype) -> np.ndarray:
    host = np.empty(int(count), dtype=dtype)
    _check(lib().qs_get_amplitudes(s, int(first), int(count), host.ctypes.data if count else None, 0))
    return host


def qs_set_amplitudes(s, first: int, src, on_device: bool = True) -> None:
    if on_device:
        _check(lib().qs_set_amplitudes(s, int(first), int(src.numel()), _ptr(src), 1))
    else:
        a = np.ascontiguousarray(src)
        _check(lib().qs_set_amplitudes(s, int(first), int(a.size), a.ctypes.data if a.size else None, 0))


def qs_cost_histogram(s, diag_dev, nbins: int, out=None) -> np.ndarray:
    """Fixed-point mass per cut value (uint64, 2^62 = probability 1), to a new
    host array or into a device tensor `out` (returned)."""
    if out is not None:
        _check(lib().qs_cost_histogram(s, _ptr(diag_dev), int(nbins), _ptr(out), 1))
        return out
    host = np.empty(max(int(nbins), 0), dtype=np.uint64)
    _check(lib().qs_cost_histogram(s, _ptr(diag_dev), int(nbins), host.ctypes.data if nbins > 0 else None, 0))
    return host


def qs_adjoint_grad(s, diag_dev, w_total_tenths: int, theta_zz, theta_x, lambda_buf=None,
                    lambda_bytes: int = 0) -> tuple:
    """Returns (E, dE/dtheta_zz[p], dE/dtheta_x[p])."""
    tzz, tx = _f64(theta_zz), _f64(theta_x)
    if tzz.shape != tx.shape:
        raise ValueError("theta_zz and theta_x must have the same length")
    p = len(tzz)
    gzz, gx, e = np.empty(p), np.empty(p), ctypes.c_double()
    _check(lib().qs_adjoint_grad(s, _ptr(diag_dev), int(w_total_tenths), p,
                                 tzz.ctypes.data if p else None, tx.ctypes.data if p else None,
                                 _ptr(lambda_buf), int(lambda_bytes), ctypes.byref(e),
                                 gzz.ctypes.data if p else None, gx.ctypes.data if p else None))
    return e.value, gzz, gx


def qs_adjoint_grad_store(s, diag_dev, w_total_tenths: int, theta_zz, theta_x, ckpt_buf=None,
                          ckpt_bytes: int = 0, lambda_buf=None, lambda_bytes: int = 0) -> tuple:
    """Store mode of the adjoint (checkpointed psi).  Returns (E, dE/dtheta_zz[p], dE/dtheta_x[p])."""
    tzz, tx = _f64(theta_zz), _f64(theta_x)
    if tzz.shape != tx.shape:
        raise ValueError("theta_zz and theta_x must have the same length")
    p = len(tzz)
    gzz, gx, e = np.empty(p), np.empty(p), ctypes.c_double()
    _check(lib().qs_adjoint_grad_store(s, _ptr(diag_dev), int(w_total_tenths), p,
                                       tzz.ctypes.data if p else None, tx.ctypes.data if p else None,
                                       _ptr(ckpt_buf), int(ckpt_bytes), _ptr(lambda_buf), int(lambda_bytes),
                                       ctypes.byref(e), gzz.ctypes.data if p else None,
                                       gx.ctypes.data if p else None))
    return e.value, gzz, gx


def qs_adjoint_ckpt_bytes(s, p: int) -> int:
    """Checkpoint bytes qs_adjoint_grad_store needs for p layers."""
    b = ctypes.c_size_t()
    _check(lib().qs_adjoint_ckpt_bytes(s, int(p), ctypes.byref(b)))
    return int(b.value)


CUT_MODES = {"auto": 0, "registers": 1, "diagonal": 2}


def qs_debug_set_cut_mode(s, mode) -> None:
    """How the tile passes get C_t: "auto", "registers" or "diagonal" (or 0, 1, 2)."""
    _check(lib().qs_debug_set_cut_mode(s, CUT_MODES[mode] if isinstance(mode, str) else int(mode)))


def qs_profile(s, enable: bool) -> None:
    _check(lib().qs_profile(s, 1 if enable else 0))


def qs_profile_read(s, kind: int) -> tuple:
    """(launches, total_ms, algorithmic bytes) of one kernel kind."""
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_profile_read(s, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return int(n.value), ms.value, by.value


def qs_plan_check(n: int, prec: int, p: int) -> tuple:
    """Host-only check of the pass plan: (code, message); code 0 = valid."""
    buf = ctypes.create_string_buffer(512)
    rc = lib().qs_plan_check(n, prec, p, buf, 512)
    return int(rc), buf.value.decode()


# ---------------------------------------------------------------- batch
def _circuits(circuits):
    keep = [np.ascontiguousarray(np.asarray(w, dtype=np.int32)) for _, _, w in circuits]
    arr = (QSCircuit * len(circuits))()
    for i, ((n, p, _), w) in enumerate(zip(circuits, keep)):
        arr[i].n, arr[i].p, arr[i].w_tenths = int(n), int(p), w.ctypes.data
    return arr, keep


def qs_batch_plan_check(circuits, prec: int) -> tuple:
    """(status, message) of the host-side check of a batch schedule."""
    arr, keep = _circuits(circuits)
    buf = ctypes.create_string_buffer(512)
    rc = lib().qs_batch_plan_check(len(circuits), ctypes.cast(arr, ctypes.c_void_p), int(prec), buf, 512)
    return rc, buf.value.decode()


def qs_batch_create(circuits, prec: int, stream=None) -> ctypes.c_void_p:
    """circuits: sequence of (n, p, w_tenths)."""
    arr = (QSCircuit * len(circuits))()
    keep = []
    for i, (n, p, w) in enumerate(circuits):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.int32))
        keep.append(w)
        arr[i] = QSCircuit(int(n), int(p), w.ctypes.data if w.size else None)
    h = ctypes.c_void_p()
    _check(lib().qs_batch_create(len(circuits), ctypes.cast(arr, ctypes.c_void_p), prec, _stream(stream),
                                 ctypes.byref(h)))
    return h


def qs_batch_info(b, i: int) -> tuple:
    """(W_t, C_max tenths, psi device address, diagonal device address) of circuit i."""
    W, cm, ps, dg = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().qs_batch_info(b, i, ctypes.byref(W), ctypes.byref(cm), ctypes.byref(ps), ctypes.byref(dg)))
    return int(W.value), int(cm.value), int(ps.value or 0), int(dg.value or 0)


def qs_batch_forward_grad(b, theta_zz, theta_x, count: int) -> tuple:
    """Concatenated per-circuit angles -> (exp_c[count], d_theta_zz, d_theta_x)."""
    tzz, tx = _f64(theta_zz), _f64(theta_x)
    if tzz.shape != tx.shape:
        raise ValueError("theta_zz and theta_x must have the same length")
    e = np.empty(count)
    gzz, gx = np.empty_like(tzz), np.empty_like(tx)
    _check(lib().qs_batch_forward_grad(b, tzz.ctypes.data, tx.ctypes.data, e.ctypes.data, gzz.ctypes.data,
                                       gx.ctypes.data))
    return e, gzz, gx


def qs_batch_free(b) -> None:
    _check(lib().qs_batch_free(b))


def qs_noise_create(n: int, prec: int, w_tenths, stream=None) -> ctypes.c_void_p:
    w = np.ascontiguousarray(np.asarray(w_tenths, dtype=np.int32))
    h = ctypes.c_void_p()
    _check(lib().qs_noise_create(int(n), int(prec), w.ctypes.data if w.size else None, _stream(stream),
                                 ctypes.byref(h)))
    return h


def qs_noise_info(h) -> tuple:
    """(W_t, C_max) in tenths."""
    W, cm = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().qs_noise_info(h, ctypes.byref(W), ctypes.byref(cm)))
    return int(W.value), int(cm.value)


def qs_noise_run(h, theta_zz, theta_x, eps: float, seed: int, traj0: int, ntraj: int, exp_c,
                 norm=None, nerr=None, states=None) -> None:
    """Trajectories traj0 .. traj0 + ntraj - 1 into device buffers (torch tensors or addresses)."""
    tzz, tx = _f64(theta_zz), _f64(theta_x)
    if tzz.shape != tx.shape:
        raise ValueError("theta_zz and theta_x must have the same length")
    _check(lib().qs_noise_run(h, len(tzz), tzz.ctypes.data, tx.ctypes.data, float(eps), int(seed), int(traj0),
                              int(ntraj), _ptr(exp_c), _ptr(norm), _ptr(nerr), _ptr(states)))


def qs_noise_free(h) -> None:
    _check(lib().qs_noise_free(h))


def qs_bandwidth_probe(kind: int, a, b=None, nbytes: int = 0, reps: int = 5, flags: int = 0, wg_per_cu: int = 0,
                       unroll: int = 0, n: int = 0, c: int = 0, q0: int = 0, swizzle: int = 1, windows: int = 1,
                       stream=None) -> tuple:
    """(ms per launch, bytes read + written per launch) of a probe kernel (include/qs_probe.h)."""
    pr = QSProbe(int(kind), int(flags), int(wg_per_cu), int(unroll), int(n), int(c), int(q0), int(swizzle),
                 int(windows))
    ms, by = ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_bandwidth_probe(ctypes.byref(pr), _ptr(a), _ptr(b), int(nbytes), int(reps), _stream(stream),
                                    ctypes.byref(ms), ctypes.byref(by)))
    return ms.value, by.value
