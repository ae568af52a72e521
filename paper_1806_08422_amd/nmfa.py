"""Thin Python binding of libnmfa.so (the C ABI declared in include/nmfa.h).

Argument marshalling only: every step of the annealing runs in the library's HIP kernels. The
library must have been built (``python -m paper_1806_08422_amd.build``); if it is missing or
cannot be loaded, importing this module raises -- there is no CPU fallback.

PyTorch, when present, is used only to pick up the current HIP stream (``stream=None``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnmfa.so")

NMFA_OK = 0
NMFA_EINVAL = -1
NMFA_ENOMEM = -2
NMFA_EDEVICE = -3
NMFA_ESTATE = -4
NMFA_ECANCELED = -5

FP64, FP32, BF16, FP8J_BF16S, FP8J_FP8S = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp8j_bf16s": FP8J_BF16S, "fp8j_fp8s": FP8J_FP8S}

FLAG_NEGATE_NOISE = 0x1
FLAG_UPPER_TRIANGULAR = 0x2
FLAG_FORCE_STEP = 0x4
FLAG_FORCE_XCD = 0x8
FLAG_FORCE_FENCED = 0x10
FLAG_FORCE_LDS_J = 0x20
FLAG_FORCE_SPARSE = 0x40
FLAG_SPARSE_GENERIC = 0x80
PATHS = ("persistent", "step", "xcd", "xcd_fenced", "xcd_rj", "xcd_rj_fenced", "sparse", "sparse_rq")
J_FORMATS = ("bf16", "fp8_e4m3", "fp4_e2m1", "native", "ell")

# Every function declared in include/nmfa.h (checked by the CPU tests against the header).
EXPORTS = (
    "nmfa_params_default", "nmfa_create", "nmfa_anneal", "nmfa_anneal_range", "nmfa_spins",
    "nmfa_energies", "nmfa_cuts", "nmfa_energies_of", "nmfa_energies_of_noalloc", "nmfa_get_state", "nmfa_set_state",
    "nmfa_trajectory", "nmfa_info", "nmfa_j_format", "nmfa_last_timing", "nmfa_debug_raise_abort",
    "nmfa_destroy", "nmfa_noise_words",
    "nmfa_noise_values", "nmfa_last_error", "nmfa_server_params_default", "nmfa_server_create",
    "nmfa_server_submit", "nmfa_server_poll", "nmfa_server_wait", "nmfa_server_result",
    "nmfa_server_release", "nmfa_server_cancel", "nmfa_server_stats_get", "nmfa_server_destroy",
)

JOB_QUEUED, JOB_RUNNING, JOB_DONE = 0, 1, 2


class NmfaError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_uint32),
        ("alpha", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("n_knots", ctypes.c_int32),
        ("knot_u", ctypes.POINTER(ctypes.c_double)),
        ("knot_T", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_uint32),
        ("record_iters", ctypes.c_int32),
        ("n_T_explicit", ctypes.c_int32),
        ("T_explicit", ctypes.POINTER(ctypes.c_double)),
    ]


class ServerParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_uint32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_active", ctypes.c_int32),
        ("chunk_iters", ctypes.c_int32),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "completed", "failed", "cancelled", "queued", "active", "bytes_in_use",
        "peak_bytes", "rounds", "batched_launches")]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first (python -m paper_1806_08422_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, u64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "nmfa_params_default": ([ctypes.POINTER(Params)], None),
        "nmfa_create": ([i32, vp, vp, ctypes.POINTER(Params), ctypes.POINTER(vp)], ctypes.c_int),
        "nmfa_anneal": ([vp, i32, i32, u64, vp], ctypes.c_int),
        "nmfa_anneal_range": ([vp, i32, i32, i32, i32, u64, vp], ctypes.c_int),
        "nmfa_spins": ([vp, vp, i32], ctypes.c_int),
        "nmfa_energies": ([vp, vp, vp], ctypes.c_int),
        "nmfa_cuts": ([vp, vp], ctypes.c_int),
        "nmfa_energies_of": ([vp, i32, vp, vp, vp], ctypes.c_int),
        "nmfa_energies_of_noalloc": ([vp, i32, vp, vp, vp, vp], ctypes.c_int),
        "nmfa_get_state": ([vp, vp], ctypes.c_int),
        "nmfa_set_state": ([vp, i32, vp], ctypes.c_int),
        "nmfa_trajectory": ([vp, vp], ctypes.c_int),
        "nmfa_info": ([vp, vp, vp, vp], ctypes.c_int),
        "nmfa_j_format": ([vp, vp], ctypes.c_int),
        "nmfa_last_timing": ([vp, vp, vp, vp], ctypes.c_int),
        "nmfa_debug_raise_abort": ([vp], ctypes.c_int),
        "nmfa_destroy": ([vp], None),
        "nmfa_noise_words": ([u64, i32, i32, i32, i32, vp], ctypes.c_int),
        "nmfa_noise_values": ([u64, i32, i32, i32, i32, i32, vp], ctypes.c_int),
        "nmfa_last_error": ([], ctypes.c_char_p),
        "nmfa_server_params_default": ([ctypes.POINTER(ServerParams)], None),
        "nmfa_server_create": ([ctypes.POINTER(ServerParams), ctypes.POINTER(vp)], ctypes.c_int),
        "nmfa_server_submit": ([vp, i32, vp, vp, i32, i32, u64, ctypes.POINTER(u64)], ctypes.c_int),
        "nmfa_server_poll": ([vp, u64, ctypes.POINTER(i32)], ctypes.c_int),
        "nmfa_server_wait": ([vp, u64, i32], ctypes.c_int),
        "nmfa_server_result": ([vp, u64, vp, vp, vp, vp], ctypes.c_int),
        "nmfa_server_release": ([vp, u64], ctypes.c_int),
        "nmfa_server_cancel": ([vp, u64], ctypes.c_int),
        "nmfa_server_stats_get": ([vp, ctypes.POINTER(ServerStats)], ctypes.c_int),
        "nmfa_server_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def _check(rc: int) -> None:
    if rc != NMFA_OK:
        raise NmfaError(rc, lib.nmfa_last_error().decode(errors="replace"))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def current_stream_handle() -> Optional[int]:
    """The raw hipStream_t of torch's current stream, or None (the null stream)."""
    try:
        import torch

        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Solver:
    """One Ising instance (h, J) prepared on the current GPU; see nmfa_create in include/nmfa.h."""

    def __init__(self, J: np.ndarray, h: Optional[np.ndarray] = None, precision="bf16",
                 alpha: float = 0.15, sigma: float = 0.15,
                 knots: Optional[Sequence[Tuple[float, float]]] = None, record_iters: int = 0,
                 temperatures: Optional[Sequence[float]] = None,
                 negate_noise: bool = False, upper_triangular: bool = False,
                 force_step: bool = False, force_xcd: bool = False, force_fenced: bool = False,
                 force_lds_j: bool = False, force_sparse: bool = False, sparse_generic: bool = False):
        J = np.ascontiguousarray(J, dtype=np.float64)
        if J.ndim != 2 or J.shape[0] != J.shape[1]:
            raise ValueError("J must be a square matrix")
        self.n = int(J.shape[0])
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
        p = Params()
        lib.nmfa_params_default(ctypes.byref(p))
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p.alpha = float(alpha)
        p.sigma = float(sigma)
        p.record_iters = int(record_iters)
        flags = 0
        if negate_noise:
            flags |= FLAG_NEGATE_NOISE
        if upper_triangular:
            flags |= FLAG_UPPER_TRIANGULAR
        if force_step:
            flags |= FLAG_FORCE_STEP
        if force_xcd:
            flags |= FLAG_FORCE_XCD
        if force_fenced:
            flags |= FLAG_FORCE_FENCED
        if force_lds_j:
            flags |= FLAG_FORCE_LDS_J
        if force_sparse:
            flags |= FLAG_FORCE_SPARSE
        if sparse_generic:
            flags |= FLAG_SPARSE_GENERIC
        p.flags = flags
        if knots is not None:
            ku = np.ascontiguousarray([k[0] for k in knots], dtype=np.float64)
            kT = np.ascontiguousarray([k[1] for k in knots], dtype=np.float64)
            p.n_knots = len(knots)
            p.knot_u = ku.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            p.knot_T = kT.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if temperatures is not None:
            Tx = np.ascontiguousarray(temperatures, dtype=np.float64)
            p.n_T_explicit = int(Tx.shape[0])
            p.T_explicit = Tx.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        handle = ctypes.c_void_p()
        _check(lib.nmfa_create(self.n, _ptr(J), _ptr(hh), ctypes.byref(p), ctypes.byref(handle)))
        self._h = handle
        self.R = 0
        self.record_iters = int(record_iters)
        self._iters_last = 0

    # -- lifecycle ---------------------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.nmfa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- annealing ----------------------------------------------------------------------------
    def anneal(self, R: int, t_f: int, seed: int, stream: Optional[int] = None) -> None:
        self.anneal_range(R, t_f, 1, t_f, seed, stream)

    def anneal_range(self, R: int, t_f: int, t_begin: int, t_end: int, seed: int,
                     stream: Optional[int] = None) -> None:
        st = current_stream_handle() if stream is None else stream
        _check(lib.nmfa_anneal_range(self._h, int(R), int(t_f), int(t_begin), int(t_end),
                                     int(seed) & (2**64 - 1), st))
        self.R = int(R)
        self._iters_last = int(t_end) - int(t_begin) + 1

    # -- results ------------------------------------------------------------------------------
    def spins(self) -> np.ndarray:
        out = np.zeros((self.R, self.n), dtype=np.int8)
        _check(lib.nmfa_spins(self._h, _ptr(out), 0))
        return out

    def spins_to_device(self, device_ptr: int) -> None:
        _check(lib.nmfa_spins(self._h, ctypes.c_void_p(device_ptr), 1))

    def energies(self) -> Tuple[np.ndarray, np.ndarray]:
        E = np.zeros(self.R)
        Ei = np.zeros(self.R, dtype=np.int64)
        _check(lib.nmfa_energies(self._h, _ptr(E), _ptr(Ei)))
        return E, Ei

    def cuts(self) -> np.ndarray:
        out = np.zeros(self.R)
        _check(lib.nmfa_cuts(self._h, _ptr(out)))
        return out

    def energies_of(self, spins: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        s = np.ascontiguousarray(spins, dtype=np.int8)
        R = int(s.shape[0])
        E = np.zeros(R)
        Ei = np.zeros(R, dtype=np.int64)
        _check(lib.nmfa_energies_of(self._h, R, _ptr(s), _ptr(E), _ptr(Ei)))
        return E, Ei

    def energies_of_noalloc(self, R: int, spins_ptr: int, E_ptr: int, E_int_ptr: Optional[int] = None,
                            stream: Optional[int] = None) -> None:
        """nmfa_energies_of_noalloc on device buffers (addresses as ints); asynchronous on stream."""
        st = current_stream_handle() if stream is None else stream
        _check(lib.nmfa_energies_of_noalloc(self._h, int(R), ctypes.c_void_p(spins_ptr), ctypes.c_void_p(E_ptr),
                                            ctypes.c_void_p(E_int_ptr) if E_int_ptr else None,
                                            ctypes.c_void_p(st) if st else None))

    def state(self) -> np.ndarray:
        out = np.zeros((self.R, self.n))
        _check(lib.nmfa_get_state(self._h, _ptr(out)))
        return out

    def set_state(self, s: np.ndarray) -> None:
        s = np.ascontiguousarray(s, dtype=np.float64)
        _check(lib.nmfa_set_state(self._h, int(s.shape[0]), _ptr(s)))
        self.R = int(s.shape[0])

    def trajectory(self) -> np.ndarray:
        k = min(self.record_iters, self._iters_last)
        out = np.zeros((k, self.R, self.n))
        _check(lib.nmfa_trajectory(self._h, _ptr(out)))
        return out

    def info(self) -> dict:
        n, p, path = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.nmfa_info(self._h, ctypes.byref(n), ctypes.byref(p), ctypes.byref(path)))
        f = ctypes.c_int32()
        _check(lib.nmfa_j_format(self._h, ctypes.byref(f)))
        return {"n": n.value, "precision": p.value, "path": PATHS[path.value], "j_format": J_FORMATS[f.value]}

    def debug_raise_abort(self) -> None:
        """Test hook: set the group kernels' abort word (see nmfa_debug_raise_abort)."""
        _check(lib.nmfa_debug_raise_abort(self._h))

    def last_timing(self) -> dict:
        a, t, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(lib.nmfa_last_timing(self._h, ctypes.byref(a), ctypes.byref(t), ctypes.byref(n)))
        return {"anneal_ms": float(a.value), "total_ms": float(t.value), "launches": int(n.value)}


def noise_words(seed: int, t: int, r0: int, n_rep: int, n_quads: int) -> np.ndarray:
    out = np.zeros((n_rep, n_quads, 4), dtype=np.uint32)
    _check(lib.nmfa_noise_words(int(seed), int(t), int(r0), int(n_rep), int(n_quads), _ptr(out)))
    return out


def noise_values(seed: int, t: int, r0: int, n_rep: int, n_quads: int, fp64: bool) -> np.ndarray:
    """Standard normal numbers z(t, r0+k, 4q+w) as [n_rep, 4*n_quads] (spin index last)."""
    out = np.zeros((n_rep, n_quads * 4))
    _check(lib.nmfa_noise_values(int(seed), int(t), int(r0), int(n_rep), int(n_quads),
                                 int(bool(fp64)), _ptr(out)))
    return out


class Server:
    """Continuous-batching annealing server (nmfa_server_* in include/nmfa.h)."""

    def __init__(self, precision="bf16", hbm_budget_bytes: int = 8 << 30, max_active: int = 256,
                 chunk_iters: int = 250):
        p = ServerParams()
        lib.nmfa_server_params_default(ctypes.byref(p))
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p.hbm_budget_bytes = int(hbm_budget_bytes)
        p.max_active = int(max_active)
        p.chunk_iters = int(chunk_iters)
        h = ctypes.c_void_p()
        _check(lib.nmfa_server_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._meta = {}

    def submit(self, J: np.ndarray, h: Optional[np.ndarray], R: int, t_f: int, seed: int) -> int:
        J = np.ascontiguousarray(J, dtype=np.float64)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
        t = ctypes.c_uint64()
        _check(lib.nmfa_server_submit(self._h, int(J.shape[0]), _ptr(J), _ptr(hh), int(R), int(t_f),
                                      int(seed) & (2**64 - 1), ctypes.byref(t)))
        self._meta[t.value] = (int(J.shape[0]), int(R))
        return int(t.value)

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32()
        _check(lib.nmfa_server_poll(self._h, int(ticket), ctypes.byref(st)))
        return int(st.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        rc = lib.nmfa_server_wait(self._h, int(ticket), int(timeout_ms))
        if rc == NMFA_ESTATE:
            return False
        _check(rc)
        return True

    def result(self, ticket: int, spins: bool = False):
        n, R = self._meta[int(ticket)]
        E = np.zeros(R)
        Ei = np.zeros(R, dtype=np.int64)
        sp = np.zeros((R, n), dtype=np.int8) if spins else None
        lat = ctypes.c_double()
        _check(lib.nmfa_server_result(self._h, int(ticket), _ptr(E), _ptr(Ei), _ptr(sp), ctypes.byref(lat)))
        return {"E": E, "E_int": Ei, "spins": sp, "latency_ms": float(lat.value)}

    def release(self, ticket: int) -> None:
        _check(lib.nmfa_server_release(self._h, int(ticket)))
        self._meta.pop(int(ticket), None)

    def cancel(self, ticket: int) -> None:
        _check(lib.nmfa_server_cancel(self._h, int(ticket)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.nmfa_server_stats_get(self._h, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.nmfa_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
