"""CPU oracle of noisy mean-field annealing -- TEST INFRASTRUCTURE ONLY.

Python bindings (ctypes) for ``nmfa_oracle.c``, a plain FP64 C implementation of the paper's
noisy mean-field annealing (Sec. II, Alg. 1), its Ising energy (Eq. 1) and a brute-force
ground-state search. Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this package; the GPU library
never does, and this package imports nothing from it.

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):

* ``philox4x32_10``      pinned: published known-answer vectors of Philox4x32-10.
* ``gauss4`` / ``noise`` pinned: Box-Muller invariants (radius^2 = -2 ln u0, angle = 2 pi u1),
                         the normal distribution (moments, Kolmogorov-Smirnov), and the counter
                         mapping (floor(i/4), r, t, 0) / lane i mod 4 rebuilt from the pinned
                         generator (a lane swap, a 0-based t or r and t exchanged fail it).
* ``normalisers``        pinned: closed forms (SK: sqrt(N-1); d-regular: sqrt(d); with fields).
* ``schedule``           pinned: knot values, geometric midpoints, monotonicity.
* ``anneal``             pinned: closed-form geometric series for J = 0, sigma = 0; alpha = 1
                         one-step form; the zero state for sigma = 0, h = 0; exact negation under
                         negated noise; exact invariance under scaling (h, J) by powers of two;
                         replica-prefix invariance; ground states found on small instances.
* ``energy`` / ``energy_int`` / ``cut``  pinned: hand-worked golden examples, flip symmetry,
                         cut = (W - E)/2 identity, pure-Python enumeration.
* ``ground_state``       pinned: pure-Python exhaustive enumeration, the Moebius-ladder closed
                         form, frustrated-triangle and ferromagnet special cases.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nmfa_oracle.c")
_LIB = os.path.join(_HERE, "libnmfa_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no contraction, OpenMP over replicas)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, u32, u64, i64 = (ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_int64)
        vp = ctypes.c_void_p
        L.nmfa_oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.nmfa_oracle_philox4x32_10.restype = None
        L.nmfa_oracle_gauss4.argtypes = [u64, u32, u32, u32, vp]
        L.nmfa_oracle_gauss4.restype = None
        L.nmfa_oracle_noise.argtypes = [u64, i32, i32, i32]
        L.nmfa_oracle_noise.restype = d
        L.nmfa_oracle_normalisers.argtypes = [i32, vp, vp, vp]
        L.nmfa_oracle_normalisers.restype = None
        L.nmfa_oracle_schedule.argtypes = [i32, vp, vp, i32, vp]
        L.nmfa_oracle_schedule.restype = ctypes.c_int
        L.nmfa_oracle_anneal.argtypes = [i32, vp, vp, d, d, vp, i32, i32, i32, vp, u64, i32, vp,
                                         i32, vp, vp, vp, i32]
        L.nmfa_oracle_anneal.restype = ctypes.c_int
        L.nmfa_oracle_energy.argtypes = [i32, vp, vp, vp]
        L.nmfa_oracle_energy.restype = d
        L.nmfa_oracle_energy_int.argtypes = [i32, vp, vp, vp, vp]
        L.nmfa_oracle_energy_int.restype = ctypes.c_int
        L.nmfa_oracle_cut.argtypes = [i32, vp, vp]
        L.nmfa_oracle_cut.restype = d
        L.nmfa_oracle_ground_state.argtypes = [i32, vp, vp, vp]
        L.nmfa_oracle_ground_state.restype = d
        L.nmfa_oracle_num_threads.argtypes = []
        L.nmfa_oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --- noise -----------------------------------------------------------------------------------

def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().nmfa_oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


def gauss4(seed: int, q: int, r: int, t: int) -> np.ndarray:
    z = np.zeros(4)
    lib().nmfa_oracle_gauss4(int(seed), int(q), int(r), int(t), _ptr(z))
    return z


def noise(seed: int, t: int, r: int, i: int) -> float:
    return float(lib().nmfa_oracle_noise(int(seed), int(t), int(r), int(i)))


# --- setup -----------------------------------------------------------------------------------

def normalisers(J: np.ndarray, h: Optional[np.ndarray] = None) -> np.ndarray:
    J = _f64(J)
    n = J.shape[0]
    out = np.zeros(n)
    lib().nmfa_oracle_normalisers(n, _ptr(J), _ptr(None if h is None else _f64(h)), _ptr(out))
    return out


DEFAULT_KNOTS = ((0.0, 10.0), (0.1, 2.0), (0.6, 0.5), (1.0, 0.05))


def schedule(t_f: int, knots=DEFAULT_KNOTS) -> np.ndarray:
    ku = _f64([k[0] for k in knots])
    kT = _f64([k[1] for k in knots])
    out = np.zeros(max(t_f, 1))
    rc = lib().nmfa_oracle_schedule(len(knots), _ptr(ku), _ptr(kT), int(t_f), _ptr(out))
    if rc != 0:
        raise ValueError("invalid schedule knots")
    return out[:t_f]


# --- Algorithm 1 -------------------------------------------------------------------------------

def anneal(J: np.ndarray, h: Optional[np.ndarray], T: np.ndarray, R: int = 1, seed: int = 0,
           alpha: float = 0.15, sigma: float = 0.15, replicas: Optional[Sequence[int]] = None,
           t_first: int = 1, s_init: Optional[np.ndarray] = None, record: int = 0,
           negate_noise: bool = False, threads: int = 0):
    """Run Algorithm 1; returns (spins int8 [R,n], s float64 [R,n], traj float64 [record,R,n])."""
    J = _f64(J)
    n = J.shape[0]
    T = _f64(T)
    t_f = T.shape[0]
    ids = None if replicas is None else np.ascontiguousarray(replicas, dtype=np.int32)
    n_rep = int(R) if ids is None else int(ids.shape[0])
    s_out = np.zeros((n_rep, n))
    spins = np.zeros((n_rep, n), dtype=np.int8)
    traj = np.zeros((record, n_rep, n)) if record > 0 else None
    si = None if s_init is None else _f64(s_init).reshape(n_rep, n)
    rc = lib().nmfa_oracle_anneal(n, _ptr(J), _ptr(None if h is None else _f64(h)), float(alpha),
                                  float(sigma), _ptr(T), t_f, int(t_first), n_rep, _ptr(ids),
                                  int(seed), int(bool(negate_noise)), _ptr(si), int(record),
                                  _ptr(traj), _ptr(s_out), _ptr(spins), int(threads))
    if rc != 0:
        raise ValueError("oracle anneal rejected its arguments")
    return spins, s_out, traj


# --- energies ------------------------------------------------------------------------------------

def energy(J: np.ndarray, h: Optional[np.ndarray], s: np.ndarray) -> float:
    J = _f64(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().nmfa_oracle_energy(J.shape[0], _ptr(J), _ptr(None if h is None else _f64(h)),
                                          _ptr(s)))


def energy_int(J: np.ndarray, h: Optional[np.ndarray], s: np.ndarray) -> int:
    J = _f64(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    E = np.zeros(1, dtype=np.int64)
    rc = lib().nmfa_oracle_energy_int(J.shape[0], _ptr(J), _ptr(None if h is None else _f64(h)),
                                      _ptr(s), _ptr(E))
    if rc != 0:
        raise ValueError("couplings or fields are not integers")
    return int(E[0])


def energies(J: np.ndarray, h: Optional[np.ndarray], spins: np.ndarray) -> np.ndarray:
    return np.array([energy(J, h, row) for row in spins])


def energies_int(J: np.ndarray, h: Optional[np.ndarray], spins: np.ndarray) -> np.ndarray:
    return np.array([energy_int(J, h, row) for row in spins], dtype=np.int64)


def cut(W: np.ndarray, s: np.ndarray) -> float:
    W = _f64(W)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().nmfa_oracle_cut(W.shape[0], _ptr(W), _ptr(s)))


def ground_state(J: np.ndarray, h: Optional[np.ndarray] = None) -> Tuple[float, np.ndarray]:
    J = _f64(J)
    n = J.shape[0]
    best = np.zeros(n, dtype=np.int8)
    E = lib().nmfa_oracle_ground_state(n, _ptr(J), _ptr(None if h is None else _f64(h)), _ptr(best))
    return float(E), best


def num_threads() -> int:
    return int(lib().nmfa_oracle_num_threads())
