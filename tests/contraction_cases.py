"""Seeded inputs of the mean-field contraction tests (the J . S step of Alg. 1, Sec. II).

Shared by the GPU tests (tests/test_gpu_contraction.py) and the CPU check that their tolerance
can fail (tests/test_contraction_tolerance.py). Inputs only -- instances, start states, fields,
replica samples and the kernel selection of each case; none of the method's arithmetic.

Start states are chosen on grids that the operand types hold exactly, so that the matrix
product on the GPU sees the same numbers as the FP64 oracle:

* ``grid``: s = k / 64 with integer |k| <= 64. At most 7 significant bits, exact in BF16 and FP32.
  Every partial sum of sum_j J_ij s_j is then a multiple of 2^-6 below 2^13 in magnitude for
  integral |J| <= 1 and n <= 8192 (19 significant bits), or a multiple of 2^-12 below 2^11 for the
  1/64-grid couplings below 4 at n = 400 (23 bits), or of 2^-6 below 2^11 for J = +-5 at n = 400:
  at most 24 significant bits, so an FP32 accumulator holds every partial sum exactly, in any order.
* ``fp8``: values of FP8 E4M3 in [-1, 1] (3 fraction bits, smallest step 2^-9), for the FP8-spin
  kernel; partial sums are multiples of 2^-9 below 2^11 (20 bits): exact in FP32.
* ``pm1``: +-1.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Tuple

import numpy as np

import instances

GRID = 64


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def grid_states(R: int, n: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(-GRID, GRID + 1, size=(R, n)).astype(np.float64) / GRID


def fp8_values_in_unit_interval() -> np.ndarray:
    """Every non-negative FP8 E4M3 value <= 1: subnormals m 2^-9 and normals (1 + m/8) 2^e."""
    vals = {m * 2.0**-9 for m in range(8)}
    for e in range(-6, 1):
        for m in range(8):
            v = (1.0 + m / 8.0) * 2.0**e
            if v <= 1.0:
                vals.add(v)
    return np.array(sorted(vals))


def fp8_states(R: int, n: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    mags = fp8_values_in_unit_interval()
    return g.choice(mags, size=(R, n)) * np.where(g.random((R, n)) < 0.5, -1.0, 1.0)


def pm1_states(R: int, n: int, seed: int) -> np.ndarray:
    return np.where(_rng(seed).random((R, n)) < 0.5, -1.0, 1.0)


def signed_fields(n: int, magnitude: float, seed: int) -> np.ndarray:
    """h_i = +-magnitude with random signs."""
    return np.where(_rng(seed).random(n) < 0.5, -magnitude, magnitude)


def bf16_grid_couplings(n: int, seed: int) -> np.ndarray:
    """Symmetric couplings on the 1/64 grid with |J| <= 255/64: 8 significant bits, exact in BF16
    but neither in FP8 E4M3 nor in FP4 E2M1."""
    g = _rng(seed)
    W = np.clip(np.round(g.normal(0.0, 1.0, (n, n)) * 64.0), -255, 255) / 64.0
    J = np.triu(W, 1)
    return J + J.T


@dataclasses.dataclass
class Case:
    name: str
    make: Callable[[], instances.Instance]  # instance with h = 0
    precision: str
    R: int
    sub: Tuple[int, ...]       # replicas compared with the oracle
    paths: Tuple[str, ...]     # acceptable kernel paths
    flags: Dict[str, bool]
    states: str = "grid"       # kind of start state of the one-step test
    j_format: str = ""         # expected storage format of J, if the case pins it
    field: float = 0.5         # magnitude of the +-fields of the saturated test

    def instance(self) -> instances.Instance:
        return self.make()

    def start_states(self, n: int, seed: int) -> np.ndarray:
        if self.states == "fp8":
            return fp8_states(self.R, n, seed)
        return grid_states(self.R, n, seed)


def _scaled_sk(n: int, seed: int, scale: float) -> instances.Instance:
    base = instances.sk(n, seed)
    return instances.Instance(scale * base.J, np.zeros(n), f"{scale}x{base.name}")


def _grid_j(n: int, seed: int) -> instances.Instance:
    return instances.Instance(bf16_grid_couplings(n, seed), np.zeros(n), f"bf16grid_n{n}_s{seed}")


_FULL_SUB = (0, 1, 63, 64, 127, 500, 511, 512, 777, 960, 1022, 1023)
_XCD_SUB = (0, 5, 127, 128, 200, 255, 256, 299)   # three groups of 128, the last ragged
_SMALL_SUB = (0, 15, 16, 100, 191, 192, 199)      # 16-replica blocks, the last ragged
_TILE_SUB = (0, 63, 127, 128, 150, 199)           # two 128-replica tiles, the second ragged

CASES: List[Case] = [
    # the launch configuration the benchmark times: G(2000, 1/2), R = 1024, register-J kernel
    Case("xrj_full_g2000", lambda: instances.gnp(2000, 0.5, 1), "fp8j_bf16s", 1024, _FULL_SUB,
         ("xcd_rj", "xcd_rj_fenced"), {}, j_format="fp4_e2m1"),
    Case("xrj8_full_g2000", lambda: instances.gnp(2000, 0.5, 1), "fp8j_fp8s", 1024, _FULL_SUB,
         ("xcd_rj", "xcd_rj_fenced"), {}, states="fp8", j_format="fp4_e2m1"),
    # the LDS-J group kernel in each of its three J formats
    Case("xcd_fp4_sk1000", lambda: instances.sk(1000, 3), "bf16", 300, _XCD_SUB,
         ("xcd", "xcd_fenced"), {"force_xcd": True, "force_lds_j": True}, j_format="fp4_e2m1"),
    Case("xcd_fp8_5sk400", lambda: _scaled_sk(400, 11, 5.0), "bf16", 300, _XCD_SUB,
         ("xcd", "xcd_fenced"), {"force_xcd": True}, j_format="fp8_e4m3"),
    Case("xcd_bf16_grid400", lambda: _grid_j(400, 12), "bf16", 300, _XCD_SUB,
         ("xcd", "xcd_fenced"), {"force_xcd": True}, j_format="bf16", field=1.0 / 128),
    Case("xcd_fp8j_g700", lambda: instances.gnp(700, 0.5, 2), "fp8j_bf16s", 300, _XCD_SUB,
         ("xcd", "xcd_fenced"), {"force_xcd": True, "force_lds_j": True}, j_format="fp4_e2m1"),
    # the persistent small-N kernel (J in LDS)
    Case("small_bf16_sk100", lambda: instances.sk(100, 2), "bf16", 200, _SMALL_SUB, ("persistent",), {}),
    Case("small_fp8j_g100", lambda: instances.gnp(100, 0.5, 2), "fp8j_bf16s", 200, _SMALL_SUB, ("persistent",), {}),
    Case("small_fp32_sk100", lambda: instances.sk(100, 2), "fp32", 200, _SMALL_SUB, ("persistent",), {}),
    # the tiled per-iteration kernel in each of its three J formats: ragged rows (300 of a 256-row
    # tile pair) and two replica tiles
    Case("tiled_bf16_sk300", lambda: instances.sk(300, 4), "bf16", 200, _TILE_SUB, ("step",),
         {"force_step": True}, j_format="fp4_e2m1"),
    # n % 4 != 0: a lane's four rows of the master state are not one aligned 16-byte word, so the
    # kernel takes its bounds-tested epilogue everywhere
    Case("tiled_bf16_sk301", lambda: instances.sk(301, 5), "bf16", 200, _TILE_SUB, ("step",),
         {"force_step": True}, j_format="fp4_e2m1"),
    Case("tiled_fp8j_g300", lambda: instances.gnp(300, 0.5, 4), "fp8j_bf16s", 200, _TILE_SUB, ("step",),
         {"force_step": True}, j_format="fp4_e2m1"),
    Case("tiled_fp8_5sk300", lambda: _scaled_sk(300, 11, 5.0), "bf16", 200, _TILE_SUB, ("step",),
         {"force_step": True}, j_format="fp8_e4m3"),
    Case("tiled_bf16_grid300", lambda: _grid_j(300, 12), "bf16", 200, _TILE_SUB, ("step",),
         {"force_step": True}, j_format="bf16", field=1.0 / 128),
    Case("tiled_fp8j_sk4100", lambda: instances.sk(4100, 7), "fp8j_bf16s", 200, _TILE_SUB, ("step",), {},
         j_format="fp4_e2m1"),
    Case("step_fp32_sk300", lambda: instances.sk(300, 4), "fp32", 200, _TILE_SUB, ("step",), {"force_step": True}),
    # the sparse kernels on a degree-3 graph
    Case("sparse_rq_d3_2000", lambda: instances.random_regular(2000, 3, 5), "bf16", 256, (0, 3, 100, 255),
         ("sparse_rq",), {}),
    Case("sparse_generic_d3_2000", lambda: instances.random_regular(2000, 3, 5), "bf16", 256, (0, 3, 100, 255),
         ("sparse",), {"sparse_generic": True}),
]

# One-step test: alpha and the constant temperature (sigma = 0; the noise has its own tests).
ONE_STEP_ALPHA = 0.6
ONE_STEP_T = 1.0
ONE_STEP_TF = 10
ONE_STEP_T_AT = 4
# Bound on |s_gpu - s_oracle| after one step from an exactly representable state (derivation in
# tests/test_gpu_contraction.py).
ONE_STEP_TOL = 1e-5

# Saturated test: alpha = 1, sigma = 0 and a temperature so low that every -tanh is exactly +-1
# in FP32 and FP64, so the whole trajectory is a sequence of +-1 vectors, equal bit for bit.
SAT_T = 1e-6
SAT_STEPS = 12
SAT_TF = 40
SAT_T_AT = 5
