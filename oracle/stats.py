"""Success statistics for annealing samples -- TEST INFRASTRUCTURE ONLY (part of the oracle).

The paper reports success probabilities over 10,000 samples per instance and the time-to-solution
(TTS) metric of the CIM literature (Sec. III, Fig. 4 caption). The TTS formula is not printed;
the standard 99% form is used: the expected time to see the target at least once with 99%
confidence, t_sample * ln(0.01) / ln(1 - p).
"""
from __future__ import annotations

import math

import numpy as np


def success_probability(E: np.ndarray, target: float, tol: float = 1e-9) -> float:
    E = np.asarray(E, dtype=np.float64)
    return float(np.mean(E <= target + tol)) if E.size else 0.0


def binomial_se(p: float, n: int) -> float:
    return math.sqrt(max(p * (1.0 - p), 0.0) / n) if n > 0 else float("inf")


def within_two_se(p_a: float, n_a: int, p_b: float, n_b: int, floor: float = 0.0) -> bool:
    """|p_a - p_b| <= 2 * sqrt(p_a(1-p_a)/n_a + p_b(1-p_b)/n_b) (plus an optional floor)."""
    se = math.sqrt(max(p_a * (1 - p_a), 0.0) / n_a + max(p_b * (1 - p_b), 0.0) / n_b)
    return abs(p_a - p_b) <= 2.0 * se + floor


def tts99(t_sample_s: float, p: float) -> float:
    if p <= 0.0:
        return float("inf")
    if p >= 0.99:
        return t_sample_s
    return t_sample_s * math.log(0.01) / math.log(1.0 - p)
