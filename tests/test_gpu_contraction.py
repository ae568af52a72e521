"""GPU parity of the mean-field contraction J . S (the field of Alg. 1, Sec. II) in every kernel
and J storage format, against the FP64 oracle, with bars that a wrong contraction cannot meet.

Early trajectories of the default schedule start at T ~ 10 where the states are ~1e-2 and the
field term barely moves them, so a trajectory tolerance there says little about J . S. These
tests instead start every kernel from a chosen state (nmfa_set_state) and compare iterations
where the field term decides the result.

1. One step at constant T = 1, alpha = 0.6, sigma = 0, from a start state the operand type holds
   exactly (tests/contraction_cases.py: a 1/64 grid, or FP8 E4M3 values for FP8 spins). Bar:
   |s_gpu - s_oracle| <= 1e-5, derived as follows.
   * Operands: J (integral, or on the 1/64 grid) and the start state are exact in the MFMA
     operand types, and every partial sum of sum_j J_ij s_j needs at most 23 significant bits, so
     the FP32 accumulation is exact whatever its order: the GPU contraction equals the FP64 one.
   * Normalisation: Phi = fma(acc, inv, h inv) with inv = fp32(1 / norm): relative error
     <= 3 * 2^-24, i.e. <= 1e-6 for |Phi| <= 5.
   * Boltzmann factor: -tanh through exp2 and a reciprocal, 2 / (1 + e) - 1: absolute error
     <= 4 * 2^-24 ~ 2.4e-7 (the reciprocal's relative error, doubled), plus the argument error
     above times |tanh'| <= 1 at T = 1.
   * Update: fma(alpha, s^, (1 - alpha) s) rounds once, <= 2^-24 ~ 6e-8.
   Sum: 0.6 * (1e-6 + 2.4e-7) + 6e-8 < 1e-6. The bar leaves a factor of ten. A contraction that
   is 1% off moves the result by 0.6 * |tanh(Phi) - tanh(0.99 Phi)|, which
   tests/test_contraction_tolerance.py shows (on the CPU, with the oracle) exceeds the bar by more
   than a factor of 100 on every case here.
2. Saturated dynamics: alpha = 1, sigma = 0, T = 1e-6 and fields +-1/2 (+-1/128 for the
   1/64-grid couplings) that keep h_i + sum_j J_ij s_j away from 0. Every -tanh is then exactly
   +-1 in FP32 and in FP64, so the trajectory is a sequence of +-1 vectors that the kernel must
   reproduce bit for bit over 12 iterations: each iteration's spins travel through the kernel's
   exchange (across the workgroups of a group, through L2) to the next. Any misplaced or dropped
   part of the contraction flips signs (the CPU test plants one and counts them). The energies
   of the readout are exact.
"""
import numpy as np
import pytest

import oracle
from contraction_cases import (CASES, ONE_STEP_ALPHA, ONE_STEP_T, ONE_STEP_TF, ONE_STEP_T_AT, ONE_STEP_TOL,
                               SAT_STEPS, SAT_T, SAT_TF, SAT_T_AT, pm1_states, signed_fields)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


def _check_kernel(case, info):
    assert info["path"] in case.paths, (case.name, info)
    if case.j_format:
        assert info["j_format"] == case.j_format, (case.name, info)


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_one_step_contraction(nmfa, case):
    inst = case.instance()
    n = inst.n
    seed = 4000 + CASES.index(case)
    s0 = case.start_states(n, seed)
    T = np.full(ONE_STEP_TF, ONE_STEP_T)
    print(f"one step: {case.name} n={n} R={case.R} {case.precision}", flush=True)
    with nmfa.Solver(inst.J, inst.h, precision=case.precision, alpha=ONE_STEP_ALPHA, sigma=0.0, temperatures=T,
                     **case.flags) as s:
        s.set_state(s0)
        s.anneal_range(case.R, ONE_STEP_TF, ONE_STEP_T_AT, ONE_STEP_T_AT, seed)
        got = s.state()
        _check_kernel(case, s.info())
    sub = list(case.sub)
    _, s_or, _ = oracle.anneal(inst.J, inst.h, T[:ONE_STEP_T_AT], replicas=sub, seed=seed, alpha=ONE_STEP_ALPHA,
                               sigma=0.0, t_first=ONE_STEP_T_AT, s_init=s0[sub])
    err = float(np.max(np.abs(got[sub] - s_or)))
    assert err <= ONE_STEP_TOL, (case.name, err)
    # the step did move the states, by far more than the bar
    assert np.max(np.abs(s_or - s0[sub])) > 1000 * ONE_STEP_TOL


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_saturated_trajectory_is_exact(nmfa, case):
    inst = case.instance()
    n = inst.n
    seed = 5000 + CASES.index(case)
    h = signed_fields(n, case.field, seed)
    s0 = pm1_states(case.R, n, seed)
    T = np.full(SAT_TF, SAT_T)
    t_end = SAT_T_AT + SAT_STEPS - 1
    print(f"saturated: {case.name} n={n} R={case.R} {case.precision}", flush=True)
    with nmfa.Solver(inst.J, h, precision=case.precision, alpha=1.0, sigma=0.0, temperatures=T,
                     record_iters=SAT_STEPS, **case.flags) as s:
        s.set_state(s0)
        s.anneal_range(case.R, SAT_TF, SAT_T_AT, t_end, seed)
        traj = s.trajectory()
        spins = s.spins()
        E, _ = s.energies()
        _check_kernel(case, s.info())
    sub = list(case.sub)
    spins_or, _, otraj = oracle.anneal(inst.J, h, T[:t_end], replicas=sub, seed=seed, alpha=1.0, sigma=0.0,
                                       t_first=SAT_T_AT, s_init=s0[sub], record=SAT_STEPS)
    assert np.all(np.abs(otraj) == 1.0)  # the oracle's own trajectory is saturated
    mism = int(np.sum(traj[:, sub, :] != otraj))
    assert mism == 0, (case.name, mism)
    assert np.array_equal(spins[sub], spins_or)
    # energies of the readout: fields and couplings are dyadic with few bits, so the FP64 sums
    # are exact in any order and equal the oracle's bit for bit
    assert np.array_equal(E[sub], oracle.energies(inst.J, h, spins[sub]))
    # the run is not a fixed point: spins change after the first recorded iteration
    assert np.mean(otraj[-1] != otraj[0]) > 0.01
