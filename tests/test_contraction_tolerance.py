"""CPU check (oracle only) that the bars of tests/test_gpu_contraction.py can fail.

* One-step test: a contraction that is 1% off, J . S -> 0.99 J . S, is what the oracle computes
  from the start state 0.99 s0 at alpha = 1 (the field term is linear in s, the field h is not
  scaled). With the test's alpha the kernel's result would move by alpha times that change; on
  every case this is more than 100 times the bar.
* Saturated test: the oracle's trajectory is +-1 throughout and not a fixed point, and dropping
  one 128-wide block of k from the contraction (one spin chunk of the group kernels) flips
  spins -- a mistake the exact comparison cannot miss.
"""
import numpy as np
import pytest

import oracle
from contraction_cases import (CASES, ONE_STEP_ALPHA, ONE_STEP_T, ONE_STEP_TF, ONE_STEP_T_AT, ONE_STEP_TOL,
                               SAT_STEPS, SAT_T, SAT_TF, SAT_T_AT, pm1_states, signed_fields)


def _one_step(inst, T, sub, seed, s_init, alpha):
    _, s, _ = oracle.anneal(inst.J, inst.h, T[:ONE_STEP_T_AT], replicas=sub, seed=seed, alpha=alpha, sigma=0.0,
                            t_first=ONE_STEP_T_AT, s_init=s_init)
    return s


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_one_percent_contraction_error_exceeds_the_bar(case):
    inst = case.instance()
    seed = 4000 + CASES.index(case)
    s0 = case.start_states(inst.n, seed)
    sub = list(case.sub)
    T = np.full(ONE_STEP_TF, ONE_STEP_T)
    exact = _one_step(inst, T, sub, seed, s0[sub], 1.0)
    off = _one_step(inst, T, sub, seed, 0.99 * s0[sub], 1.0)
    shift = ONE_STEP_ALPHA * float(np.max(np.abs(off - exact)))
    assert shift > 100 * ONE_STEP_TOL, (case.name, shift)
    moved = _one_step(inst, T, sub, seed, s0[sub], ONE_STEP_ALPHA)
    assert np.max(np.abs(moved - s0[sub])) > 1000 * ONE_STEP_TOL


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_saturated_run_is_exact_and_a_dropped_block_shows(case):
    inst = case.instance()
    n = inst.n
    seed = 5000 + CASES.index(case)
    h = signed_fields(n, case.field, seed)
    s0 = pm1_states(case.R, n, seed)
    sub = list(case.sub)
    T = np.full(SAT_TF, SAT_T)
    t_end = SAT_T_AT + SAT_STEPS - 1
    _, _, traj = oracle.anneal(inst.J, h, T[:t_end], replicas=sub, seed=seed, alpha=1.0, sigma=0.0,
                               t_first=SAT_T_AT, s_init=s0[sub], record=SAT_STEPS)
    assert np.all(np.abs(traj) == 1.0)
    assert np.mean(traj[-1] != traj[0]) > 0.01
    # the same run with the couplings of one k block (columns 0..127, or all of them for n < 128)
    # left out of the field, as a contraction that skipped a chunk would compute (the normaliser,
    # which also changes, is positive and cannot change a sign)
    J_cut = inst.J.copy()
    J_cut[:, : min(128, n)] = 0.0
    J_cut[: min(128, n), :] = 0.0  # kept symmetric, as the oracle requires of J
    _, _, traj_cut = oracle.anneal(J_cut, h, T[:t_end], replicas=sub, seed=seed, alpha=1.0, sigma=0.0,
                                   t_first=SAT_T_AT, s_init=s0[sub], record=SAT_STEPS)
    assert np.sum(traj_cut != traj) > 0
