"""Parity at the largest instance the library accepts, n = 16384.

At this size a dense instance runs on the per-iteration kernel and a degree-3 graph on the generic
sparse kernel (the register-ELL variant stops at n = 4096). Both are checked against the FP64
oracle: the FP32 trajectory of every replica for the first iterations to 1e-4, and the exact
integer energies of the readout bit for bit.
"""
import numpy as np
import pytest

import instances
import oracle

pytestmark = pytest.mark.gpu

N = 16384


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


def _check(nmfa, inst, R, t_f, seed, expect_path):
    with nmfa.Solver(inst.J, inst.h, precision="fp32", record_iters=t_f) as s:
        s.anneal(R, t_f, seed)
        assert s.info()["path"] == expect_path
        traj, spins, E_int = s.trajectory(), s.spins(), s.energies()[1]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=R, seed=seed, record=t_f,
                                threads=oracle.num_threads())
    assert np.max(np.abs(traj - otraj)) <= 1e-4
    assert np.array_equal(E_int, oracle.energies_int(inst.J, inst.h, spins))


def test_dense_sk_at_max_n(nmfa):
    _check(nmfa, instances.sk(N, 5), R=3, t_f=8, seed=3, expect_path="step")


def test_degree3_graph_at_max_n(nmfa):
    _check(nmfa, instances.random_regular(N, 3, 9), R=5, t_f=8, seed=4, expect_path="sparse")
