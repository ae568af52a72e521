"""Parity at large sizes, up to the largest instance the library accepts, n = 16384.

Above n = 2048 a dense instance runs on the per-iteration kernels (the tiled BF16 matrix product
for the BF16-operand precisions, the tiled FP64 one for FP64, the direct one for FP32) and a
degree-3 graph on the generic sparse kernel (the register-ELL variant stops at n = 4096). All are
checked against the FP64 oracle: FP64 trajectories of every replica for the first iterations to
1e-9, FP32 ones to 1e-4, BF16 ones to 5e-3 (BF16 operand rounding of states of order 0.1), and the
exact integer energies of the readout bit for bit.
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


def _check(nmfa, inst, R, t_f, seed, expect_path, precision="fp32", tol=1e-4):
    with nmfa.Solver(inst.J, inst.h, precision=precision, record_iters=t_f) as s:
        s.anneal(R, t_f, seed)
        assert s.info()["path"] == expect_path
        traj, spins, E_int = s.trajectory(), s.spins(), s.energies()[1]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=R, seed=seed, record=t_f,
                                threads=oracle.num_threads())
    assert np.max(np.abs(traj - otraj)) <= tol
    assert np.array_equal(E_int, oracle.energies_int(inst.J, inst.h, spins))


def test_dense_sk_at_max_n(nmfa):
    _check(nmfa, instances.sk(N, 5), R=3, t_f=8, seed=3, expect_path="step")


def test_degree3_graph_at_max_n(nmfa):
    _check(nmfa, instances.random_regular(N, 3, 9), R=5, t_f=8, seed=4, expect_path="sparse")


def test_bf16_tiled_step_at_max_n(nmfa):
    _check(nmfa, instances.sk(N, 6), R=3, t_f=8, seed=5, expect_path="step", precision="bf16", tol=5e-3)


def test_fp64_tiled_step_at_max_n(nmfa):
    _check(nmfa, instances.sk(N, 8), R=3, t_f=8, seed=6, expect_path="step", precision="fp64", tol=1e-9)


def test_fp64_tiled_step_ragged(nmfa):
    # n = 4100 (33 row tiles of 128, the last nearly empty), R = 70 (two replica tiles of 64, the
    # second ragged), with fields
    inst = instances.sk(4100, 11)
    inst.h = np.round(instances.gaussian_fields(4100, 1.0, 5))
    _check(nmfa, inst, R=70, t_f=8, seed=12, expect_path="step", precision="fp64", tol=1e-9)


def test_bf16_tiled_step_ragged(nmfa):
    # n = 4100 (17 row tiles of 256, the last nearly empty), R = 200 (two replica tiles, the second
    # ragged), with fields; then replica-prefix and resume invariance, bit for bit
    inst = instances.sk(4100, 7)
    inst.h = np.round(instances.gaussian_fields(4100, 1.0, 3))
    R, t_f, seed, n_rec = 200, 300, 9, 10
    sub = [0, 127, 128, 199]
    with nmfa.Solver(inst.J, inst.h, precision="fp8j_bf16s", record_iters=n_rec) as s:
        s.anneal(R, t_f, seed)
        assert s.info()["path"] == "step"
        traj, spins, E_int, full = s.trajectory(), s.spins(), s.energies()[1], s.state()
        s.anneal(77, t_f, seed)
        prefix = s.state()
        s.anneal_range(77, t_f, 1, 140, seed)
        s.anneal_range(77, t_f, 141, t_f, seed)
        resumed = s.state()
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:n_rec], replicas=sub, seed=seed,
                                record=n_rec, threads=oracle.num_threads())
    assert np.max(np.abs(traj[:, sub, :] - otraj)) <= 5e-3
    rows = np.arange(0, R, 9)
    assert np.array_equal(E_int[rows], oracle.energies_int(inst.J, inst.h, spins[rows]))
    assert np.array_equal(prefix, full[:77])
    assert np.array_equal(resumed, prefix)
