"""GPU parity of the sparse (ELL) kernel for degree-d graphs (the paper's degree-3 class).

Bars:
* FP64: the trajectory follows the FP64 oracle to 1e-9 (the ELL row sum is the dense sum without
  its exact zero terms), energies bit-exact;
* FP32 / BF16 precisions (FP32 arithmetic): early trajectory within 1e-4 of the oracle (the fast
  FP32 noise and tanh track FP64 to ~1e-6 per step), energies bit-exact;
* replica-prefix and checkpoint/resume invariances are bit-exact; negated noise negates the FP64
  trajectory bit-exactly;
* ragged sizes (N not a multiple of 4, R not a multiple of the replicas per workgroup);
* a serving mix with sparse jobs gives each job the result it gets alone;
* the register-ELL kernel and the generic ELL kernel give bit-identical states, trajectories and
  resumed runs over every replica-block size, padded degree and quads-per-thread variant.
"""
import numpy as np
import pytest

import instances
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


def _run(nmfa, inst, precision, R, t_f, seed, n_rec, **kw):
    with nmfa.Solver(inst.J, inst.h, precision=precision, record_iters=n_rec, **kw) as s:
        s.anneal(R, t_f, seed)
        info = s.info()
        return info, s.trajectory(), s.spins(), s.energies(), s.state()


def test_fp64_moebius_with_fields_follows_oracle(nmfa):
    inst = instances.moebius_ladder(300)
    inst.h = instances.gaussian_fields(300, 0.3, 4)
    R, t_f, seed, n_rec = 37, 200, 11, 20
    info, traj, spins, (E, _), _ = _run(nmfa, inst, "fp64", R, t_f, seed, n_rec)
    assert info["path"] == "sparse_rq" and info["j_format"] == "ell"
    sub = [0, 18, 36]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:n_rec], replicas=sub, seed=seed,
                                record=n_rec)
    assert np.max(np.abs(traj[:, sub, :] - otraj)) <= 1e-9
    assert np.array_equal(E, oracle.energies(inst.J, inst.h, spins))


@pytest.mark.parametrize("precision,n,d", [("fp32", 1000, 5), ("bf16", 500, 3), ("fp8j_bf16s", 777, 10)])
def test_fp32_arithmetic_regular_graphs(nmfa, precision, n, d):
    inst = instances.random_regular(n, d, 7)
    inst.h = np.round(instances.gaussian_fields(inst.n, 1.0, 8))
    R, t_f, seed, n_rec = 70, 300, 5, 10
    info, traj, spins, (E, Ei), _ = _run(nmfa, inst, precision, R, t_f, seed, n_rec)
    assert info["path"] == "sparse_rq"
    sub = [0, 33, 69]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:n_rec], replicas=sub, seed=seed,
                                record=n_rec)
    assert np.max(np.abs(traj[:, sub, :] - otraj)) <= 1e-4
    assert np.array_equal(Ei, oracle.energies_int(inst.J, inst.h, spins))


def test_small_ragged_forced_sparse(nmfa):
    inst = instances.moebius_ladder(50)  # N = 50: 13 quads, the last one half empty
    R, t_f, seed, n_rec = 9, 150, 3, 12
    info, traj, spins, (E, Ei), _ = _run(nmfa, inst, "fp64", R, t_f, seed, n_rec, force_sparse=True)
    assert info["path"] == "sparse_rq"
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:n_rec], replicas=list(range(R)), seed=seed,
                                record=n_rec)
    assert np.max(np.abs(traj - otraj)) <= 1e-9
    assert np.array_equal(Ei, oracle.energies_int(inst.J, inst.h, spins))


def test_prefix_resume_and_negation(nmfa):
    inst = instances.random_regular(400, 4, 2)
    t_f, seed = 220, 9
    with nmfa.Solver(inst.J, None, precision="fp32") as s:
        assert s.info()["path"] == "sparse"  # before an anneal the two sparse kernels are not told apart
        s.anneal(50, t_f, seed)
        full50 = s.state()
        s.anneal(21, t_f, seed)
        full21 = s.state()
        s.anneal_range(21, t_f, 1, 101, seed)
        s.anneal_range(21, t_f, 102, t_f, seed)
        resumed = s.state()
    assert np.array_equal(full50[:21], full21)
    assert np.array_equal(resumed, full21)
    # negation: bit-exact in FP64 (tanh is odd there; the FP32 tanh 2/(1+2^a)-1 is odd only to
    # rounding, since 2^-a is not exactly 1/2^a)
    out = {}
    for neg in (False, True):
        with nmfa.Solver(inst.J, None, precision="fp64", negate_noise=neg) as s:
            s.anneal(21, t_f, seed)
            assert s.info()["path"] == "sparse_rq"
            out[neg] = s.state()
    assert np.array_equal(out[True], -out[False])


def test_serving_mix_with_sparse_jobs(nmfa):
    jobs = []
    for k, (n, d, R, t_f) in enumerate([(600, 3, 64, 400), (300, 6, 96, 350), (900, 4, 128, 300)]):
        inst = instances.random_regular(n, d, 40 + k)
        jobs.append((inst, R, t_f, 900 + k))
    jobs.append((instances.sk(120, 3), 64, 300, 950))  # a dense small job alongside
    alone = []
    for inst, R, t_f, seed in jobs:
        with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
            s.anneal(R, t_f, seed)
            alone.append(s.energies()[0])
    with nmfa.Server(precision="bf16", chunk_iters=64) as srv:
        tickets = [srv.submit(inst.J, inst.h, R, t_f, seed) for inst, R, t_f, seed in jobs]
        for E, t in zip(alone, tickets):
            assert srv.wait(t, 120000)
            assert np.array_equal(srv.result(t)["E"], E)


# (precision, n, degree, R): RB = 4 / 2 / 1 follow from R on a 256-CU device (one workgroup per CU
# at least); degrees 3 / 7 / 13 pad to 4 / 8 / 16 couplings per row; n = 2500 gives two quads per
# thread; degree 20 stays on the generic kernel.
RQ_CASES = [
    ("fp32", 500, 3, 1024), ("bf16", 998, 7, 600), ("fp8j_bf16s", 402, 13, 130), ("fp32", 2500, 5, 700),
    ("fp64", 300, 3, 600), ("fp64", 501, 6, 70), ("fp64", 2100, 4, 40), ("fp32", 600, 20, 300),
]


@pytest.mark.parametrize("precision,n,d,R", RQ_CASES)
def test_register_kernel_matches_generic(nmfa, precision, n, d, R):
    inst = instances.random_regular(n, d, 17 + d)
    inst.h = np.round(instances.gaussian_fields(n, 1.0, 5))
    t_f, seed, n_rec = 160, 23, 6
    got = {}
    for generic in (False, True):
        with nmfa.Solver(inst.J, inst.h, precision=precision, record_iters=n_rec, sparse_generic=generic) as s:
            s.anneal_range(R, t_f, 1, 70, seed)
            s.anneal_range(R, t_f, 71, t_f, seed)
            path = s.info()["path"]
            got[generic] = (path, s.trajectory(), s.state(), s.energies()[1])
    expect_rq = d <= 16
    assert got[False][0] == ("sparse_rq" if expect_rq else "sparse")
    assert got[True][0] == "sparse"
    for a, b in zip(got[False][1:], got[True][1:]):
        assert np.array_equal(a, b)
