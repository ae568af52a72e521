"""GPU parity of the FP8-spin precision (NMFA_FP8J_FP8S): the register-J kernel with FP4 couplings
and FP8 E4M3 spin operands on the scaled FP4 x FP8 matrix instruction.

Bars:
* early trajectory (first 10 iterations) within 5e-4 of the FP64 oracle. The FP8 spin operands
  are rounded to within 2^-4 of the state, so the normalised mean field errs by about 0.04 s_rms;
  at the early temperatures (T ~ 10, states ~ 1e-2) that moves a state by ~1e-5 per iteration
  (measured: 6e-5 after 10; an operand-layout error measured 1.3e-3). Energies of the returned
  spins are bit-exact;
* at a constant cold temperature the trajectory stays within 2e-2 of the oracle (see that test);
* replica-prefix and checkpoint/resume invariance are bit-exact; the XCD-local and the
  device-fenced exchange give bit-identical states;
* on a K2000-class instance the success probability at the FP64 path's 10th-percentile energy is
  within 2 binomial standard errors of the FP64 path's;
* instances the kernel cannot take are refused with NMFA_EINVAL.
"""
import numpy as np
import pytest

import instances
import oracle
from oracle import stats

pytestmark = pytest.mark.gpu
P = "fp8j_fp8s"


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


@pytest.mark.parametrize("n,R,t_f", [(200, 300, 400), (70, 40, 400), (1000, 129, 400), (2000, 1024, 5000)])
def test_fp8s_early_trajectory_and_energies(nmfa, n, R, t_f):
    inst = instances.sk(n, 3)
    inst.h = np.round(instances.gaussian_fields(n, 1.0, 2))
    sub = [0, R // 2, R - 1]
    n_rec, seed = 10, 17
    with nmfa.Solver(inst.J, inst.h, precision=P, record_iters=n_rec) as s:
        s.anneal(R, t_f, seed)
        traj, spins, (E, Ei), path = s.trajectory(), s.spins(), s.energies(), s.info()["path"]
    assert path in ("xcd_rj", "xcd_rj_fenced")
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:n_rec], replicas=sub, seed=seed, record=n_rec)
    err = float(np.max(np.abs(traj[:, sub, :] - otraj)))
    print(f"n={n} R={R}: max |ds| over 10 iterations {err:.2e}")
    assert err <= 5e-4, err
    rows = np.arange(0, R, max(1, R // 40))
    assert np.array_equal(Ei[rows], oracle.energies_int(inst.J, inst.h, spins[rows]))


def test_fp8s_prefix_resume_and_fenced(nmfa):
    inst = instances.sk(900, 8)
    t_f, seed = 300, 5
    with nmfa.Solver(inst.J, inst.h, precision=P) as s:
        s.anneal(100, t_f, seed)
        full100 = s.state()
        s.anneal(37, t_f, seed)
        full37 = s.state()
        s.anneal_range(37, t_f, 1, 120, seed)
        s.anneal_range(37, t_f, 121, t_f, seed)
        resumed = s.state()
    assert np.array_equal(full100[:37], full37)
    assert np.array_equal(resumed, full37)
    with nmfa.Solver(inst.J, inst.h, precision=P, force_fenced=True) as s:
        s.anneal(100, t_f, seed)
        assert s.info()["path"] == "xcd_rj_fenced"
        assert np.array_equal(s.state(), full100)


def test_fp8s_k2000_success_vs_fp64(nmfa):
    inst = instances.sk(2000, 4)
    R, t_f = 1024, 5000
    with nmfa.Solver(inst.J, inst.h, precision="fp64") as s:
        s.anneal(R, t_f, 2023)
        E_ref = s.energies()[0]
        s.anneal(R, t_f, 2024)
        E64 = s.energies()[0]
    with nmfa.Solver(inst.J, inst.h, precision=P) as s:
        s.anneal(R, t_f, 2026)
        E8 = s.energies()[0]
        assert s.info()["path"] == "xcd_rj"
    target = float(np.percentile(E_ref, 10))
    p64 = stats.success_probability(E64, target)
    p8 = stats.success_probability(E8, target)
    print(f"K2000 class: p_fp64 {p64:.4f}  p_fp8s {p8:.4f}  mean E {E64.mean():.1f} vs {E8.mean():.1f}")
    assert stats.within_two_se(p8, R, p64, R), (p8, p64)


def test_fp8s_refuses_what_the_kernel_cannot_take(nmfa):
    gauss = np.triu(np.random.default_rng(1).normal(size=(300, 300)), 1)
    with pytest.raises(nmfa.NmfaError) as ei:
        nmfa.Solver(gauss + gauss.T, None, precision=P)  # not exact in FP4
    assert ei.value.code == -1
    with pytest.raises(nmfa.NmfaError):
        nmfa.Solver(instances.sk(2100, 1).J, None, precision=P)  # n > 2048
    with pytest.raises(nmfa.NmfaError):
        nmfa.Solver(instances.sk(300, 1).J, None, precision=P, force_sparse=True)


def test_fp8s_follows_the_mean_field_when_cold(nmfa):
    """At a constant T = 0.5 the states follow the mean field from the first iterations, so an
    operand-layout error shows at once (a misplaced k block moves a state by ~alpha * 2 s_rms per
    iteration). FP8 rounding alone errs by ~0.04 s_rms in the field, ~0.01 s_rms per iteration in
    the state, amplified by at most (1 - alpha) + alpha * 2 lambda / T ~ 1.5 per iteration."""
    inst = instances.sk(800, 12)
    knots = [(0.0, 0.5), (1.0, 0.5)]
    R, t_f, seed, n_rec = 64, 6, 31, 6
    with nmfa.Solver(inst.J, inst.h, precision=P, knots=knots, record_iters=n_rec) as s:
        s.anneal(R, t_f, seed)
        traj = s.trajectory()
    sub = [0, 17, 63]
    _, _, otraj = oracle.anneal(inst.J, inst.h, np.full(t_f, 0.5), replicas=sub, seed=seed, record=n_rec)
    err = [float(np.max(np.abs(traj[k, sub, :] - otraj[k]))) for k in range(n_rec)]
    rms = [float(np.sqrt(np.mean(otraj[k] ** 2))) for k in range(n_rec)]
    print("cold schedule: max |ds| per iteration", ["%.1e" % e for e in err], "state rms", ["%.2f" % r for r in rms])
    assert max(err) <= 2e-2, err  # measured 4.4e-3 after 6 iterations (state rms 0.11)
