"""GPU parity of the method's parameter variants against the FP64 oracle.

The paper tunes alpha = sigma = 0.15 only coarsely (Sec. II), calls the noise-free iteration
mean-field annealing (Sec. I), and gives its schedule only as a figure (Fig. 2): the library takes
alpha, sigma, schedule knots or an explicit temperature array as parameters. Bars:

* FP64 path (persistent small-N kernel, per-iteration kernel, sparse kernel): trajectories within
  1e-9 of the oracle for 50 iterations and exact integer energies, for alpha = 0.05 and 0.6,
  sigma = 0.3, sigma = 0 with integral fields h != 0 (mean-field annealing proper; with h = 0 the
  noise-free state never leaves 0), custom knots, and an explicit (non-monotone) temperature array.
* BF16 / FP8-J paths (register-J group kernel at the benchmark size, persistent small-N kernel):
  the noise-free variants as one step from an exactly representable state, within the 1e-5 bar
  derived in tests/test_gpu_contraction.py.
"""
import numpy as np
import pytest

import instances
import oracle
from contraction_cases import ONE_STEP_TOL, grid_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


T_F = 300
KNOTS = ((0.0, 5.0), (0.3, 1.0), (1.0, 0.1))


def _explicit_T(t_f):
    t = np.arange(1, t_f + 1)
    return 1.5 + np.sin(t / 7.0) + 4.0 * np.exp(-t / 40.0)  # positive, not monotone


VARIANTS = {
    "alpha_0.05": dict(alpha=0.05, sigma=0.15),
    "alpha_0.6": dict(alpha=0.6, sigma=0.15),
    "sigma_0.3": dict(alpha=0.15, sigma=0.3),
    "mfa_sigma0_fields": dict(alpha=0.15, sigma=0.0),
    "knots": dict(alpha=0.15, sigma=0.15, knots=KNOTS),
    "explicit_T": dict(alpha=0.15, sigma=0.15, temperatures=_explicit_T(T_F)),
}


def _schedule(v):
    if "temperatures" in v:
        return np.asarray(v["temperatures"], dtype=np.float64)
    return oracle.schedule(T_F, v.get("knots", oracle.DEFAULT_KNOTS))


@pytest.mark.parametrize("kernel", ["persistent", "step", "sparse"])
@pytest.mark.parametrize("name", list(VARIANTS))
def test_fp64_variant_trajectory(nmfa, name, kernel):
    v = VARIANTS[name]
    if kernel == "sparse":
        inst = instances.random_regular(60, 3, 9)
    else:
        inst = instances.sk(40, 7)
    inst.h = np.round(instances.gaussian_fields(inst.n, 2.0, 8))
    assert np.any(inst.h != 0)
    R, seed, rec = 70, 321, 50
    flags = {"step": {"force_step": True}, "sparse": {"force_sparse": True}}.get(kernel, {})
    print(f"fp64 variant {name} on {kernel}", flush=True)
    with nmfa.Solver(inst.J, inst.h, precision="fp64", record_iters=rec, **v, **flags) as s:
        s.anneal(R, T_F, seed)
        traj = s.trajectory()
        spins = s.spins()
        _, Ei = s.energies()
        path = s.info()["path"]
    assert path.startswith(kernel), path
    _, _, otraj = oracle.anneal(inst.J, inst.h, _schedule(v), R=R, seed=seed, alpha=v["alpha"], sigma=v["sigma"],
                                record=rec)
    assert np.max(np.abs(traj - otraj)) <= 1e-9
    assert np.array_equal(Ei, oracle.energies_int(inst.J, inst.h, spins))
    if v["sigma"] == 0.0:
        # noise-free: every replica follows the same deterministic trajectory, and it moves
        assert np.all(traj == traj[:, :1, :])
        assert np.max(np.abs(otraj[-1])) > 0.1


BF16_VARIANTS = {
    "alpha_0.05_knots": dict(alpha=0.05, knots=KNOTS),
    "alpha_1": dict(alpha=1.0),
    "mfa_fields": dict(alpha=0.15),
    "explicit_T": dict(alpha=0.3, temperatures=_explicit_T(T_F)),
}


@pytest.mark.parametrize("where", ["xrj_g2000", "small_sk100"])
@pytest.mark.parametrize("name", list(BF16_VARIANTS))
def test_reduced_precision_noise_free_variant_one_step(nmfa, name, where):
    v = dict(BF16_VARIANTS[name])
    if where == "xrj_g2000":
        inst, precision, R, sub, path = instances.gnp(2000, 0.5, 1), "fp8j_bf16s", 1024, [0, 64, 700, 1023], "xcd_rj"
    else:
        inst, precision, R, sub, path = instances.sk(100, 2), "bf16", 200, [0, 17, 199], "persistent"
    inst.h = np.round(instances.gaussian_fields(inst.n, 3.0, 5))
    t_at = 150
    seed = 77
    s0 = grid_states(R, inst.n, 31)
    print(f"reduced-precision variant {name} on {where}", flush=True)
    with nmfa.Solver(inst.J, inst.h, precision=precision, sigma=0.0, **v) as s:
        s.set_state(s0)
        s.anneal_range(R, T_F, t_at, t_at, seed)
        got = s.state()
        assert s.info()["path"] == path
    T = _schedule(v)
    _, s_or, _ = oracle.anneal(inst.J, inst.h, T[:t_at], replicas=sub, seed=seed, alpha=v["alpha"], sigma=0.0,
                               t_first=t_at, s_init=s0[sub])
    assert np.max(np.abs(got[sub] - s_or)) <= ONE_STEP_TOL
