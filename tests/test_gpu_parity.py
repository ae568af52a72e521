"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bars (written in each test):
* FP64 path: trajectories within 1e-9 of the oracle for the first 50 iterations; integer
  energies bit-exact; Philox words bit-exact; FP64 Gaussians within 1e-12.
* FP32 path: trajectories within 1e-4 for the first 20 iterations (FP32 arithmetic and FP32
  noise against FP64); success probability within 2 binomial standard errors of FP64.
* BF16 / FP8-J paths: trajectories within 5e-3 for the first 10 iterations (BF16 operand
  rounding, relative 2^-9, on states of order 0.1); success probability within 2 SE of FP64.
"""
import numpy as np
import pytest

import instances
import oracle
from oracle import stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nmfa():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m


def _run(nmfa, inst, precision, R, t_f, seed, record=0, **kw):
    with nmfa.Solver(inst.J, inst.h, precision=precision, record_iters=record, **kw) as s:
        s.anneal(R, t_f, seed)
        out = {
            "spins": s.spins(),
            "E": s.energies()[0],
            "E_int": s.energies()[1],
            "state": s.state(),
            "path": s.info()["path"],
        }
        if record:
            out["traj"] = s.trajectory()
    return out


# --------------------------------------------------------------------------------------------
# noise stream
# --------------------------------------------------------------------------------------------

def test_philox_words_bit_exact(nmfa):
    seed = 0x123456789ABCDEF
    for t, r0 in [(1, 0), (777, 4000), (5000, 16000)]:
        w = nmfa.noise_words(seed, t, r0, 8, 40)
        for k in (0, 3, 7):
            for q in (0, 1, 17, 39):
                key = [seed & 0xFFFFFFFF, seed >> 32]
                assert tuple(int(v) for v in w[k, q]) == oracle.philox4x32_10([q, r0 + k, t, 0], key)


def test_noise_values_fp64_and_fp32(nmfa):
    seed = 99
    z64 = nmfa.noise_values(seed, 12, 5, 4, 25, fp64=True)
    z32 = nmfa.noise_values(seed, 12, 5, 4, 25, fp64=False)
    ref = np.array([[oracle.noise(seed, 12, 5 + k, i) for i in range(100)] for k in range(4)])
    assert np.max(np.abs(z64 - ref)) <= 1e-12
    assert np.max(np.abs(z32 - ref)) <= 5e-5


# --------------------------------------------------------------------------------------------
# FP64 path: trajectory parity
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("force_step", [False, True])
def test_fp64_trajectory_sk20(nmfa, force_step):
    """SK N=20, R=256, t_f=1000 (the FP64 validation workload): |ds| <= 1e-9 for t <= 50."""
    inst = instances.sk(20, 1)
    R, t_f, seed = 256, 1000, 1001
    g = _run(nmfa, inst, "fp64", R, t_f, seed, record=50, force_step=force_step)
    assert g["path"] == ("step" if force_step else "persistent")
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=R, seed=seed, record=50)
    assert np.max(np.abs(g["traj"] - otraj)) <= 1e-9
    # energies of the returned spins are exact integers equal to the oracle's
    assert np.array_equal(g["E_int"], oracle.energies_int(inst.J, inst.h, g["spins"]))
    assert np.array_equal(g["E"], g["E_int"].astype(np.float64))
    # readout is the sign of the returned state
    assert np.array_equal(g["spins"], np.where(g["state"] >= 0, 1, -1).astype(np.int8))


def test_fp64_success_matches_oracle_sk20(nmfa):
    inst = instances.sk(20, 2)
    E0, _ = oracle.ground_state(inst.J, inst.h)
    R, t_f, seed = 256, 1000, 77
    g = _run(nmfa, inst, "fp64", R, t_f, seed)
    spins_o, s_o, _ = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=R, seed=seed)
    Eo = oracle.energies(inst.J, inst.h, spins_o)
    # same noise, FP64 on both sides: the final states agree closely for nearly all replicas
    close = np.max(np.abs(g["state"] - s_o), axis=1) <= 1e-6
    assert close.mean() >= 0.9
    assert np.all(g["E"] >= E0)
    p_g, p_o = stats.success_probability(g["E"], E0), stats.success_probability(Eo, E0)
    assert stats.within_two_se(p_g, R, p_o, R)


@pytest.mark.parametrize("n,R,force_step", [(1, 5, False), (17, 33, False), (70, 100, True),
                                           (130, 70, True), (300, 130, True)])
def test_fp64_ragged_shapes(nmfa, n, R, force_step):
    """Ragged spins and replicas (not multiples of the 16/64 tiles), a single spin, fields. The
    per-iteration FP64 kernel works on 128-row x 64-replica workgroup tiles: n = 300, R = 130 spans
    3 x 3 of them with ragged last tiles."""
    inst = instances.gnp(n, 0.5, 3) if n > 1 else instances.Instance(np.zeros((1, 1)), np.zeros(1), "one")
    h = np.round(instances.gaussian_fields(n, 2.0, 4))
    inst.h = h
    t_f, seed = 120, 5
    g = _run(nmfa, inst, "fp64", R, t_f, seed, record=40, force_step=force_step)
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=R, seed=seed, record=40)
    assert np.max(np.abs(g["traj"] - otraj)) <= 1e-9
    assert np.array_equal(g["E_int"], oracle.energies_int(inst.J, inst.h, g["spins"]))


def test_fp64_negated_noise_is_exact_negation(nmfa):
    inst = instances.sk(24, 4)
    a = _run(nmfa, inst, "fp64", 32, 60, 11, record=60)
    b = _run(nmfa, inst, "fp64", 32, 60, 11, record=60, negate_noise=True)
    assert np.array_equal(a["traj"], -b["traj"])


def test_noiseless_zero_field_reads_plus_one(nmfa):
    inst = instances.sk(12, 1)
    for prec in ("fp64", "fp32", "bf16"):
        g = _run(nmfa, inst, prec, 20, 50, 3, sigma=0.0)
        assert np.all(g["state"] == 0.0) and np.all(g["spins"] == 1)


# --------------------------------------------------------------------------------------------
# FP32 path (Moebius ladder N=100, R=4096, t_f=1000)
# --------------------------------------------------------------------------------------------

def test_fp32_moebius100(nmfa):
    inst = instances.moebius_ladder(100)
    R, t_f, seed = 4096, 1000, 7
    g = _run(nmfa, inst, "fp32", R, t_f, seed, record=20)
    sub = [0, 1, 15, 16, 1000, 4095]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:20], replicas=sub, seed=seed,
                                record=20)
    assert np.max(np.abs(g["traj"][:, sub, :] - otraj)) <= 1e-4
    assert np.array_equal(g["E_int"], oracle.energies_int(inst.J, inst.h, g["spins"]))
    # success probability at the exact ground energy -146 against the FP64 oracle
    Ro = 512
    spins_o, _, _ = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f), R=Ro, seed=seed)
    p_o = stats.success_probability(oracle.energies(inst.J, inst.h, spins_o), -146)
    p_g = stats.success_probability(g["E"], -146)
    assert stats.within_two_se(p_g, R, p_o, Ro), (p_g, p_o)


# --------------------------------------------------------------------------------------------
# BF16 and FP8-J paths
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["bf16", "fp8j_bf16s"])
def test_bf16_early_trajectory_sk100(nmfa, precision):
    inst = instances.sk(100, 1)
    R, t_f, seed = 256, 1000, 3
    g = _run(nmfa, inst, precision, R, t_f, seed, record=10)
    sub = [0, 5, 100, 255]
    _, _, otraj = oracle.anneal(inst.J, inst.h, oracle.schedule(t_f)[:10], replicas=sub, seed=seed,
                                record=10)
    assert np.max(np.abs(g["traj"][:, sub, :] - otraj)) <= 5e-3
    assert np.array_equal(g["E_int"], oracle.energies_int(inst.J, inst.h, g["spins"]))


def test_bf16_success_vs_fp64_sk100(nmfa):
    """Dense SK N=100: BF16 MFMA with FP32 accumulation vs the FP64 GPU path (R=16384 each)."""
    inst = instances.sk(100, 1)
    R, t_f = 16384, 1000
    f64 = _run(nmfa, inst, "fp64", R, t_f, 1001)
    b16 = _run(nmfa, inst, "bf16", R, t_f, 1002)
    target = min(f64["E"].min(), b16["E"].min())
    p64 = stats.success_probability(f64["E"], target)
    p16 = stats.success_probability(b16["E"], target)
    assert stats.within_two_se(p16, R, p64, R), (p16, p64)
    # energy means within 4 standard errors
    se = np.sqrt(f64["E"].var() / R + b16["E"].var() / R)
    assert abs(f64["E"].mean() - b16["E"].mean()) <= 4 * se


# --------------------------------------------------------------------------------------------
# invariances on the GPU
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("precision,force_step", [("fp64", False), ("bf16", False), ("fp32", True)])
def test_replica_prefix_and_resume(nmfa, precision, force_step):
    inst = instances.sk(40, 6)
    t_f, seed = 300, 21
    with nmfa.Solver(inst.J, inst.h, precision=precision, force_step=force_step) as s:
        s.anneal(48, t_f, seed)
        full48 = s.state()
        s.anneal(17, t_f, seed)
        full17 = s.state()
        s.anneal_range(17, t_f, 1, 120, seed)
        s.anneal_range(17, t_f, 121, t_f, seed)
        resumed = s.state()
    assert np.array_equal(full48[:17], full17)
    assert np.array_equal(resumed, full17)


def test_energies_of_exact(nmfa):
    rng = np.random.default_rng(5)
    for inst, h in [(instances.sk(37, 2), None), (instances.gnp(300, 0.5, 1), None),
                    (instances.random_regular(200, 5, 3), np.round(instances.gaussian_fields(200, 3, 1))),
                    (instances.sk(64, 9), instances.gaussian_fields(64, 0.5, 2))]:
        if h is not None:
            inst.h = h
        spins = rng.choice(np.array([-1, 1], dtype=np.int8), size=(20, inst.n))
        with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
            E, Ei = s.energies_of(spins)
        Eo = oracle.energies(inst.J, inst.h, spins)
        assert np.array_equal(E, Eo)
        if h is None or np.all(h == np.round(h)):
            assert np.array_equal(Ei, oracle.energies_int(inst.J, inst.h, spins))


def test_exact_energies_beyond_int8_couplings(nmfa):
    """Integral couplings outside the int8 range (|J| up to 300) still give exact integer energies
    (Eq. 1), through the FP64 energy kernel, for the readout and for given spin vectors."""
    inst = instances.sk(50, 12)
    rng = np.random.Generator(np.random.PCG64(3))
    W = np.triu(rng.integers(-300, 301, (50, 50)).astype(np.float64), 1)
    J = W + W.T
    h = np.round(instances.gaussian_fields(50, 40.0, 4))
    with nmfa.Solver(J, h, precision="fp64") as s:
        s.anneal(40, 200, 9)
        spins = s.spins()
        E, Ei = s.energies()
        E2, Ei2 = s.energies_of(-spins)
    assert np.array_equal(Ei, oracle.energies_int(J, h, spins))
    assert np.array_equal(E, Ei.astype(np.float64))
    assert np.array_equal(Ei2, oracle.energies_int(J, h, -spins))
    assert inst.n == 50
