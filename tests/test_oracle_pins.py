"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each test checks an oracle function against something the paper or mathematics fixes -- a
published known-answer vector, a closed form, an invariant, an independent brute force -- so that
a plausible slip in the oracle (a dropped term, a wrong sign or index, a transposed operand)
fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import stats as sps

import instances
import oracle
from oracle import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------------------------
# Noise: Philox4x32-10 and the Gaussian transform
# --------------------------------------------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            words = [int(w, 16) for w in line.split()]
            rows.append((words[0:4], words[4:6], tuple(words[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert oracle.philox4x32_10(ctr, key) == expect


def test_box_muller_invariants():
    """z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi) for the Philox words."""
    for seed, q, r, t in [(1, 0, 0, 1), (2**40 + 5, 7, 3, 999), (12345, 123, 4095, 5000)]:
        key = [seed & 0xFFFFFFFF, seed >> 32]
        x = oracle.philox4x32_10([q, r, t, 0], key)
        z = oracle.gauss4(seed, q, r, t)
        for pair in range(2):
            u0 = (x[2 * pair] + 0.5) / 2**32
            u1 = (x[2 * pair + 1] + 0.5) / 2**32
            z0, z1 = z[2 * pair], z[2 * pair + 1]
            assert math.isclose(z0 * z0 + z1 * z1, -2.0 * math.log(u0), rel_tol=1e-13)
            ang = math.atan2(z1, z0) % (2 * math.pi)
            d = abs(ang - 2 * math.pi * u1)
            assert min(d, 2 * math.pi - d) < 1e-10


def _box_muller_lane(words, lane):
    """Lane `lane` of the Box-Muller transform (Box & Muller 1958) of four Philox words:
    (u0, u1) -> lanes 0, 1 and (u2, u3) -> lanes 2, 3 with u = (x + 1/2) / 2^32."""
    pair = lane // 2
    u0 = (words[2 * pair] + 0.5) / 2**32
    u1 = (words[2 * pair + 1] + 0.5) / 2**32
    rho = math.sqrt(-2.0 * math.log(u0))
    theta = 2.0 * math.pi * u1
    return rho * math.cos(theta) if lane % 2 == 0 else rho * math.sin(theta)


_NOISE_CASES = [(1, 1, 0, 0), (1, 1, 0, 3), (2**40 + 5, 17, 3, 6), (12345, 5000, 4095, 1999),
                (0xFFFFFFFFFFFF, 2, 1, 9), (77, 333, 700, 14), (9, 4, 9, 1)]


@pytest.mark.parametrize("seed,t,r,i", _NOISE_CASES)
def test_noise_counter_mapping(seed, t, r, i):
    """The noise of spin i, replica r, iteration t (1-based) is lane i mod 4 of the Gaussians of
    counter (floor(i/4), r, t, 0) under key (seed low word, seed high word) (the reading of the
    unspecified N(0, sigma) source of Sec. II). Rebuilt here from the known-answer-pinned
    generator: a lane swap within the quad, a 0-based t, or r and t exchanged in the counter
    each give a different value."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    words = oracle.philox4x32_10([i // 4, r, t, 0], key)
    expect = _box_muller_lane(words, i % 4)
    got = oracle.noise(seed, t, r, i)
    assert math.isclose(got, expect, rel_tol=1e-12, abs_tol=1e-12)
    mutants = [
        _box_muller_lane(words, (i % 4) ^ 1),                                      # lanes swapped
        _box_muller_lane(oracle.philox4x32_10([i // 4, r, t - 1, 0], key), i % 4),  # t counted from 0
        _box_muller_lane(oracle.philox4x32_10([i // 4, t, r, 0], key), i % 4),      # r and t exchanged
        _box_muller_lane(oracle.philox4x32_10([i, r, t, 0], key), i % 4),           # spin, not quad, index
    ]
    if r == t:
        mutants.pop(2)  # exchanging equal r and t changes nothing
    if i == 0:
        mutants.pop()  # quad and spin index coincide
    for m in mutants:
        assert abs(m - got) > 1e-6


def test_noise_is_standard_normal():
    """Moments and a Kolmogorov-Smirnov test over many (t, r, i) draws."""
    rng = np.random.default_rng(0)
    zs = []
    for _ in range(40000):
        t, r, i = int(rng.integers(1, 5000)), int(rng.integers(0, 16384)), int(rng.integers(0, 2000))
        zs.append(oracle.noise(77, t, r, i))
    zs = np.array(zs)
    n = zs.size
    assert abs(zs.mean()) < 5 / math.sqrt(n)
    assert abs(zs.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert sps.kstest(zs, "norm").pvalue > 1e-3


def test_noise_streams_are_distinct():
    """Adjacent spins, replicas, iterations and seeds get different, uncorrelated draws."""
    base = np.array([oracle.noise(5, 10, r, i) for r in range(64) for i in range(64)])
    shifted_i = np.array([oracle.noise(5, 10, r, i + 1) for r in range(64) for i in range(64)])
    shifted_r = np.array([oracle.noise(5, 10, r + 1, i) for r in range(64) for i in range(64)])
    shifted_t = np.array([oracle.noise(5, 11, r, i) for r in range(64) for i in range(64)])
    other_seed = np.array([oracle.noise(6, 10, r, i) for r in range(64) for i in range(64)])
    for other in (shifted_i, shifted_r, shifted_t, other_seed):
        assert abs(np.corrcoef(base, other)[0, 1]) < 0.08
        assert np.mean(base == other) < 0.01


# --------------------------------------------------------------------------------------------
# Setup: normaliser and schedule
# --------------------------------------------------------------------------------------------

def test_normaliser_closed_forms():
    n = 37
    assert np.allclose(oracle.normalisers(instances.sk(n, 3).J), math.sqrt(n - 1), rtol=0, atol=1e-14)
    assert np.allclose(oracle.normalisers(instances.moebius_ladder(20).J), math.sqrt(3), atol=1e-14)
    reg = instances.random_regular(30, 5, 2)
    assert np.allclose(oracle.normalisers(reg.J), math.sqrt(5), atol=1e-14)
    g = instances.gnp(40, 0.5, 1)
    deg = g.J.sum(axis=1)
    h = np.linspace(-2, 2, 40)
    assert np.allclose(oracle.normalisers(g.J, h), np.sqrt(deg + h * h), atol=1e-14)


def test_schedule_knots_and_geometric_midpoints():
    knots = ((0.0, 8.0), (0.5, 2.0), (1.0, 0.5))
    # u = 0, .25, .5, .75, 1: knots exactly, geometric means in between
    assert np.array_equal(oracle.schedule(5, knots), [8.0, 4.0, 2.0, 1.0, 0.5])
    T = oracle.schedule(1000)
    assert T[0] == 10.0 and T[-1] == 0.05
    assert np.all(np.diff(T) < 0)
    assert oracle.schedule(1, knots)[0] == 8.0


def test_schedule_rejects_bad_knots():
    with pytest.raises(ValueError):
        oracle.schedule(10, ((0.0, 1.0), (0.5, -1.0), (1.0, 0.5)))
    with pytest.raises(ValueError):
        oracle.schedule(10, ((0.0, 1.0), (0.7, 1.0), (0.6, 0.5), (1.0, 0.1)))


# --------------------------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------------------------

def test_decoupled_noiseless_geometric_series():
    """J = 0, sigma = 0, constant T: s_t = c (1 - (1 - alpha)^t), c = -tanh(sign(h_i) / T)."""
    n, t_f, alpha, T0 = 6, 40, 0.15, 0.7
    h = np.array([1.0, -2.0, 0.5, -0.25, 3.0, -1.0])
    J = np.zeros((n, n))
    _, _, traj = oracle.anneal(J, h, np.full(t_f, T0), R=2, seed=1, alpha=alpha, sigma=0.0,
                               record=t_f)
    c = -np.tanh(np.sign(h) / T0)
    for t in range(1, t_f + 1):
        expect = c * (1.0 - (1.0 - alpha) ** t)
        assert np.allclose(traj[t - 1], expect[None, :], rtol=0, atol=1e-13)


def test_alpha_one_uses_the_noise_of_each_iteration():
    """J = 0, alpha = 1: s after iteration t is -tanh((sign h_i + sigma z(t, r, i)) / T_t)."""
    n, t_f, sigma, seed = 9, 7, 0.3, 2024
    h = np.array([1, -1, 2, -3, 1, 1, -1, 4, -2], dtype=float)
    T = np.linspace(3.0, 0.5, t_f)
    _, _, traj = oracle.anneal(np.zeros((n, n)), h, T, R=3, seed=seed, alpha=1.0, sigma=sigma,
                               record=t_f)
    for t in range(1, t_f + 1):
        for r in range(3):
            z = np.array([oracle.noise(seed, t, r, i) for i in range(n)])
            expect = -np.tanh((np.sign(h) + sigma * z) / T[t - 1])
            assert np.allclose(traj[t - 1, r], expect, rtol=0, atol=1e-14)


def test_noiseless_zero_field_stays_at_zero_and_reads_plus_one():
    inst = instances.sk(12, 1)
    spins, s, _ = oracle.anneal(inst.J, inst.h, oracle.schedule(50), R=4, seed=3, sigma=0.0)
    assert np.all(s == 0.0)
    assert np.all(spins == 1)


def test_zero_normaliser_sees_only_noise():
    """An isolated spin with h_i = 0 has a zero normaliser; its field term is read as 0."""
    n, t_f = 4, 5
    J = np.zeros((n, n))
    J[0, 1] = J[1, 0] = 1.0
    h = np.zeros(n)
    T = np.full(t_f, 1.0)
    _, _, traj = oracle.anneal(J, h, T, R=1, seed=9, alpha=1.0, sigma=0.2, record=t_f)
    for t in range(1, t_f + 1):
        for i in (2, 3):
            assert traj[t - 1, 0, i] == pytest.approx(-math.tanh(0.2 * oracle.noise(9, t, 0, i)),
                                                      abs=1e-15)


def test_negated_noise_negates_the_trajectory_exactly():
    """At h = 0 the map is odd (tanh odd, field linear): z -> -z gives s -> -s bit for bit."""
    inst = instances.sk(24, 4)
    T = oracle.schedule(60)
    _, s_a, tr_a = oracle.anneal(inst.J, inst.h, T, R=5, seed=11, record=60)
    _, s_b, tr_b = oracle.anneal(inst.J, inst.h, T, R=5, seed=11, record=60, negate_noise=True)
    assert np.array_equal(tr_a, -tr_b)
    assert np.array_equal(s_a, -s_b)


@pytest.mark.parametrize("scale", [2.0, 0.25, 8.0])
def test_power_of_two_scaling_is_exact(scale):
    """The normalisation makes the dynamics invariant under (h, J) -> c (h, J), c > 0; for c a
    power of two every rounding is unchanged, so the trajectory is bit-identical."""
    inst = instances.gnp(30, 0.5, 2)
    h = instances.gaussian_fields(30, 0.5, 5)
    T = oracle.schedule(80)
    _, s_a, tr_a = oracle.anneal(inst.J, h, T, R=3, seed=1, record=80)
    _, s_b, tr_b = oracle.anneal(inst.J * scale, h * scale, T, R=3, seed=1, record=80)
    assert np.array_equal(tr_a, tr_b)
    assert np.array_equal(s_a, s_b)


def test_replica_prefix_and_subset_invariance():
    inst = instances.sk(16, 2)
    T = oracle.schedule(100)
    sp8, s8, _ = oracle.anneal(inst.J, inst.h, T, R=8, seed=21)
    sp3, s3, _ = oracle.anneal(inst.J, inst.h, T, R=3, seed=21)
    assert np.array_equal(s8[:3], s3)
    sps_, ss, _ = oracle.anneal(inst.J, inst.h, T, replicas=[6, 1], seed=21)
    assert np.array_equal(ss, s8[[6, 1]])
    assert np.array_equal(sps_, sp8[[6, 1]])


def test_resume_is_exact():
    inst = instances.sk(16, 5)
    T = oracle.schedule(120)
    _, s_full, _ = oracle.anneal(inst.J, inst.h, T, R=4, seed=8)
    _, s_mid, _ = oracle.anneal(inst.J, inst.h, T[:50], R=4, seed=8)
    _, s_res, _ = oracle.anneal(inst.J, inst.h, T, R=4, seed=8, t_first=51, s_init=s_mid)
    assert np.array_equal(s_full, s_res)


def test_ferromagnet_aligns():
    """J_ij = -1 (ferromagnetic under minimisation of Eq. 1): every sample ends fully aligned.
    A wrong sign in the Boltzmann step would anti-align instead."""
    n = 10
    J = -(np.ones((n, n)) - np.eye(n))
    spins, _, _ = oracle.anneal(J, None, oracle.schedule(300), R=32, seed=4)
    assert np.all(np.abs(spins.sum(axis=1)) == n)


def test_finds_brute_force_ground_states():
    """On small SK instances NMFA reaches the exhaustive-search ground energy in most samples
    (random guessing would succeed with probability 2^(1-n))."""
    for seed in (1, 2, 3):
        inst = instances.sk(14, seed)
        E0, _ = oracle.ground_state(inst.J, inst.h)
        spins, _, _ = oracle.anneal(inst.J, inst.h, oracle.schedule(400), R=64, seed=100 + seed)
        E = oracle.energies(inst.J, inst.h, spins)
        assert np.all(E >= E0 - 1e-9)
        assert stats.success_probability(E, E0) > 0.5


def test_fields_break_the_flip_symmetry_in_the_right_direction():
    """Strong uniform field h_i = +5 and no couplings: every spin ends at -1 (H has +h s)."""
    n = 8
    spins, _, _ = oracle.anneal(np.zeros((n, n)), np.full(n, 5.0), oracle.schedule(200), R=8,
                                seed=2)
    assert np.all(spins == -1)


# --------------------------------------------------------------------------------------------
# Energies, cuts, ground states
# --------------------------------------------------------------------------------------------

def _golden_energy_rows():
    rows = []
    with open(os.path.join(GOLDEN, "energy_hand_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, n, up, h, s, E = [p.strip() for p in line.split("|")]
            n = int(n)
            J = np.zeros((n, n))
            vals = [float(v) for v in up.split()]
            k = 0
            for i in range(n):
                for j in range(i + 1, n):
                    J[i, j] = J[j, i] = vals[k]
                    k += 1
            hv = np.array([float(v) for v in h.split()])
            sv = np.array([1 if c == "+" else -1 for c in s.split()], dtype=np.int8)
            rows.append(pytest.param(J, hv, sv, float(E), id=name))
    return rows


@pytest.mark.parametrize("J,h,s,E", _golden_energy_rows())
def test_energy_hand_examples(J, h, s, E):
    assert oracle.energy(J, h, s) == E
    assert oracle.energy_int(J, h, s) == int(E)


def _python_energy(J, h, s):
    n = len(s)
    return sum(J[i][j] * s[i] * s[j] for i in range(n) for j in range(i + 1, n)) + sum(
        h[i] * s[i] for i in range(n))


def test_energy_flip_symmetry_and_python_enumeration():
    inst = instances.sk(11, 7)
    h = np.round(instances.gaussian_fields(11, 2.0, 3))
    for bits in itertools.islice(itertools.product((1, -1), repeat=11), 0, 2048, 37):
        s = np.array(bits, dtype=np.int8)
        assert oracle.energy(inst.J, None, s) == oracle.energy(inst.J, None, -s)
        assert oracle.energy_int(inst.J, h, s) == _python_energy(inst.J, h, s)


def test_energy_int_rejects_fractional_couplings():
    J = np.array([[0, 0.5], [0.5, 0]])
    with pytest.raises(ValueError):
        oracle.energy_int(J, None, np.array([1, 1], dtype=np.int8))


def test_cut_identity():
    """MAX-CUT value = (sum of weights - Ising energy) / 2 for J = W, h = 0."""
    g = instances.gnp(25, 0.5, 9)
    W_tot = np.triu(g.J, 1).sum()
    rng = np.random.default_rng(1)
    for _ in range(50):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=25)
        assert oracle.cut(g.J, s) == (W_tot - oracle.energy(g.J, None, s)) / 2


def _python_ground(J, h):
    n = J.shape[0]
    best = None
    for bits in itertools.product((1, -1), repeat=n):
        E = _python_energy(J, h, bits)
        best = E if best is None or E < best else best
    return best


@pytest.mark.parametrize("n,seed,with_h", [(6, 1, False), (8, 2, True), (10, 3, False), (9, 4, True)])
def test_ground_state_matches_python_enumeration(n, seed, with_h):
    inst = instances.sk(n, seed)
    h = np.round(instances.gaussian_fields(n, 1.5, seed)) if with_h else np.zeros(n)
    E0, best = oracle.ground_state(inst.J, h)
    assert E0 == _python_ground(inst.J, h)
    assert oracle.energy(inst.J, h, best) == E0


@pytest.mark.parametrize("n", [6, 8, 10, 12, 14, 16, 18, 20])
def test_moebius_ladder_closed_form(n):
    """Moebius ladder with J = +1 on edges: bipartite when n/2 is odd (all 3n/2 edges cut,
    E0 = -3n/2); otherwise two edges must stay uncut (E0 = -3n/2 + 4)."""
    inst = instances.moebius_ladder(n)
    E0, best = oracle.ground_state(inst.J, inst.h)
    expect = -1.5 * n + (4 if (n // 2) % 2 == 0 else 0)
    assert E0 == expect
    assert oracle.cut(inst.J, best) == 1.5 * n - (2 if (n // 2) % 2 == 0 else 0)


def test_ground_state_special_cases():
    tri = np.ones((3, 3)) - np.eye(3)
    assert oracle.ground_state(tri)[0] == -1.0
    n = 9
    ferro = -(np.ones((n, n)) - np.eye(n))
    E0, best = oracle.ground_state(ferro)
    assert E0 == -n * (n - 1) / 2 and abs(int(best.sum())) == n


def test_tts99():
    assert stats.tts99(1.0, 0.0) == float("inf")
    assert stats.tts99(2.0, 0.995) == 2.0
    # p = 0.9: ln(0.01)/ln(0.1) = 2 samples
    assert stats.tts99(3.0, 0.9) == pytest.approx(6.0)


def test_uniform_mode_two_cycle_closed_form():
    """Complete graph J = 1, uniform field h = 0.5, sigma = 0, T = 1e-4 (saturated tanh): all spins
    share m_t with m_{t+1} = (1 - alpha) m_t - alpha sign(h + (n-1) m_t), which converges to the
    2-cycle -alpha/(2-alpha) (odd t) <-> +alpha/(2-alpha) (even t). This is the period-2
    instability of the uniform mode that dense antiferromagnetic instances fall into."""
    n, alpha, t_f = 50, 0.15, 200
    J = np.ones((n, n)) - np.eye(n)
    h = np.full(n, 0.5)
    _, _, traj = oracle.anneal(J, h, np.full(t_f, 1e-4), R=1, seed=1, alpha=alpha, sigma=0.0,
                               record=t_f)
    amp = alpha / (2 - alpha)
    assert traj[0, 0, 0] == -alpha  # first step: -alpha * sign(h)
    assert np.allclose(traj[-1], amp, rtol=0, atol=1e-12)      # t = 200 (even)
    assert np.allclose(traj[-2], -amp, rtol=0, atol=1e-12)     # t = 199 (odd)
