"""nmfa_energies_of_noalloc (device buffers, scratch from a fixed device array) against
nmfa_energies_of on the same spins: integer energies bit-exact, FP64 energies identical (the same
kernels run), on two calls in a row, the second with fewer replicas, so that the second call
reuses scratch that the first left behind. Also at the largest replica count the scratch admits
for n = 2000, and the rejection of one more replica block."""
import numpy as np
import pytest

import instances
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa

    return nmfa, torch


def _signs(R, n, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((R, n)) < 0.5, -1, 1).astype(np.int8)


def _noalloc(nmfa, torch, solver, spins, with_int=True):
    R = spins.shape[0]
    d_s = torch.from_numpy(spins).cuda()
    d_E = torch.full((R,), -7.5, dtype=torch.float64, device="cuda")
    d_Ei = torch.full((R,), -7, dtype=torch.int64, device="cuda") if with_int else None
    solver.energies_of_noalloc(R, d_s.data_ptr(), d_E.data_ptr(), d_Ei.data_ptr() if with_int else None)
    torch.cuda.synchronize()
    return d_E.cpu().numpy(), (d_Ei.cpu().numpy() if with_int else None)


CASES = {
    # integral J (|J| <= 127: the int8 matrix-core kernels and the scratch array)
    "sk300_int8": (lambda: instances.sk(300, 11), None, (700, 130)),
    "sk200_int_fields": (lambda: instances.sk(200, 12),
                         lambda n: np.random.default_rng(5).integers(-3, 4, n).astype(float), (257, 64)),
    "sk200_real_fields": (lambda: instances.sk(200, 13), lambda n: instances.gaussian_fields(n, 0.5, 6), (300, 33)),
    # non-integral J: the FP64 energy kernel, no scratch; E_int reported as 0
    "scaled_sk150": (lambda: instances.sk(150, 14), None, (190, 65)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_matches_energies_of_twice(env, name):
    nmfa, torch = env
    make, hfun, Rs = CASES[name]
    inst = make()
    J = inst.J * (0.37 if name == "scaled_sk150" else 1.0)
    h = hfun(inst.n) if hfun else None
    print(f"[no_alloc] case={name} n={inst.n} R={Rs}", flush=True)
    with nmfa.Solver(J, h, precision="fp32") as s:
        for k, R in enumerate(Rs):
            spins = _signs(R, inst.n, 100 + k)
            E_ref, Ei_ref = s.energies_of(spins)
            E, Ei = _noalloc(nmfa, torch, s, spins)
            assert np.array_equal(Ei, Ei_ref), f"call {k}: integer energies differ"
            assert np.array_equal(E, E_ref), f"call {k}: energies differ"
            sub = slice(0, 16)
            if name in ("scaled_sk150", "sk200_real_fields"):
                assert not Ei.any()  # not exact integers: reported as 0
                assert np.allclose(E[sub], oracle.energies(J, h, spins[sub]), rtol=0, atol=1e-9)
            else:
                assert np.array_equal(Ei[sub], oracle.energies_int(J, h, spins[sub]))
            E2, _ = _noalloc(nmfa, torch, s, spins, with_int=False)
            assert np.array_equal(E2, E_ref)


def _scratch_need(R, n):
    """Bytes of scratch the int8 energy kernels take for R replicas of n spins."""
    sp = -(-R // 64) * 64 * (-(-n // 64) * 64)
    return -(-sp // 256) * 256 + 8 * R


def test_noalloc_at_the_scratch_limit(env):
    nmfa, torch = env
    inst = instances.gnp(2000, 0.5, 21)
    limit = 16 << 20
    # n = 2000 -> 2048 padded columns: 8128 replicas fit in 16 MiB, 8129 (one more block of 64) do not
    R_max = 8128
    assert _scratch_need(R_max, 2000) <= limit < _scratch_need(R_max + 1, 2000)
    print(f"[no_alloc] scratch limit n=2000 R={R_max}", flush=True)
    with nmfa.Solver(inst.J, None, precision="fp8j_bf16s") as s:
        spins = _signs(R_max, inst.n, 7)
        E_ref, Ei_ref = s.energies_of(spins)
        E, Ei = _noalloc(nmfa, torch, s, spins)
        assert np.array_equal(Ei, Ei_ref) and np.array_equal(E, E_ref)
        small = _signs(100, inst.n, 8)
        E_ref, Ei_ref = s.energies_of(small)
        E, Ei = _noalloc(nmfa, torch, s, small)
        assert np.array_equal(Ei, Ei_ref) and np.array_equal(E, E_ref)
        assert np.array_equal(Ei[:4], oracle.energies_int(inst.J, None, small[:4]))
        # one replica more does not fit: rejected on the host before any launch (the buffers
        # passed are still large enough for R_max + 1 replicas)
        big_s = torch.ones((R_max + 1, inst.n), dtype=torch.int8, device="cuda")
        big_E = torch.zeros(R_max + 1, dtype=torch.float64, device="cuda")
        with pytest.raises(nmfa.NmfaError) as ei:
            s.energies_of_noalloc(R_max + 1, big_s.data_ptr(), big_E.data_ptr(), None)
        assert ei.value.code == nmfa.NMFA_EINVAL and "scratch" in str(ei.value)
        torch.cuda.synchronize()
