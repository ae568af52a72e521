"""A run recorded into a HIP graph and replayed gives the eager run's results, bit for bit.

Each case runs one eager anneal (which also allocates the run buffers and uploads the schedule),
records the same call into a graph on a side stream, and then replays the graph three times with
eager anneals of other seeds in between, checking every replay's energies and spins against the
first eager run. The cases cover every kernel path: the persistent small-N kernel (BF16 and
FP64), the group kernels (register-J with BF16 and with FP8 spins, LDS-J; a zero-fill kernel
clears their control block inside the run), the sparse kernels (register and generic), and the
per-iteration kernels (tiled BF16, tiled FP64 and plain FP32). A last test checks that a replayed group-kernel
run whose abort word is set is reported when its results are read.
"""
import numpy as np
import pytest

import instances

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_08422_amd import nmfa as m

    return m, torch


def _replays_match(nmfa, torch, inst, R, t_f, seed, precision="bf16", **kw):
    with nmfa.Solver(inst.J, inst.h, precision=precision, **kw) as s:
        s.anneal(R, t_f, seed)
        torch.cuda.synchronize()
        E_ref = s.energies()[0].copy()
        sp_ref = s.spins()
        path = s.info()["path"]
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            s.anneal(R, t_f, seed, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        for k in range(3):
            s.anneal(R, t_f, seed + 1 + k)
            torch.cuda.synchronize()
            assert not np.array_equal(s.spins(), sp_ref)  # the eager run in between left other spins
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(s.energies()[0], E_ref), (path, k)
            assert np.array_equal(s.spins(), sp_ref), (path, k)
        return path


def test_graph_replay_small_kernel(env):
    nmfa, torch = env
    assert _replays_match(nmfa, torch, instances.sk(100, 41), 256, 300, 77) == "persistent"


def test_graph_replay_group_kernel(env):
    nmfa, torch = env
    assert _replays_match(nmfa, torch, instances.sk(1000, 42), 192, 200, 78).startswith("xcd_rj")


def test_graph_replay_sparse_kernel(env):
    nmfa, torch = env
    assert _replays_match(nmfa, torch, instances.random_regular(1200, 3, 43), 128, 200, 79) == "sparse_rq"


def test_graph_replay_tiled_step_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.sk(640, 44), 128, 60, 80, force_step=True)
    assert path == "step"


def test_graph_replay_small_kernel_fp64(env):
    nmfa, torch = env
    assert _replays_match(nmfa, torch, instances.sk(60, 45), 64, 150, 81, precision="fp64") == "persistent"


def test_graph_replay_lds_j_group_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.sk(700, 46), 200, 120, 82, force_xcd=True, force_lds_j=True)
    assert path in ("xcd", "xcd_fenced")


def test_graph_replay_fp8_spin_group_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.gnp(900, 0.5, 47), 128, 150, 83, precision="fp8j_fp8s")
    assert path.startswith("xcd_rj")


def test_graph_replay_generic_sparse_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.random_regular(1000, 4, 48), 96, 120, 84, sparse_generic=True)
    assert path == "sparse"


def test_graph_replay_fp64_tiled_step_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.sk(300, 51), 100, 40, 86, precision="fp64", force_step=True)
    assert path == "step"


def test_graph_replay_fp32_step_kernel(env):
    nmfa, torch = env
    path = _replays_match(nmfa, torch, instances.sk(300, 49), 100, 40, 85, precision="fp32", force_step=True)
    assert path == "step"


def test_abort_of_a_replayed_group_run_is_reported(env):
    """The group kernels' abort word is read whenever results are read, also after a replay that
    did not go through the library's own launch call. The word is set from the host (as a timed-out
    barrier would set it); no kernel is made to time out."""
    nmfa, torch = env
    inst = instances.sk(1000, 50)
    R, t_f, seed = 128, 100, 86
    with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
        s.anneal(R, t_f, seed)
        torch.cuda.synchronize()
        E_ref = s.energies()[0].copy()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            s.anneal(R, t_f, seed, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(s.energies()[0], E_ref)  # a clean replay reads fine (twice)
        assert np.array_equal(s.energies()[0], E_ref)
        s.debug_raise_abort()
        with pytest.raises(nmfa.NmfaError) as ei:
            s.energies()
        assert ei.value.code == nmfa.NMFA_EDEVICE
        # a new run from t = 1 clears the control block again
        s.anneal(R, t_f, seed)
        assert np.array_equal(s.energies()[0], E_ref)
