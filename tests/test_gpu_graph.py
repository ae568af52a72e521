"""A run recorded into a HIP graph and replayed gives the eager run's results, bit for bit.

Each case runs one eager anneal (which also allocates the run buffers and uploads the schedule),
records the same call into a graph on a side stream, and then replays the graph three times with
eager anneals of other seeds in between, checking every replay's energies and spins against the
first eager run. The cases cover the persistent small-N kernel, the XCD-group kernel (whose
control block a zero-fill kernel clears inside the run), the sparse register kernel and the
per-iteration tiled kernel.
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


def _replays_match(nmfa, torch, inst, R, t_f, seed, **kw):
    with nmfa.Solver(inst.J, inst.h, precision="bf16", **kw) as s:
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
