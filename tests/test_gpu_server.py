"""Serving (continuous batching) on the GPU through the C ABI.

* each request's result is bit-identical alone (nmfa_anneal) and inside a mixed stream served
  with admission by a memory budget, chunked rounds and batched launches;
* admission never holds more than the budget; a request larger than the budget fails cleanly;
* requests that arrive while others run are admitted and finish;
* cancellation of queued and running requests.
"""
import time

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


def _mix():
    jobs = []
    for k, (kind, n, R, t_f) in enumerate([("sk", 60, 64, 500), ("reg", 150, 128, 700), ("sk", 100, 256, 600),
                                           ("sk", 300, 64, 400), ("reg", 40, 96, 900), ("sk", 700, 128, 300),
                                           ("sk", 20, 33, 450), ("reg", 256, 64, 520)]):
        inst = instances.sk(n, 10 + k) if kind == "sk" else instances.random_regular(n, 3 + k % 5, 20 + k)
        if k % 3 == 1:
            inst.h = instances.gaussian_fields(inst.n, 0.5, 5 + k)
        jobs.append((inst, R, t_f, 7000 + k))
    return jobs


def test_alone_equals_in_the_mix(nmfa):
    jobs = _mix()
    alone = []
    for inst, R, t_f, seed in jobs:
        with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
            s.anneal(R, t_f, seed)
            alone.append((s.energies()[0], s.spins()))
    with nmfa.Server(precision="bf16", hbm_budget_bytes=64 << 20, max_active=4, chunk_iters=128) as srv:
        tickets = []
        for k, (inst, R, t_f, seed) in enumerate(jobs):
            tickets.append(srv.submit(inst.J, inst.h, R, t_f, seed))
            if k == 3:
                time.sleep(0.05)  # later requests arrive while the first ones run
        for t in tickets:
            assert srv.wait(t, 120000)
        for (E, sp), t in zip(alone, tickets):
            res = srv.result(t, spins=True)
            assert np.array_equal(res["E"], E)
            assert np.array_equal(res["spins"], sp)
            assert res["latency_ms"] > 0
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0
        assert st["peak_bytes"] <= 64 << 20
        assert st["batched_launches"] >= 1 and st["rounds"] >= 2


def test_energies_in_the_mix_are_exact(nmfa):
    jobs = _mix()[:4]
    with nmfa.Server(precision="bf16") as srv:
        tickets = [srv.submit(inst.J, inst.h, R, t_f, seed) for inst, R, t_f, seed in jobs]
        for (inst, R, t_f, seed), t in zip(jobs, tickets):
            assert srv.wait(t, 120000)
            res = srv.result(t, spins=True)
            assert np.array_equal(res["E"], oracle.energies(inst.J, inst.h, res["spins"]))


def test_budget_rejects_oversized_request(nmfa):
    inst = instances.sk(500, 1)
    with nmfa.Server(precision="bf16", hbm_budget_bytes=1 << 20) as srv:
        t = srv.submit(inst.J, inst.h, 1024, 100, 1)
        assert srv.wait(t, 60000)
        assert srv.poll(t) == nmfa.NMFA_ENOMEM
        with pytest.raises(nmfa.NmfaError):
            srv.result(t)


def test_cancel_queued_and_running(nmfa):
    big = instances.sk(2000, 2)
    small = instances.sk(200, 2)
    with nmfa.Server(precision="bf16", max_active=1, chunk_iters=20) as srv:
        t1 = srv.submit(big.J, big.h, 4096, 5000, 1)    # hundreds of rounds
        t2 = srv.submit(small.J, small.h, 64, 100, 2)
        srv.cancel(t2)  # still queued behind t1 (max_active = 1)
        assert srv.poll(t2) == nmfa.NMFA_ECANCELED
        deadline = time.time() + 60
        while srv.poll(t1) == nmfa.JOB_QUEUED and time.time() < deadline:
            time.sleep(0.001)
        assert srv.poll(t1) == nmfa.JOB_RUNNING
        srv.cancel(t1)
        assert srv.wait(t1, 60000)
        assert srv.poll(t1) == nmfa.NMFA_ECANCELED
        t3 = srv.submit(small.J, small.h, 64, 100, 3)
        assert srv.wait(t3, 60000) and srv.poll(t3) == nmfa.JOB_DONE
        assert srv.stats()["cancelled"] == 2


def test_large_jobs_side_by_side(nmfa):
    # dense group-kernel jobs, sparse jobs and small batched jobs in the same rounds, on four
    # streams: each result is the one the job gets alone, bit for bit
    specs = [("sk", 500, 96, 400), ("sk", 900, 128, 300), ("sk", 1300, 64, 350),
             ("reg", 600, 200, 380), ("reg", 1100, 64, 420), ("reg", 1500, 130, 300),
             ("sk", 120, 80, 300), ("reg", 200, 50, 360)]
    jobs = []
    for k, (kind, n, R, t_f) in enumerate(specs):
        inst = instances.sk(n, 60 + k) if kind == "sk" else instances.random_regular(n, 3 + k % 4, 70 + k)
        jobs.append((inst, R, t_f, 8100 + k))
    alone, paths = [], []
    for inst, R, t_f, seed in jobs:
        with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
            s.anneal(R, t_f, seed)
            alone.append(s.energies()[0])
            paths.append(s.info()["path"])
    assert {"xcd_rj", "xcd_rj_fenced"} & set(paths) and {"sparse_rq"} & set(paths) and "persistent" in paths
    with nmfa.Server(precision="bf16", max_active=64, chunk_iters=100) as srv:
        tickets = [srv.submit(inst.J, inst.h, R, t_f, seed) for inst, R, t_f, seed in jobs]
        for E, t in zip(alone, tickets):
            assert srv.wait(t, 120000)
            assert np.array_equal(srv.result(t)["E"], E)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0


def test_group_requests_side_by_side_with_capped_launches(nmfa):
    # several dense requests on the XCD-group kernels in the same rounds: they run on different
    # streams under per-stream workgroup budgets, and the largest (16 groups of 12 workgroups)
    # needs more than one launch under any budget below the whole chip; each result is the one
    # the request gets alone, bit for bit
    specs = [(1500, 1024, 260), (900, 512, 240), (2000, 300, 220), (1100, 64, 250), (700, 200, 230)]
    jobs = [(instances.sk(n, 90 + k), R, t_f, 9100 + k) for k, (n, R, t_f) in enumerate(specs)]
    alone = []
    for inst, R, t_f, seed in jobs:
        with nmfa.Solver(inst.J, inst.h, precision="bf16") as s:
            s.anneal(R, t_f, seed)
            assert s.info()["path"].startswith("xcd_rj")
            alone.append((s.energies()[0], s.spins()))
    with nmfa.Server(precision="bf16", max_active=64, chunk_iters=80) as srv:
        tickets = [srv.submit(inst.J, inst.h, R, t_f, seed) for inst, R, t_f, seed in jobs]
        for (E, sp), t in zip(alone, tickets):
            assert srv.wait(t, 120000)
            res = srv.result(t, spins=True)
            assert np.array_equal(res["E"], E)
            assert np.array_equal(res["spins"], sp)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0


def test_alone_equals_in_the_mix_on_jobs_sampled_from_the_serving_stream(nmfa):
    """100 requests sampled from the benchmark's 10,000-request Poisson stream (every 100th job:
    N in [50, 2000], half dense SK and half random d-regular graphs, fields on a quarter of them,
    R in {64 .. 1024}) with t_f capped at 250 to bound the runtime: each result is the one the
    request gets alone, bit for bit, served under the benchmark's 2 GiB admission budget."""
    import bench

    stream = instances.serving_stream(10000, 80.0, 6)  # the job mix does not depend on the rate
    sample = stream[::100]
    assert len(sample) == 100
    cache = bench._InstanceCache(instances)
    jobs = []
    for j in sample:
        J, h = cache.get(j)
        jobs.append((J, h, j.R, min(j.t_f, 250), j.noise_seed))
    kinds = {j.kind for j in sample}
    assert kinds == {"sk", "regular"} and any(j.with_fields for j in sample)
    alone = []
    for J, h, R, t_f, seed in jobs:
        with nmfa.Solver(J, h, precision="bf16") as s:
            s.anneal(R, t_f, seed)
            alone.append((s.energies()[0], s.spins()))
    print(f"[server] {len(jobs)} sampled jobs run alone", flush=True)
    with nmfa.Server(precision="bf16", hbm_budget_bytes=2 << 30, max_active=256, chunk_iters=100) as srv:
        tickets = []
        for k, (J, h, R, t_f, seed) in enumerate(jobs):
            tickets.append(srv.submit(J, h, R, t_f, seed))
            if k % 10 == 9:
                time.sleep(0.01)  # later requests arrive while earlier ones run
        for (E, sp), t in zip(alone, tickets):
            assert srv.wait(t, 300000)
            res = srv.result(t, spins=True)
            assert np.array_equal(res["E"], E)
            assert np.array_equal(res["spins"], sp)
            srv.release(t)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0
        assert st["peak_bytes"] <= 2 << 30
