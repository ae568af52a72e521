"""Seeded synthetic Ising instances, shared by the GPU library's tests/benchmarks and the oracle.

This module only *generates inputs*. It contains none of the annealing arithmetic, so both the
HIP path and the CPU oracle may take their inputs from it without sharing any of the method.

The instance classes are the ones the paper evaluates (Sec. III, the Fig. 4 caption and the
text that follows it):

* Sherrington-Kirkpatrick (SK): J_ij = +1 with probability 1/2, else -1, all pairs coupled.
* dense MAX-CUT: J_ij = 1 with probability p = 1/2, else 0 (an Erdos-Renyi graph G(N, p)).
* degree-3 MAX-CUT: every spin coupled to three others with J_ij = 1; the Moebius ladder used in
  the Fig. 3 example is one such graph.

The paper's own instance files are not available, so these generators produce instances of the
same classes and sizes from a seed. Couplings are returned as a dense, symmetric float64 matrix
with a zero diagonal (the Ising energy of Eq. 1 read over pairs i < j), and fields as float64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Instance",
    "sk",
    "moebius_ladder",
    "gnp",
    "random_regular",
    "gaussian_fields",
    "ServingJob",
    "serving_stream",
]


@dataclasses.dataclass
class Instance:
    """A dense Ising instance (h, J) plus a short description."""

    J: np.ndarray  # (n, n) float64, symmetric, zero diagonal
    h: np.ndarray  # (n,) float64
    name: str

    @property
    def n(self) -> int:
        return int(self.J.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _symmetrise_upper(upper: np.ndarray) -> np.ndarray:
    """Mirror the strict upper triangle of ``upper`` into a symmetric zero-diagonal matrix."""
    u = np.triu(upper, k=1)
    return (u + u.T).astype(np.float64)


def sk(n: int, seed: int) -> Instance:
    """SK instance: each pair i < j gets J_ij = +1 or -1 with probability 1/2 each; h = 0."""
    if n < 1:
        raise ValueError("n must be >= 1")
    g = _rng(seed)
    signs = np.where(g.random((n, n)) < 0.5, 1.0, -1.0)
    return Instance(_symmetrise_upper(signs), np.zeros(n), f"sk_n{n}_s{seed}")


def moebius_ladder(n: int) -> Instance:
    """Moebius ladder on n (even) spins: ring edges i--i+1 (mod n) and chords i--i+n/2; J = +1.

    This is a degree-3 graph; with J = +1 on edges and h = 0 minimising the Ising energy is the
    MAX-CUT problem on the ladder.
    """
    if n < 4 or n % 2:
        raise ValueError("the Moebius ladder needs an even n >= 4")
    J = np.zeros((n, n))
    for i in range(n):
        for j in ((i + 1) % n, (i + n // 2) % n):
            J[i, j] = 1.0
            J[j, i] = 1.0
    return Instance(J, np.zeros(n), f"moebius_n{n}")


def gnp(n: int, p: float, seed: int) -> Instance:
    """Dense MAX-CUT instance: each pair i < j is an edge (J_ij = 1) with probability p; h = 0."""
    if n < 1:
        raise ValueError("n must be >= 1")
    g = _rng(seed)
    edges = (g.random((n, n)) < p).astype(np.float64)
    return Instance(_symmetrise_upper(edges), np.zeros(n), f"gnp_n{n}_p{p}_s{seed}")


def random_regular(n: int, d: int, seed: int) -> Instance:
    """Sparse MAX-CUT instance: a uniformly random d-regular graph with J = 1 on its edges.

    If n*d is odd no such graph exists; one vertex is then dropped (n - 1 spins).
    """
    import networkx as nx  # graph sampling only

    if (n * d) % 2:
        n -= 1
    graph = nx.random_regular_graph(d, n, seed=int(seed))
    J = np.zeros((n, n))
    for a, b in graph.edges():
        J[a, b] = 1.0
        J[b, a] = 1.0
    return Instance(J, np.zeros(n), f"regular_n{n}_d{d}_s{seed}")


def gaussian_fields(n: int, std: float, seed: int) -> np.ndarray:
    """Local fields h_i drawn i.i.d. from a normal distribution with the given standard deviation."""
    return _rng(seed).normal(0.0, std, size=n)


@dataclasses.dataclass
class ServingJob:
    """One annealing request of the serving workload."""

    job_id: int
    arrival_s: float  # arrival time, seconds from the start of the stream
    kind: str  # "sk" or "regular"
    n: int
    degree: int  # 0 for dense SK
    with_fields: bool
    R: int
    t_f: int
    instance_seed: int
    noise_seed: int

    def instance(self) -> Instance:
        if self.kind == "sk":
            inst = sk(self.n, self.instance_seed)
        else:
            inst = random_regular(self.n, self.degree, self.instance_seed)
        if self.with_fields:
            inst.h = gaussian_fields(inst.n, 0.5, self.instance_seed + 7919)
        return inst


def serving_stream(
    n_requests: int,
    rate_per_s: float,
    seed: int,
    n_range: Tuple[int, int] = (50, 2000),
    r_choices: Tuple[int, ...] = (64, 128, 256, 512, 1024),
    tf_range: Tuple[int, int] = (500, 5000),
    degree_range: Tuple[int, int] = (3, 10),
    field_fraction: float = 0.25,
    max_n: Optional[int] = None,
) -> List[ServingJob]:
    """A Poisson stream of annealing requests with a mixed size, density, field and replica mix.

    Half of the jobs are dense SK instances and half are sparse random d-regular graphs; a
    fraction of them carry Gaussian local fields (std 0.5). Arrival gaps are exponential with
    the given rate.
    """
    g = _rng(seed)
    jobs: List[ServingJob] = []
    t = 0.0
    hi_n = n_range[1] if max_n is None else min(n_range[1], max_n)
    for k in range(n_requests):
        t += float(g.exponential(1.0 / rate_per_s)) if rate_per_s > 0 else 0.0
        n = int(g.integers(n_range[0], hi_n + 1))
        dense = bool(g.random() < 0.5)
        degree = 0 if dense else int(g.integers(degree_range[0], degree_range[1] + 1))
        jobs.append(
            ServingJob(
                job_id=k,
                arrival_s=t,
                kind="sk" if dense else "regular",
                n=n,
                degree=degree,
                with_fields=bool(g.random() < field_fraction),
                R=int(g.choice(r_choices)),
                t_f=int(g.integers(tf_range[0], tf_range[1] + 1)),
                instance_seed=int(g.integers(1, 2**31 - 1)),
                noise_seed=int(g.integers(1, 2**62)),
            )
        )
    return jobs
