"""The paper's experiments, re-run in form on synthetic stand-in instances (library API only).

The paper's instance sets, figure data and Gset graphs are not available, so these reproduce the
*shape* of each experiment on seeded synthetic instances of the same classes and sizes; nothing
here compares against the paper's numbers.

* ``fig3``  -- Sec. II, Fig. 3: a 16-spin Moebius ladder with the schedule compressed to 100
  iterations; per-iteration spin values of one sample and the Ising energy of their signs.
* ``fig4``  -- Sec. III, Fig. 4: success probability and time to solution (99%) against N for
  SK (J = +-1), dense MAX-CUT (p = 1/2) and degree-3 MAX-CUT instances (10, 10 and 20 instances
  per size), 10,000 samples per instance. The success target of an instance is the best energy
  seen in any of its samples.
* ``table1`` -- Table I: mean and best MAX-CUT value over 100 runs on 2000-spin instances: a
  random graph with 19,990 unit edges (the G22 class), a scale-free Barabasi-Albert graph with
  about 12,000 unit edges (the G39 class) and a complete graph with +-1 weights (K2000 class).
* ``sweep`` -- the method's own parameters (Sec. II: alpha = sigma = 0.15 and the schedule of
  Fig. 2 were tuned coarsely): success probability over a grid of damping alpha and noise sigma
  (sigma = 0 is plain mean-field annealing, Sec. I) and over schedule variants, on SK instances.
  An instance's target is the best energy seen in any sample of any variant, so the variants
  are compared against one target.

Usage: python -m paper_1806_08422_amd.experiments {fig3,fig4,table1,sweep} [--out FILE.json]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import instances  # noqa: E402
from paper_1806_08422_amd import nmfa  # noqa: E402


def fig3(seed: int = 3, t_f: int = 100):
    inst = instances.moebius_ladder(16)
    with nmfa.Solver(inst.J, inst.h, precision="fp64", record_iters=t_f) as s:
        s.anneal(1, t_f, seed)
        traj = s.trajectory()[:, 0, :]  # [t, spin]
        # Eq. 1 of the sign readout of every recorded iteration, evaluated by the library's energy
        # kernels (s >= 0 reads as +1, as the readout of Alg. 1 does)
        signs = np.where(traj >= 0, 1, -1).astype(np.int8)
        energies, _ = s.energies_of(signs)
    return {"instance": "moebius ladder, 16 spins", "t_f": t_f, "spins": traj.tolist(),
            "energy_of_signs": energies.tolist(), "ground_energy_closed_form": -20}


def _tts99(t_sample, p):
    if p <= 0:
        return math.inf
    if p >= 0.99:
        return t_sample
    return t_sample * math.log(0.01) / math.log(1 - p)


def fig4(sizes=(20, 40, 60, 80, 100), samples=10000, t_f=1000, precision="bf16", counts=(10, 10, 20)):
    classes = {
        "sk": (counts[0], lambda n, k: instances.sk(n, 100 + k)),
        "dense_maxcut": (counts[1], lambda n, k: instances.gnp(n, 0.5, 200 + k)),
        "degree3_maxcut": (counts[2], lambda n, k: instances.random_regular(n, 3, 300 + k)),
    }
    out = {}
    for name, (count, make) in classes.items():
        rows = []
        for n in sizes:
            ps, tts, best = [], [], []
            for k in range(count):
                inst = make(n, k)
                with nmfa.Solver(inst.J, inst.h, precision=precision) as s:
                    t0 = time.perf_counter()
                    s.anneal(samples, t_f, 5000 + k)
                    E = s.energies()[0]
                    dt = time.perf_counter() - t0
                p = float(np.mean(E <= E.min()))
                ps.append(p)
                best.append(float(E.min()))
                tts.append(_tts99(dt / samples, p))
            rows.append({"n": n, "success_median": float(np.median(ps)),
                         "success_iqr": [float(np.percentile(ps, 25)), float(np.percentile(ps, 75))],
                         "tts99_median_s": float(np.median(tts)), "success": ps, "best_energy": best})
        out[name] = rows
    return {"samples_per_instance": samples, "t_f": t_f, "precision": precision, "classes": out}


# schedule variants for the sweep: (u, T) knots, T interpolated geometrically between knots
SCHEDULES = {
    "paper (Fig. 2)": None,
    "one geometric ramp 10 -> 0.05": ((0.0, 10.0), (1.0, 0.05)),
    "cold start 2 -> 0.05": ((0.0, 2.0), (0.6, 0.5), (1.0, 0.05)),
    "constant T = 0.5": ((0.0, 0.5), (1.0, 0.5)),
}


def sweep(n=100, count=5, samples=10000, t_f=1000, precision="bf16", alphas=(0.05, 0.1, 0.15, 0.3, 0.6),
          sigmas=(0.0, 0.05, 0.15, 0.3, 0.5), schedules=SCHEDULES):
    variants = [("grid", a, sg, "paper (Fig. 2)") for a in alphas for sg in sigmas]
    variants += [("schedule", 0.15, 0.15, name) for name in schedules if name != "paper (Fig. 2)"]
    energies = {}  # (variant index, instance) -> energies of all samples
    for k in range(count):
        inst = instances.sk(n, 400 + k)
        for v, (_, a, sg, sched) in enumerate(variants):
            with nmfa.Solver(inst.J, inst.h, precision=precision, alpha=a, sigma=sg, knots=schedules[sched]) as s:
                s.anneal(samples, t_f, 9000 + k)
                energies[(v, k)] = s.energies()[0]
    target = [min(float(energies[(v, k)].min()) for v in range(len(variants))) for k in range(count)]
    rows = []
    for v, (kind, a, sg, sched) in enumerate(variants):
        ps = [float(np.mean(energies[(v, k)] <= target[k])) for k in range(count)]
        rows.append({"kind": kind, "alpha": a, "sigma": sg, "schedule": sched,
                     "success_median": float(np.median(ps)), "success": ps,
                     "mean_energy": float(np.mean([energies[(v, k)].mean() for k in range(count)])),
                     "distinct_energies_max": int(max(len(np.unique(energies[(v, k)])) for k in range(count)))})
    return {"n": n, "instances": count, "samples_per_instance": samples, "t_f": t_f, "precision": precision,
            "targets": target, "variants": rows}


def _ba_graph(n, m, seed):
    import networkx as nx

    g = nx.barabasi_albert_graph(n, m, seed=seed)
    J = np.zeros((n, n))
    for a, b in g.edges():
        J[a, b] = J[b, a] = 1.0
    return J


def _random_graph_m(n, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    J = np.zeros((n, n))
    edges = set()
    while len(edges) < m:
        a, b = rng.integers(0, n, size=2)
        if a != b:
            edges.add((min(a, b), max(a, b)))
    for a, b in edges:
        J[a, b] = J[b, a] = 1.0
    return J


def table1(runs=100, t_f=5000, precision="fp8j_bf16s"):
    cases = {
        "random (G22 class)": _random_graph_m(2000, 19990, 22),
        "scale-free (G39 class)": _ba_graph(2000, 6, 39),
        "fully connected +-1 (K2000 class)": instances.sk(2000, 2000).J,
    }
    out = {}
    for name, J in cases.items():
        with nmfa.Solver(J, None, precision=precision) as s:
            s.anneal(runs, t_f, 777)
            cuts = s.cuts()
            path = s.info()["path"]
        W = np.triu(J, 1)
        out[name] = {"mean_cut": float(cuts.mean()), "best_cut": float(cuts.max()), "runs": runs,
                     "edges_weight": float(W.sum()), "positive_weight": float(W[W > 0].sum()), "kernel_path": path}
    return {"t_f": t_f, "precision": precision, "instances": out}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["fig3", "fig4", "table1", "sweep"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--samples", type=int, default=10000)
    args = ap.parse_args(argv)
    if args.experiment == "fig3":
        res = fig3()
    elif args.experiment == "fig4":
        res = fig4(samples=args.samples)
    elif args.experiment == "sweep":
        res = sweep(samples=args.samples)
    else:
        res = table1()
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text[:2000])


if __name__ == "__main__":
    main()
