"""Write oracle reference energies for the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded synthetic problems of
paper_2307_10675_amd.synthetic; nothing here touches the device path.
Each output records the sha256 of the problem it was computed from.

    python tests/golden/make_oracle_refs.py [--only NAME] [--jobs N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fci, ifci  # noqa: E402
from paper_2307_10675_amd import synthetic  # noqa: E402


def _solve(args):
    problem, S = args
    r = fci.solve_increment(problem, S)
    return S, r["E"], r["gap"]


def energies(problem, subsets, jobs):
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        out = list(ex.map(_solve, [(problem, S) for S in subsets], chunksize=1))
    return {S: (e, g) for S, e, g in out}


def dump(name, problem, subsets, jobs, full_expansion):
    t = time.time()
    res = energies(problem, subsets, jobs)
    e_ref = ifci.reference_energy(problem)
    doc = dict(
        problem=problem.meta, sha256=problem.sha256(), order=problem.order, e_ref=e_ref,
        increments=[dict(bodies=list(S), E=res[S][0], gap=res[S][1]) for S in subsets],
        seconds=time.time() - t,
    )
    if full_expansion:
        E = {S: res[S][0] for S in subsets}
        eps, by_order, total = ifci.increments_from_energies(E, e_ref, problem.order)
        doc["eps"] = [eps[S] for S in subsets]
        doc["by_order"] = by_order
        doc["total"] = total
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"{name}: {len(subsets)} increments in {doc['seconds']:.1f} s -> {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    ap.add_argument("--jobs", type=int, default=os.cpu_count())
    a = ap.parse_args()
    todo = {}
    for r in range(10):
        p = synthetic.workload(0, r)
        todo[f"w0_r{r}"] = (p, [(0,)], True)
    p1 = synthetic.workload(1)
    todo["w1"] = (p1, ifci.increments(p1.n_bodies, p1.order), True)
    p4 = synthetic.chain(4, seed=1100, order=4)
    todo["chain4_full"] = (p4, ifci.increments(4, 4), True)
    p2 = synthetic.workload(2)
    inc2 = ifci.increments(p2.n_bodies, p2.order)
    sample = [S for S in inc2 if len(S) <= 2] + [S for S in inc2 if len(S) == 3][::28] + \
             [S for S in inc2 if len(S) == 4][::91]
    todo["w2_sample"] = (p2, sample, False)
    p3 = synthetic.chain(12, seed=3000, order=4)
    inc3 = ifci.increments(12, 4)
    todo["w3o4_sample"] = (p3, [S for S in inc3 if len(S) <= 2] + [S for S in inc3 if len(S) == 4][::99], False)
    for name, (p, subsets, full) in todo.items():
        if a.only and a.only != name:
            continue
        dump(name, p, subsets, a.jobs, full)


if __name__ == "__main__":
    main()
