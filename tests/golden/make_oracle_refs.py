"""Write oracle reference energies for the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded synthetic problems of
paper_2307_10675_amd.synthetic; nothing here touches the device path.
Each output records the sha256 of the problem it was computed from.

    python tests/golden/make_oracle_refs.py [--only NAME] [--jobs N] [--checkpoint FILE]

--checkpoint FILE appends each finished increment energy to FILE (JSON lines)
and skips increments already listed there, so a long run can be resumed.
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

import numpy as np  # noqa: E402

from oracle import fci, ifci, rdm  # noqa: E402
from paper_2307_10675_amd import synthetic  # noqa: E402


def _solve(args):
    problem, S = args
    r = fci.solve_increment(problem, S)
    return S, r["E"], r["gap"]


def energies(problem, subsets, jobs, checkpoint=None):
    """{S: (E, gap)} for every S; the largest increments are started first."""
    done = {}
    if checkpoint and os.path.exists(checkpoint):
        with open(checkpoint) as f:
            for line in f:
                r = json.loads(line)
                if r.get("sha256") == problem.sha256():
                    done[tuple(r["bodies"])] = (r["E"], r["gap"])
    todo = sorted((S for S in subsets if tuple(S) not in done), key=lambda S: -len(S))
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        for S, e, g in ex.map(_solve, [(problem, S) for S in todo], chunksize=1):
            done[tuple(S)] = (e, g)
            if checkpoint:
                with open(checkpoint, "a") as f:
                    f.write(json.dumps(dict(sha256=problem.sha256(), bodies=list(S), E=e, gap=g)) + "\n")
    return {S: done[tuple(S)] for S in subsets}


def _densities(args):
    problem, S = args
    return S, rdm.increment_densities(problem, S)


def dump_gradient(name, problem, jobs, n_sample=4096, seed=3):
    """Every increment energy of the expansion and its gradient (weighted
    1- and 2-particle densities) from the oracle, in increment order: the
    whole dE/dh and a seeded sample of dE/d(pq|rs) entries (with the
    Frobenius norm of the whole array), as JSON."""
    t = t0 = time.time()
    subsets = ifci.increments(problem.n_bodies, problem.order)
    E, gap = {}, {}

    def stream(ex):
        for t, (S, d) in enumerate(ex.map(_densities, [(problem, S) for S in subsets], chunksize=1)):
            E[S], gap[S] = d["E"], d["gap"]
            if (t + 1) % 50 == 0:
                print(f"{name}: {t + 1} of {len(subsets)} increments, {time.time() - t0:.0f} s", flush=True)
            yield S, d

    with ProcessPoolExecutor(max_workers=jobs) as ex:
        e_tot, dh, deri = rdm.accumulate_gradient(problem, stream(ex))
    e_ref = ifci.reference_energy(problem)
    eps, by_order, total = ifci.increments_from_energies(E, e_ref, problem.order)
    idx = np.random.default_rng(seed).choice(deri.size, size=min(n_sample, deri.size), replace=False)
    idx.sort()
    grad = dict(e_total=float(e_tot), dE_dh=[float(x) for x in dh.ravel()],
                dE_deri_index=[int(i) for i in idx], dE_deri_value=[float(x) for x in deri.ravel()[idx]],
                dE_deri_norm=float(np.linalg.norm(deri)))
    doc = dict(problem=problem.meta, sha256=problem.sha256(), order=problem.order, e_ref=e_ref,
               increments=[dict(bodies=list(S), E=E[S], gap=gap[S]) for S in subsets],
               eps=[eps[S] for S in subsets], by_order=by_order, total=total,
               gradient=grad, seconds=time.time() - t)
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(doc, f)
    print(f"{name}: {len(subsets)} increments and the gradient in {doc['seconds']:.1f} s -> {path}")


def dump(name, problem, subsets, jobs, full_expansion, checkpoint=None):
    t = time.time()
    res = energies(problem, subsets, jobs, checkpoint)
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
    ap.add_argument("--checkpoint", default=None)
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
    todo["w2"] = (p2, inc2, True)
    # shapes above 8 active orbitals away from half filling, which take the
    # device-wide solver's general (materialised) product: 9 orbitals with 6
    # electrons (three bodies of 3 orbitals, one doubly occupied each) and 12
    # orbitals with 4 electrons (two bodies of 6 orbitals, one occupied each)
    p9 = synthetic.chain(3, orbs_per_body=3, nocc_per_body=1, seed=3093, order=3)
    todo["wide_9o6e"] = (p9, ifci.increments(3, 3), True)
    p12 = synthetic.chain(2, orbs_per_body=6, nocc_per_body=1, seed=3124, order=2)
    todo["wide_12o4e"] = (p12, ifci.increments(2, 2), True)
    # a chain whose pair increments fall off with distance (for the
    # connected n-body screening)
    pl = synthetic.local_chain(10, seed=5100, order=4, rate=1.0)
    todo["local10"] = (pl, ifci.increments(pl.n_bodies, pl.order), True)
    for name, (p, subsets, full) in todo.items():
        if a.only and a.only != name:
            continue
        dump(name, p, subsets, a.jobs, full, a.checkpoint)
    # workload 3 at order 4 (12 bodies, 793 increments up to 8o8e): energies
    # and the expansion gradient
    if a.only in (None, "w3o4"):
        dump_gradient("w3o4", synthetic.chain(12, seed=3000, order=4), a.jobs)


if __name__ == "__main__":
    main()
