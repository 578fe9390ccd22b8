"""GPU grouped contributions (ifci_group_sums) against the oracle's sums
over its exact increments: the 10-body workload with three labels, and the
change between two calculations of one chain (two seeds standing for two
geometries with comparable orbitals)."""
import numpy as np
import pytest

from oracle import analysis, ifci as oifci
from paper_2307_10675_amd import ifci, synthetic
from tests.helpers import load_golden

pytestmark = pytest.mark.gpu


def test_group_sums_against_oracle():
    p = synthetic.workload(1)
    g = load_golden("w1")
    assert p.sha256() == g["sha256"]
    labels = [b % 3 for b in range(p.n_bodies)]
    plan, res = ifci.solve(p, r_tol=1e-9, max_iter=500)
    got = plan.group_sums(res["eps"], labels, 3)
    eps_o = {tuple(x["bodies"]): e for x, e in zip(g["increments"], g["eps"])}
    want = analysis.group_sums(eps_o, labels)
    assert set(k for k, v in got.items()) >= set(want)
    for c, v in got.items():
        n = sum(1 for S in eps_o if analysis.combination(S, labels) == c)
        assert abs(v - want.get(c, 0.0)) <= 1e-9 * 2 ** len(c) * max(1, n), c
    assert abs(sum(got.values()) - (res["total"] - res["e_ref"])) <= 1e-9


def test_group_differences_of_two_calculations():
    pa = synthetic.chain(6, seed=7001, order=3)
    pb = synthetic.chain(6, seed=7002, order=3)
    labels = [0, 1, 1, 0, 2, 2]
    sums = []
    for p in (pa, pb):
        plan, res = ifci.solve(p, r_tol=1e-10, max_iter=500)
        sums.append(plan.group_sums(res["eps"], labels, 3))
    got = ifci.group_differences(sums[0], sums[1])
    ra, rb = oifci.run(pa), oifci.run(pb)
    want = analysis.group_differences(ra["eps"], rb["eps"], labels)
    for c, v in want.items():
        assert abs(got[c] - v) <= 1e-8, c
