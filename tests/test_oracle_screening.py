"""Pins of the connected n-body screening oracle (oracle/screening.py)
against what fixes it independently: the closed-form inclusion-exclusion
weights when nothing is dropped or only pairs are kept, non-interacting
bodies (every pair increment vanishes, so every increment of three or more
bodies is dropped and the expansion is still exact), a hand-worked path of
four bodies, linearity of the screened sum in the increment energies, and a
union-find check of the connectivity test."""
import itertools
import math

import numpy as np
import pytest

from oracle import ifci, screening
from paper_2307_10675_amd import synthetic


def _random_energies(nb, order, seed):
    rng = np.random.default_rng(seed)
    return {S: float(rng.normal(-1.0, 0.3)) for S in ifci.increments(nb, order)}, float(rng.normal(-0.5, 0.1))


@pytest.mark.parametrize("nb,order", [(4, 3), (5, 4), (6, 4)])
def test_threshold_zero_is_the_inclusion_exclusion_sum(nb, order):
    E, e_ref = _random_energies(nb, order, 11 * nb + order)
    keep = screening.cnb_keep(E, e_ref, nb, order, 0.0)
    assert keep == ifci.increments(nb, order)
    _, _, total = screening.screened_expansion(E, e_ref, order, keep)
    w = ifci.weights_closed(nb, order)
    want = e_ref + math.fsum(w[len(S) - 1] * (E[S] - e_ref) for S in E)
    assert abs(total - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("nb,order", [(4, 4), (6, 3)])
def test_infinite_threshold_keeps_pairs_only(nb, order):
    E, e_ref = _random_energies(nb, order, 7 * nb + order)
    keep = screening.cnb_keep(E, e_ref, nb, order, 1e30)
    assert keep == ifci.increments(nb, 2)
    _, by_order, total = screening.screened_expansion(E, e_ref, order, keep)
    w2 = ifci.weights_closed(nb, 2)
    want = e_ref + math.fsum(w2[len(S) - 1] * (E[S] - e_ref) for S in keep)
    assert abs(total - want) <= 1e-12 * max(1.0, abs(want))
    assert all(x == 0.0 for x in by_order[2:])


def test_non_interacting_bodies_drop_everything_above_pairs_and_stay_exact():
    p = synthetic.separable(4, seed=5, order=4)
    res = ifci.run(p)
    keep = screening.cnb_keep(res["E"], res["e_ref"], 4, 4, 1e-10)
    assert keep == ifci.increments(4, 2)
    _, _, total = screening.screened_expansion(res["E"], res["e_ref"], 4, keep)
    # the full-order expansion is exact (the FCI of all four bodies)
    assert abs(total - res["E"][(0, 1, 2, 3)]) < 1e-12


def test_hand_worked_path_of_four_bodies():
    """Pairs 01, 12, 23 above the threshold, 02, 03, 13 below: the 3-body
    increments 012 and 123 and the 4-body one are kept (connected), 013 and
    023 dropped; eps_0123 subtracts the kept subsets only."""
    e_ref = -1.0
    Ec1 = {0: -0.1, 1: -0.2, 2: -0.15, 3: -0.12}
    pair = {(0, 1): -0.01, (1, 2): -0.02, (2, 3): -0.03, (0, 2): 1e-6, (0, 3): -2e-6, (1, 3): 5e-7}
    E = {}
    for i, v in Ec1.items():
        E[(i,)] = e_ref + v
    for (i, j), v in pair.items():
        E[(i, j)] = e_ref + Ec1[i] + Ec1[j] + v
    Ec3 = {(0, 1, 2): -0.4805, (0, 1, 3): -0.4301, (0, 2, 3): -0.4002, (1, 2, 3): -0.5203}
    for S, v in Ec3.items():
        E[S] = e_ref + v
    E[(0, 1, 2, 3)] = e_ref - 0.651
    keep = screening.cnb_keep(E, e_ref, 4, 4, 1e-4)
    assert keep == [(0,), (1,), (2,), (3,), (0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3),
                    (0, 1, 2), (1, 2, 3), (0, 1, 2, 3)]
    eps, by_order, total = screening.screened_expansion(E, e_ref, 4, keep)
    e1 = dict(Ec1)
    e2 = dict(pair)
    e012 = Ec3[(0, 1, 2)] - e1[0] - e1[1] - e1[2] - e2[(0, 1)] - e2[(0, 2)] - e2[(1, 2)]
    e123 = Ec3[(1, 2, 3)] - e1[1] - e1[2] - e1[3] - e2[(1, 2)] - e2[(1, 3)] - e2[(2, 3)]
    e0123 = -0.651 - sum(e1.values()) - sum(e2.values()) - e012 - e123
    assert abs(eps[(0, 1, 2)] - e012) < 1e-15
    assert abs(eps[(1, 2, 3)] - e123) < 1e-15
    assert (0, 1, 3) not in eps and (0, 2, 3) not in eps
    assert abs(eps[(0, 1, 2, 3)] - e0123) < 1e-15
    assert abs(total - (e_ref + sum(e1.values()) + sum(e2.values()) + e012 + e123 + e0123)) < 1e-14


@pytest.mark.parametrize("threshold", [0.0, 0.05, 0.2])
def test_coefficients_are_the_linear_map(threshold):
    nb, order = 6, 4
    E, e_ref = _random_energies(nb, order, 99)
    keep = screening.cnb_keep(E, e_ref, nb, order, threshold)
    c = screening.screened_coefficients(keep, order)
    _, _, total = screening.screened_expansion(E, e_ref, order, keep)
    assert abs(e_ref + math.fsum(c[T] * (E[T] - e_ref) for T in c) - total) < 1e-12
    assert set(c) <= set(keep)
    if threshold == 0.0:
        w = ifci.weights_closed(nb, order)
        assert all(c[T] == w[len(T) - 1] for T in ifci.increments(nb, order))


def test_connectivity_against_union_find():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(3, 7))
        edges = {(i, j) for i, j in itertools.combinations(range(n), 2) if rng.random() < 0.35}
        parent = list(range(n))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a

        for i, j in edges:
            parent[find(i)] = find(j)
        want = len({find(a) for a in range(n)}) == 1
        assert screening.connected(tuple(range(n)), lambda i, j: (i, j) in edges) == want
