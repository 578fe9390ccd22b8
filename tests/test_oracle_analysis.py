"""Pins of the grouped-contribution oracle (oracle/analysis.py): one group
gives the order sums of eq. 1, all groups together the correlation energy,
a hand-worked labelling of three bodies, and the two-calculation
difference; and the C ABI's combination count and argument checks."""
import ctypes
import math

import numpy as np
import pytest

from oracle import analysis, ifci
from paper_2307_10675_amd import ifci as pifci, synthetic


def _eps(nb, order, seed):
    rng = np.random.default_rng(seed)
    return {S: float(rng.normal(0.0, 0.01)) for S in ifci.increments(nb, order)}


def test_one_group_gives_the_order_sums():
    eps = _eps(6, 4, 1)
    g = analysis.group_sums(eps, [0] * 6)
    for k in range(1, 5):
        assert g[(0,) * k] == math.fsum(e for S, e in eps.items() if len(S) == k)
    assert abs(math.fsum(g.values()) - math.fsum(eps.values())) < 1e-15


def test_hand_worked_three_bodies():
    eps = {(0,): 1.0, (1,): 2.0, (2,): 4.0, (0, 1): 8.0, (0, 2): 16.0, (1, 2): 32.0, (0, 1, 2): 64.0}
    g = analysis.group_sums(eps, [0, 1, 0])
    assert g == {(0,): 5.0, (1,): 2.0, (0, 0): 16.0, (0, 1): 40.0, (0, 0, 1): 64.0}
    eps_b = {S: 2.0 * v for S, v in eps.items()}
    d = analysis.group_differences(eps, eps_b, [0, 1, 0])
    assert d == g


def test_group_count_and_argument_checks():
    L = pifci.lib()
    p = synthetic.chain(5, seed=3, order=4)
    a = pifci.Plan(p, tuning=None)
    n = ctypes.c_int64()
    assert L.ifci_group_count(a._h, 3, ctypes.byref(n)) == 0
    assert n.value == 3 + 6 + 10 + 15
    assert L.ifci_group_count(a._h, 1, ctypes.byref(n)) == 0 and n.value == 4
    assert L.ifci_group_count(a._h, 0, ctypes.byref(n)) == 1
    bad = np.array([0, 1, 2, 3, 0], dtype=np.int32)
    out = np.zeros(34)
    assert L.ifci_group_sums(a._h, ctypes.c_void_p(256), bad.ctypes.data_as(ctypes.c_void_p), 3,
                             out.ctypes.data_as(ctypes.c_void_p), None, None) == 1
    assert L.ifci_group_sums(a._h, None, bad.ctypes.data_as(ctypes.c_void_p), 4,
                             out.ctypes.data_as(ctypes.c_void_p), None, None) == 1
    a.close()
