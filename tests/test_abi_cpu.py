"""The C ABI on the CPU: exported symbols, bit-exact string and link tables
against the oracle, increment enumeration and weights, argument errors.
No device work is queued by any of these calls."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import ifci as oifci
from oracle import strings as ostr
from paper_2307_10675_amd import ifci, synthetic

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ifci.h")


@pytest.fixture(scope="module")
def L():
    return ifci.lib()


def test_exports_every_declared_symbol(L):
    text = open(HEADER).read()
    names = set(re.findall(r"\b(ifci_[a-z_]+)\s*\(", text))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n
    assert L.ifci_abi_version() == 4


@pytest.mark.parametrize("k,n", [(k, n) for k in range(1, 13) for n in range(0, k + 1)])
def test_tables_bit_exact(k, n):
    s, link = ifci.tables(k, n)
    assert list(s) == ostr.strings(k, n)
    ref = ostr.link_table(k, n)
    got = [[tuple(int(x) for x in e) for e in row] for row in link]
    assert got == [[tuple(e) for e in row] for row in ref]


def test_tables_reject_bad_shape(L):
    assert L.ifci_tables(17, 8, None, None) == 1
    assert L.ifci_tables(4, 5, None, None) == 1


@pytest.mark.parametrize("nb,order", [(4, 2), (10, 3), (16, 4), (6, 6)])
def test_increment_enumeration_and_weights(nb, order):
    p = synthetic.chain(nb, seed=1, order=order)
    plan = ifci.Plan(p)
    incs = plan.increments()
    ref = oifci.increments(nb, order)
    assert [i.bodies for i in incs] == ref
    for S, inf in zip(ref, incs):
        k = 2 * len(S)
        assert inf.n_act == k and inf.n_alpha == len(S)
        assert inf.n_det == math.comb(k, len(S)) ** 2
    assert plan.weights() == [float(w) for w in oifci.weights_closed(nb, order)]
    info = plan.info()
    assert info["n_inc"] == len(ref)
    assert info["workspace_bytes"] > 0
    plan.close()


def test_workload_sizes():
    """The batched workload: 16 + 120 + 560 + 1820 increments, 9,146,384 determinants."""
    p = synthetic.workload(2)
    plan = ifci.Plan(p)
    incs = plan.increments()
    sizes = [sum(1 for i in incs if len(i.bodies) == k) for k in range(1, 5)]
    assert sizes == [16, 120, 560, 1820]
    assert sum(i.n_det for i in incs) == 9_146_384
    plan.close()


def _problem_struct(n_orb, bodies, nocc, order):
    ptr = np.cumsum([0] + [len(b) for b in bodies]).astype(np.int32)
    orb = np.array([o for b in bodies for o in b], dtype=np.int32)
    no = np.array(nocc, dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    pr = ifci.Problem(n_orb=n_orb, n_bodies=len(bodies), body_ptr=ptr.ctypes.data_as(P),
                      body_orb=orb.ctypes.data_as(P), body_nocc=no.ctypes.data_as(P), order=order, e_const=0.0)
    return pr, (ptr, orb, no)


@pytest.mark.parametrize("n_orb,bodies,nocc,order,code", [
    (4, [[0, 1], [1, 2]], [1, 1], 1, 1),          # overlapping bodies
    (4, [[0, 1], [2, 3]], [1, 1], 3, 1),          # order > n_bodies
    (4, [[0, 1], [2, 5]], [1, 1], 1, 1),          # orbital out of range
    (4, [[0, 1], [2, 3]], [3, 1], 1, 1),          # more occupied than orbitals
    (4, [[0, 1], [2, 3]], [1, 1], 0, 1),          # order 0
    (34, [list(range(17)), list(range(17, 34))], [8, 8], 1, 2),   # 17 active orbitals
])
def test_plan_argument_errors(L, n_orb, bodies, nocc, order, code):
    pr, keep = _problem_struct(n_orb, bodies, nocc, order)
    h = ctypes.c_void_p()
    opt = ifci.default_options()
    assert L.ifci_plan_create(ctypes.byref(pr), ctypes.byref(opt), 0, ctypes.byref(h)) == code
    assert not h.value
    assert len(L.ifci_last_error()) > 0


def test_bad_options_and_state_errors(L):
    pr, keep = _problem_struct(4, [[0, 1], [2, 3]], [1, 1], 2)
    h = ctypes.c_void_p()
    bad = ifci.default_options(max_space=1)
    assert L.ifci_plan_create(ctypes.byref(pr), ctypes.byref(bad), 0, ctypes.byref(h)) == 1
    opt = ifci.default_options()
    assert L.ifci_plan_create(ctypes.byref(pr), ctypes.byref(opt), 0, ctypes.byref(h)) == 0
    # no workspace yet: integrals, sigma and Davidson are refused before any device work
    assert L.ifci_set_integrals(h, ctypes.c_void_p(256), ctypes.c_void_p(512), None) == 6
    assert L.ifci_set_workspace(h, None, 1 << 20) == 1
    assert L.ifci_set_workspace(h, ctypes.c_void_p(257), 1 << 40) == 1   # misaligned
    assert L.ifci_sigma(h, 0, ctypes.c_void_p(256), ctypes.c_void_p(512), 0, None) == 6
    assert L.ifci_sigma(h, 99, ctypes.c_void_p(256), ctypes.c_void_p(512), 0, None) == 1
    assert L.ifci_davidson(h, 0, 99, ctypes.c_void_p(256), ctypes.c_void_p(512), None, None, None, None) == 1
    assert L.ifci_plan_destroy(h) == 0
    assert L.ifci_status_string(5) == b"not converged"


def test_davidson_group_argument_errors(L):
    """ifci_davidson_group refuses null plans, mismatched options and plans
    without workspace before any device work."""
    import ctypes
    from paper_2307_10675_amd import ifci, synthetic
    p = synthetic.single(4, 12, 1)
    a = ifci.Plan(p)
    b = ifci.Plan(p, precision=ifci.MIXED)
    null = (ctypes.c_void_p * 1)(None)
    assert L.ifci_davidson_group(None, 1, null, null, None, None, None) == 1
    two = (ctypes.c_void_p * 2)(a._h.value, b._h.value)
    outs = (ctypes.c_void_p * 2)(1, 1)
    assert L.ifci_davidson_group(two, 2, outs, outs, None, None, None) == 1   # options differ
    same = (ctypes.c_void_p * 2)(a._h.value, a._h.value)
    assert L.ifci_davidson_group(same, 2, outs, outs, None, None, None) == 1  # listed twice
    one = (ctypes.c_void_p * 1)(a._h.value)
    assert L.ifci_davidson_group(one, 1, outs, outs, None, None, None) == 6   # no workspace


def test_set_tuning_arguments(L, tmp_path):
    """ifci_set_tuning takes k 1..8, FP64 or MIXED, ps_block -1..64 and
    e_waves 0..8; the tuner cache round-trips through load_tuning."""
    import json
    from paper_2307_10675_amd import ifci, synthetic
    p = synthetic.single(4, 12, 1)
    a = ifci.Plan(p, tuning=None)
    h = a._h
    assert L.ifci_set_tuning(h, 8, ifci.MIXED, 64, 0) == 0
    assert L.ifci_set_tuning(h, 1, ifci.FP64, -1, 8) == 0
    for k, pr, ps, ew in ((0, 0, 0, 0), (9, 0, 0, 0), (4, 2, 0, 0), (4, 0, -2, 0), (4, 0, 65, 0), (4, 0, 0, 9),
                          (4, 0, 0, -1)):
        assert L.ifci_set_tuning(h, k, pr, ps, ew) == 1
    assert L.ifci_set_tuning(None, 4, 0, 0, 0) == 1
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"entries": [{"k": 8, "precision": 1, "ps_block": 48, "e_waves": 6},
                                         {"k": 6, "precision": 0, "ps_block": 0, "e_waves": 0}]}))
    t = ifci.load_tuning(str(f))
    assert t == {(8, 1): (48, 6), (6, 0): (0, 0)}
    assert ifci.load_tuning(str(tmp_path / "missing.json")) == {}
    b = ifci.Plan(p, tuning=t)
    b.close()
    a.close()


def test_screen_needs_solved_plan(L):
    """ifci_screen refuses a plan without workspace and integrals (no device
    work), and an invalid plan."""
    import ctypes
    from paper_2307_10675_amd import ifci, synthetic
    p = synthetic.chain(3, seed=1, order=3)
    a = ifci.Plan(p, tuning=None)
    n = ctypes.c_int64()
    assert L.ifci_screen(a._h, ctypes.c_void_p(256), 1e-4, None, ctypes.byref(n), None) == 6
    assert L.ifci_screen(None, ctypes.c_void_p(256), 1e-4, None, ctypes.byref(n), None) == 1
    a.close()


def test_sno_argument_checks(L):
    """The SNO entry points refuse bad sizes and a short work buffer before
    any device work."""
    import ctypes
    d = ctypes.c_void_p(256)
    assert L.ifci_sno_orbitals(d, 12, d, 17, d, 4, 2, 3.0, d, d, None) == 1      # n_vir > 16
    assert L.ifci_sno_orbitals(None, 12, d, 8, d, 4, 2, 3.0, d, d, None) == 1
    # m = 2 + 8 + 2 = 12 orbitals of 12: needs 12 * 12 + 2 * 12^4 doubles
    need = 12 * 12 + 2 * 12 ** 4
    assert L.ifci_sno_transform(d, d, 12, d, 8, d, 2, 2, d, 8, d, need - 1, d, d, None) == 1
    assert L.ifci_sno_transform(d, d, 12, d, 8, d, 2, 2, d, 9, d, need, d, d, None) == 1   # n_keep > n_vir
    assert L.ifci_sno_transform(d, d, 12, d, 8, d, 3, 2, d, 8, d, need, d, d, None) == 1   # too many orbitals


def test_hbci_options_and_argument_checks(L):
    """The HBCI entry points: the paper's thresholds as defaults, the work
    size growing with the capacities, and refusals before any device work
    (bad options, no integrals, a short or misaligned buffer)."""
    import ctypes
    from paper_2307_10675_amd import ifci, synthetic
    o = ifci.hbci_options()
    assert (o.eps1, o.eps2) == (1e-3, 1e-6)
    assert 2 <= o.m_max <= 16 and o.max_iter >= 1 and o.max_det >= 2
    p = synthetic.chain(3, seed=1, order=2)
    a = ifci.Plan(p, tuning=None)
    small = ifci.hbci_options(max_det=64, max_nnz=1024, max_ext=256)
    big = ifci.hbci_options(max_det=128, max_nnz=1024, max_ext=256)
    nb_s, nb_b = ctypes.c_int64(), ctypes.c_int64()
    assert L.ifci_hbci_work_bytes(a._h, 3, ctypes.byref(small), ctypes.byref(nb_s)) == 0
    assert L.ifci_hbci_work_bytes(a._h, 3, ctypes.byref(big), ctypes.byref(nb_b)) == 0
    assert 0 < nb_s.value < nb_b.value
    assert L.ifci_hbci_work_bytes(a._h, 99, ctypes.byref(small), ctypes.byref(nb_s)) == 1
    bad = ifci.hbci_options(max_det=64, max_nnz=1024, max_ext=256, m_max=17)
    assert L.ifci_hbci_work_bytes(a._h, 0, ctypes.byref(bad), ctypes.byref(nb_s)) == 1
    res = (ctypes.c_double * 8)()
    w = ctypes.c_void_p(1 << 20)
    # bad options first, then the missing integrals
    neg = ifci.hbci_options(max_det=64, max_nnz=1024, max_ext=256, eps1=-1.0)
    assert L.ifci_hbci_solve(a._h, 0, ctypes.byref(neg), w, 1 << 30, res, None, None, None) == 1
    assert L.ifci_hbci_solve(a._h, 0, ctypes.byref(small), w, 1 << 30, res, None, None, None) == 6
    assert L.ifci_hbci_solve(None, 0, ctypes.byref(small), w, 1 << 30, res, None, None, None) == 1
    a.close()
