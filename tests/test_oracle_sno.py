"""Pins of the summation-natural-orbital oracle (oracle/sno.py): keeping
every natural orbital reproduces the increment's FCI over all virtuals (the
energy does not depend on the basis of the virtual space), the SNO energies
do not change when the input's virtual orbitals are rotated, the one-body
density of two electrons has the traces a two-electron state must have,
and truncation raises each increment energy, less as more orbitals are
kept (the truncated space is a subspace)."""
import numpy as np
import pytest

from oracle import fci, ifci, sno
from paper_2307_10675_amd import synthetic


@pytest.fixture(scope="module")
def system():
    return synthetic.sno_system(3, 6, seed=8100, order=2)


def _full_increment(p, S_occ):
    """FCI of S's occupied orbitals plus every virtual, the rest frozen."""
    others = [j for j in p.occ if j not in S_occ]
    q = sno._P(p.h, p.eri, [list(S_occ) + p.vir] + [[j] for j in others], [len(S_occ)] + [1] * len(others), 1)
    return fci.solve_increment(q, (0,))["E"]


def test_keeping_every_natural_orbital_gives_the_full_virtual_space(system):
    p = system
    rho = {i: sno.one_body_density(p.h, p.eri, p.occ, p.vir, i)[0] for i in p.occ}
    for S_occ in ([p.occ[0]], [p.occ[0], p.occ[2]]):
        w, U = np.linalg.eigh(sum(rho[i] for i in S_occ))
        q = sno.rotated_problem(p.h, p.eri, p.occ, p.vir, S_occ, U)
        e = fci.solve_increment(q, (0,))["E"]
        assert abs(e - _full_increment(p, S_occ)) < 1e-11


def test_one_body_density_traces(system):
    p = system
    for i in p.occ:
        rho, d = sno.one_body_density(p.h, p.eri, p.occ, p.vir, i)
        g = d["gamma"]
        assert abs(np.trace(g) - 2 * len(p.occ)) < 1e-12
        assert abs(np.trace(rho) - (2.0 - g[i, i])) < 1e-12
        w = np.linalg.eigvalsh(rho)
        assert w.min() > -1e-12 and w.max() < 2.0


def test_invariant_under_rotation_of_the_virtuals(system):
    p = system
    n = p.n_orb
    Q = np.eye(n)
    rng = np.random.default_rng(5)
    A = rng.normal(size=(len(p.vir), len(p.vir)))
    R, _ = np.linalg.qr(A)
    Q[np.ix_(p.vir, p.vir)] = R
    h2 = Q.T @ p.h @ Q
    eri2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", p.eri, Q, Q, Q, Q, optimize=True)
    a = sno.sno_expansion(p.h, p.eri, p.occ, p.vir, 2, eta=3.0)
    b = sno.sno_expansion(h2, eri2, p.occ, p.vir, 2, eta=3.0)
    for S in a["E"]:
        assert a["n_keep"][S] == b["n_keep"][S]
        assert abs(a["E"][S] - b["E"][S]) < 1e-10, S
    assert abs(a["total"] - b["total"]) < 1e-10


def test_truncation_is_variational_and_monotone(system):
    p = system
    prev = None
    for eta in (1.0, 2.0, 4.0):
        r = sno.sno_expansion(p.h, p.eri, p.occ, p.vir, 2, eta=eta)
        for S, e in r["E"].items():
            full = _full_increment(p, [p.occ[b] for b in S])
            assert e >= full - 1e-11
            if prev is not None:
                assert e <= prev["E"][S] + 1e-11
                assert r["n_keep"][S] >= prev["n_keep"][S]
        prev = r
    low = sno.sno_expansion(p.h, p.eri, p.occ, p.vir, 2, eta=1.0)
    assert any(v < len(p.vir) for v in low["n_keep"].values()), "eta 1 truncates nothing: the pin would be empty"
