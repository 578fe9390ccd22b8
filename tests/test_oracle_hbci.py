"""Pins of the HBCI oracle (oracle/hbci.py).

* Two orbitals, two electrons, with integrals whose single replacements
  vanish (the minimal-basis H2 pattern): the variational root is the 2 x 2
  closed form, a determinant enters exactly when |K| > eps1 (for either sign
  of K), and from the reference alone E_PT2 = K^2 / (E_0 - E_D).
* eps1 = 0 reaches the whole space and the exact increment energy, with no
  second-order remainder.
* E_PT2 equals the second derivative at 0 of the lowest root of the
  Epstein-Nesbet partitioned Hamiltonian [[H_VV, l H_VA], [l H_AV, diag H_AA]],
  diagonalised exactly (the definition of second-order Epstein-Nesbet
  perturbation theory, not its formula).
* The reference determinant's diagonal is the closed-shell energy; E_var is
  an upper bound to the exact energy and falls as eps1 does; the spaces are
  closed under the spin flip and their roots symmetric under it (a
  selected space need not be spin-complete, so <S^2> is not checked).
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import fci, hbci, ifci
from paper_2307_10675_amd import synthetic


def _h2_like(h11, h22, j11, j22, j12, k12):
    h = np.diag([h11, h22])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0], eri[1, 1, 1, 1] = j11, j22
    eri[0, 0, 1, 1] = eri[1, 1, 0, 0] = j12
    for p, q, r, s in ((0, 1, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1)):
        eri[p, q, r, s] = k12
    return SimpleNamespace(h=h, eri=eri, bodies=[[0, 1]], nocc=[1], order=1, e_const=0.0, n_orb=2, n_bodies=1)


@pytest.mark.parametrize("k12", [0.18, -0.18])
def test_two_orbital_closed_forms(k12):
    p = _h2_like(-1.25, -0.45, 0.67, 0.70, 0.66, k12)
    e0 = 2 * -1.25 + 0.67
    ed = 2 * -0.45 + 0.70
    # |K| > eps1: the doubly excited determinant joins; the 2 x 2 root
    r = hbci.solve_increment(p, (0,), eps1=abs(k12) / 2, eps2=0.0)
    exact = 0.5 * (e0 + ed) - math.sqrt(0.25 * (ed - e0) ** 2 + k12 * k12)
    assert sorted(r["dets"]) == sorted([0b0101, 0b1010])
    assert abs(r["E_var"] - exact) < 1e-13
    assert r["E_pt2"] == 0.0 and r["n_ext"] == 0
    assert r["converged"] and r["n_iter"] == 2
    # |K| < eps1: the reference alone, and the second-order energy
    r = hbci.solve_increment(p, (0,), eps1=2 * abs(k12), eps2=0.0)
    assert r["dets"] == [0b0101]
    assert abs(r["E_var"] - e0) < 1e-14
    assert abs(r["E_pt2"] - k12 * k12 / (e0 - ed)) < 1e-14
    assert r["n_ext"] == 1
    # eps2 above |K| screens the only coupling out
    r = hbci.solve_increment(p, (0,), eps1=2 * abs(k12), eps2=2 * abs(k12))
    assert r["E_pt2"] == 0.0 and r["n_ext"] == 0


@pytest.fixture(scope="module")
def chain3():
    return synthetic.chain(3, seed=7300, order=3)


def test_eps1_zero_is_the_exact_increment(chain3):
    S = (0, 1, 2)
    r = hbci.solve_increment(chain3, S, eps1=0.0, eps2=0.0)
    ex = fci.solve_increment(chain3, S)
    assert len(r["V"]) == len(ex["dets"])
    assert abs(r["E_var"] - ex["E"]) < 1e-10
    assert r["E_pt2"] == 0.0 and r["converged"]


def test_reference_diagonal_is_the_closed_shell_energy(chain3):
    sp = hbci.Space(chain3, (0, 1))
    assert abs(sp.H[sp.ref, sp.ref] - ifci.reference_energy(chain3)) < 1e-12


def _en_partitioned_second_derivative(H, V, e_var):
    A = [a for a in range(H.shape[0]) if a not in set(V)]
    order = list(V) + A
    M = H[np.ix_(order, order)].copy()
    nv = len(V)
    M[nv:, nv:] = np.diag(np.diag(M)[nv:])

    def root(lam):
        X = M.copy()
        X[:nv, nv:] *= lam
        X[nv:, :nv] *= lam
        w = np.linalg.eigvalsh(X)
        return w[np.argmin(np.abs(w - e_var))]

    f = {lam: (root(lam) - e_var) / lam ** 2 for lam in (0.02, 0.01)}
    return (4 * f[0.01] - f[0.02]) / 3       # Richardson: the lambda^2 term removed


@pytest.mark.parametrize("eps1", [3e-2, 5e-3])
def test_pt2_is_the_epstein_nesbet_second_order_energy(chain3, eps1):
    sp = hbci.Space(chain3, (0, 1, 2))
    r = hbci.solve(sp, eps1=eps1, eps2=0.0)
    assert 1 < len(r["V"]) < len(sp.dets)
    ref = _en_partitioned_second_derivative(sp.H, r["V"], r["E_var"])
    assert abs(r["E_pt2"] - ref) < 2e-6 * abs(ref)
    # eps2 > 0 drops terms: fewer external determinants, and the screened
    # energy approaches the unscreened one as eps2 falls
    diffs = []
    for eps2 in (1e-3, 1e-4, 1e-5, 1e-7):
        e2, n_ext = hbci.pt2(sp.H, r["V"], r["c"], r["E_var"], eps2)
        assert n_ext <= r["n_ext"]
        diffs.append(abs(e2 - r["E_pt2"]))
    assert diffs == sorted(diffs, reverse=True) and diffs[-1] < 1e-6 * abs(r["E_pt2"])


def test_variational_bound_spin_and_monotone_spaces(chain3):
    S = (0, 1, 2)
    sp = hbci.Space(chain3, S)
    exact = fci.solve_increment(chain3, S)["E"]
    prev = None
    for eps1 in (1e-1, 2e-2, 5e-3, 1e-3):
        r = hbci.solve(sp, eps1=eps1, eps2=0.0)
        assert r["E_var"] >= exact - 1e-12
        assert r["E_var"] + r["E_pt2"] <= r["E_var"] + 1e-15
        Vs = set(r["V"])
        assert all(int(sp.flip[a]) in Vs for a in Vs)
        pos = {d: t for t, d in enumerate(r["V"])}
        back = [pos[int(sp.flip[d])] for d in r["V"]]
        assert np.abs(r["c"][back] - r["c"]).max() < 1e-12
        if prev is not None:
            assert r["E_var"] <= prev + 1e-12
        prev = r["E_var"]
    assert abs(prev - exact) < 1e-3


def test_selection_against_the_definition(chain3):
    """One step from a fixed space: every added determinant has a coupling
    above eps1 or is the partner of one that has, and no other has."""
    sp = hbci.Space(chain3, (0, 1, 2))
    V = [sp.ref]
    c = np.ones(1)
    for _ in range(2):
        V = V + hbci.select(sp.H, V, c, 1e-2, sp.flip)
        _, c = hbci.lowest_in(sp.H, V, sp.flip)
    new = hbci.select(sp.H, V, c, 1e-2, sp.flip)
    strong = {a for a in range(len(sp.dets)) if a not in V
              and np.max(np.abs(sp.H[a, V] * c)) > 1e-2}
    assert set(new) == strong | {int(sp.flip[a]) for a in strong}
