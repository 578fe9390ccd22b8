"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, textbook special cases, invariances, brute force and the numbers
the paper prints.  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import certify, fci, hamiltonian, ifci, rdm, strings
from paper_2307_10675_amd import synthetic


# ------------------------------------------------------------------ strings
def _tuple_apply(occ, p, q):
    """E_pq on an ordered tuple of occupied orbitals by explicit
    anticommutation: a_q removes q at position i (sign (-1)^i), a+_p inserts p
    at position j (sign (-1)^j).  Independent of strings.excite."""
    occ = list(occ)
    if q not in occ:
        return None
    i = occ.index(q)
    sign = (-1) ** i
    occ.pop(i)
    if p in occ:
        return None
    j = sum(1 for o in occ if o < p)
    sign *= (-1) ** j
    occ.insert(j, p)
    return sign, tuple(occ)


@pytest.mark.parametrize("k,n", [(k, n) for k in range(1, 11) for n in range(0, k + 1)])
def test_strings_count_order_address(k, n):
    s = strings.strings(k, n)
    assert len(s) == math.comb(k, n)
    assert s == sorted(s)
    assert [strings.address(m) for m in s] == list(range(len(s)))


@pytest.mark.parametrize("k,n", [(4, 2), (6, 3), (7, 2), (8, 4)])
def test_excite_matches_operator_algebra(k, n):
    for m in strings.strings(k, n):
        occ = tuple(strings.occupied(m))
        for p in range(k):
            for q in range(k):
                a = strings.excite(m, p, q)
                b = _tuple_apply(occ, p, q)
                if b is None:
                    assert a is None
                else:
                    assert a == (b[0], sum(1 << o for o in b[1]))


@pytest.mark.parametrize("k,n", [(2, 1), (4, 2), (6, 3), (8, 4), (10, 5), (7, 3)])
def test_link_table_structure(k, n):
    table = strings.link_table(k, n)
    s = strings.strings(k, n)
    for I, row in enumerate(table):
        assert len(row) == n * (k - n + 1)
        pairs = {(max(p, q), min(p, q)) for p, q, _, _ in row}
        assert len(pairs) == len(row)          # one link per unordered pair at most
        for p, q, J, sg in row:
            assert strings.excite(s[I], p, q) == (sg, s[J])


def test_table1_counts():
    """Table 1: term counts are C(n_occ, k) of the increment enumerator and the
    FCI determinant counts are C(n_orb, n_occ)^2 (2 significant digits)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_problem_size.json")
    data = json.load(open(path))["molecules"]
    for name, row in data.items():
        n_occ = row["valence_electrons"] // 2
        counts = [math.comb(n_occ, k) for k in range(1, 5)]
        assert counts == row["terms"], name
        ndet = math.comb(row["active_orbitals"], n_occ) ** 2
        assert float(f"{ndet:.1e}") == row["fci_determinants"], name
    # the enumerator itself on the smallest molecule (TFA, 21 bodies)
    inc = ifci.increments(21, 4)
    assert [sum(1 for S in inc if len(S) == k) for k in range(1, 5)] == data["TFA"]["terms"]
    assert inc == sorted(inc, key=lambda S: (len(S), S))


# ------------------------------------------------------------------ Hamiltonian
def _two_orbital(h, g):
    """Textbook 2-orbital / 2-electron CI.  Singlet basis |11>, |22>,
    (|1a2b> + |2a1b>)/sqrt2; triplet h11 + h22 + (11|22) - (12|12)."""
    a = 2 * h[0, 0] + g[0, 0, 0, 0]
    b = 2 * h[1, 1] + g[1, 1, 1, 1]
    c = h[0, 0] + h[1, 1] + g[0, 0, 1, 1] + g[0, 1, 0, 1]
    K = g[0, 1, 0, 1]
    t1 = math.sqrt(2) * (h[0, 1] + g[0, 0, 0, 1])
    t2 = math.sqrt(2) * (h[0, 1] + g[1, 1, 0, 1])
    S = np.array([[a, K, t1], [K, b, t2], [t1, t2, c]])
    T = h[0, 0] + h[1, 1] + g[0, 0, 1, 1] - g[0, 1, 0, 1]
    return np.linalg.eigvalsh(S), T, a, b, K


@pytest.mark.parametrize("seed", range(8))
def test_two_orbital_closed_form(seed):
    p = synthetic.single(2, 12, seed)
    r = fci.solve_increment(p, (0,))
    sing, trip, *_ = _two_orbital(p.h, p.eri)
    assert abs(r["E"] - sing[0]) < 1e-13
    full = np.sort(np.linalg.eigvalsh(r["H"]))
    assert np.allclose(full, np.sort(np.append(sing, trip)), atol=1e-13)


def test_two_orbital_special_case():
    """h12 = (11|12) = (22|12) = 0: E = (a+b)/2 - sqrt((a-b)^2/4 + K^2)."""
    h = np.diag([-1.2, 0.3])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0], g[1, 1, 1, 1], g[0, 0, 1, 1] = 0.7, 0.6, 0.5
    g[1, 1, 0, 0] = 0.5
    for idx in [(0, 1, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1)]:
        g[idx] = 0.15
    p = synthetic.Problem(h, g, [[0, 1]], [1], 1)
    a, b, K = 2 * -1.2 + 0.7, 2 * 0.3 + 0.6, 0.15
    exact = 0.5 * (a + b) - math.sqrt(0.25 * (a - b) ** 2 + K * K)
    assert abs(fci.solve_increment(p, (0,))["E"] - exact) < 1e-14


def test_diagonal_integrals_give_hartree_fock():
    """h = diag(e), (pq|rs) = d_pq d_rs J_pr: H is diagonal; the lowest state is
    the closed shell 2 sum e_i + 2 sum_ij J_ij - sum_i J_ii."""
    n = 6
    e = np.array([-2.0, -1.5, -1.0, 1.0, 1.5, 2.0])
    rng = np.random.default_rng(3)
    A = rng.normal(0, 0.1, (n, 3))
    J = A @ A.T
    g = np.zeros((n,) * 4)
    for p_ in range(n):
        for r_ in range(n):
            g[p_, p_, r_, r_] = J[p_, r_]
    p = synthetic.Problem(np.diag(e), g, [list(range(n))], [3], 1)
    r = fci.solve_increment(p, (0,))
    H = r["H"]
    assert np.abs(H - np.diag(np.diag(H))).max() == 0.0
    occ = [0, 1, 2]
    hf = 2 * e[occ].sum() + 2 * J[np.ix_(occ, occ)].sum() - J[occ, occ].sum()
    assert abs(r["E"] - hf) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_slater_condon_equals_operator_algebra(seed):
    p = synthetic.chain(2, seed=seed, order=2)
    for S in [(0,), (1,), (0, 1)]:
        dets, _, act = fci.increment_dets(p.n_orb, p.bodies, p.nocc, S)
        H1 = hamiltonian.build(dets, p.h, p.eri, act, e_const=0.25)
        H2 = hamiltonian.build_by_operators(dets, p.h, p.eri, e_const=0.25)
        assert np.abs(H1 - H2).max() < 1e-13
        assert np.abs(H1 - H1.T).max() == 0.0


def test_slater_condon_equals_operator_algebra_three_bodies():
    p = synthetic.chain(3, seed=7, order=3)
    dets, _, act = fci.increment_dets(p.n_orb, p.bodies, p.nocc, (0, 2))
    H1 = hamiltonian.build(dets, p.h, p.eri, act)
    H2 = hamiltonian.build_by_operators(dets, p.h, p.eri)
    assert np.abs(H1 - H2).max() < 1e-13


def test_closed_shell_energy_is_slater_condon_diagonal():
    p = synthetic.chain(4, seed=11, order=1)
    ints = hamiltonian.SpinOrbitalIntegrals(p.h, p.eri)
    occ = [b[0] for b in p.bodies]
    m = sum(1 << o for o in occ)
    d = m | (m << p.n_orb)
    assert abs(hamiltonian.diagonal(ints, d) - ifci.closed_shell_energy(p.h, p.eri, occ)) < 1e-13


# ------------------------------------------------------------------ eigensolve / sector
@pytest.mark.parametrize("seed", range(4))
def test_sector_projection_vs_full_eigh(seed):
    p = synthetic.single(4, 12, seed)
    r = fci.solve_increment(p, (0,))
    w, v = np.linalg.eigh(r["H"])
    n = r["n_str"]
    sym = [i for i in range(len(w)) if np.abs(v[:, i].reshape(n, n) - v[:, i].reshape(n, n).T).max() < 1e-8]
    assert abs(w[sym[0]] - r["E"]) < 1e-12
    C = r["c"].reshape(n, n)
    assert np.abs(C - C.T).max() < 1e-12
    # even spin: <S^2> = S(S+1) with S even
    s2 = fci.spin_squared(r["c"], r["dets"], p.n_orb)
    S = (-1 + math.sqrt(1 + 4 * s2)) / 2
    assert abs(S - round(S)) < 1e-8 and round(S) % 2 == 0


def _det(alpha, beta, n):
    """Determinant bit pattern: spatial orbitals `alpha` with spin alpha,
    `beta` with spin beta (bit n + p)."""
    return sum(1 << p for p in alpha) | sum(1 << (n + p) for p in beta)


def test_spin_squared_two_electrons_in_two_orbitals():
    """<S^2> pinned on textbook two-electron states (two spatial orbitals):
    a closed shell is a singlet (0); the high-spin determinant |1a 2a> has
    S = Sz = 1 (2); one open-shell Ms = 0 determinant |1a 2b> is half singlet,
    half triplet (1); of the two combinations |1a 2b> +- |2a 1b> one is the
    singlet (0) and the other the Ms = 0 triplet (2), and the one with a
    symmetric coefficient matrix C[alpha][beta] is the singlet."""
    n = 2
    assert abs(fci.spin_squared(np.array([1.0]), [_det([0], [0], n)], n)) < 1e-14
    assert abs(fci.spin_squared(np.array([1.0]), [_det([0, 1], [], n)], n) - 2.0) < 1e-14
    assert abs(fci.spin_squared(np.array([1.0]), [_det([0], [1], n)], n) - 1.0) < 1e-14
    dets = [_det([0], [1], n), _det([1], [0], n)]
    plus = fci.spin_squared(np.array([1.0, 1.0]), dets, n)
    minus = fci.spin_squared(np.array([1.0, -1.0]), dets, n)
    assert sorted([round(plus, 12), round(minus, 12)]) == [0.0, 2.0]
    # the library's determinant order (alpha creators first, ascending):
    # C[a][b] = C[b][a] for strings a = {1}, b = {2} is the + combination
    assert abs(plus) < 1e-14 and abs(minus - 2.0) < 1e-14


def test_spin_squared_high_spin_and_normalisation():
    """Three electrons in three orbitals, all alpha: S = 3/2, <S^2> = 15/4
    whatever the (unnormalised) coefficient; a mixture of Ms = 0 singlet and
    triplet weights 1:3 gives 3/4 * 2 = 1.5."""
    n = 3
    assert abs(fci.spin_squared(np.array([2.5]), [_det([0, 1, 2], [], n)], n) - 3.75) < 1e-14
    dets = [_det([0], [1], n), _det([1], [0], n)]
    s = np.array([1.0, 1.0]) / np.sqrt(2.0)     # singlet
    t = np.array([1.0, -1.0]) / np.sqrt(2.0)    # Ms = 0 triplet
    c = 0.5 * s + np.sqrt(0.75) * t
    assert abs(fci.spin_squared(c, dets, n) - 1.5) < 1e-14


def test_workload0_singlet_and_reference():
    p = synthetic.workload(0)
    r = fci.solve_increment(p, (0,))
    assert abs(fci.spin_squared(r["c"], r["dets"], p.n_orb)) < 1e-10
    assert r["E"] <= ifci.reference_energy(p) + 1e-14


def _rotate(h, g, U):
    h2 = U.T @ h @ U
    g2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", g, U, U, U, U, optimize=True)
    return h2, g2


@pytest.mark.parametrize("seed", [0, 1])
def test_fci_invariant_under_orbital_rotation(seed):
    p = synthetic.single(5, 12, seed)
    U, _ = np.linalg.qr(np.random.default_rng(seed + 100).normal(size=(5, 5)))
    h2, g2 = _rotate(p.h, p.eri, U)
    q = synthetic.Problem(h2, g2, p.bodies, p.nocc, 1)
    e1 = fci.solve_increment(p, (0,))["E"]
    e2 = fci.solve_increment(q, (0,))["E"]
    assert abs(e1 - e2) < 1e-11


# ------------------------------------------------------------------ expansion
@pytest.mark.parametrize("nb,n", [(3, 1), (4, 2), (5, 3), (6, 6), (10, 3), (16, 4), (12, 5), (12, 4), (7, 4)])
def test_weights_recursion_equals_closed_form(nb, n):
    assert ifci.weights(nb, n) == ifci.weights_closed(nb, n)


def test_weights_examples():
    assert ifci.weights_closed(10, 3) == [28, -7, 1]
    assert ifci.weights_closed(16, 4) == [-364, 78, -12, 1]
    assert ifci.weights_closed(12, 5) == [210, -84, 28, -7, 1]
    assert ifci.weights_closed(6, 6) == [0, 0, 0, 0, 0, 1]


def test_increments_from_energies_matches_eqs_2_to_5():
    """Spell eqs. 2-5 out term by term for four bodies."""
    rng = np.random.default_rng(0)
    S_all = ifci.increments(4, 4)
    E = {S: float(rng.normal()) for S in S_all}
    eref = 0.3
    eps, by, tot = ifci.increments_from_energies(E, eref, 4)
    Ec = {S: E[S] - eref for S in S_all}
    i, j, k, l = 0, 1, 2, 3
    e1 = {(a,): Ec[(a,)] for a in range(4)}
    e2 = {(a, b): Ec[(a, b)] - e1[(a,)] - e1[(b,)] for a, b in itertools.combinations(range(4), 2)}
    e3 = {(a, b, c): Ec[(a, b, c)] - e2[(a, b)] - e2[(a, c)] - e2[(b, c)] - e1[(a,)] - e1[(b,)] - e1[(c,)]
          for a, b, c in itertools.combinations(range(4), 3)}
    e4 = (Ec[(i, j, k, l)] - e3[(i, j, k)] - e3[(i, j, l)] - e3[(i, k, l)] - e3[(j, k, l)]
          - e2[(i, j)] - e2[(i, k)] - e2[(i, l)] - e2[(j, k)] - e2[(j, l)] - e2[(k, l)]
          - e1[(i,)] - e1[(j,)] - e1[(k,)] - e1[(l,)])
    for d in (e1, e2, e3):
        for S, v in d.items():
            assert abs(eps[S] - v) < 1e-12
    assert abs(eps[(0, 1, 2, 3)] - e4) < 1e-12
    # eq. 1 truncated at 4 with weights
    w = ifci.weights_closed(4, 4)
    assert abs(tot - (eref + sum(w[len(S) - 1] * Ec[S] for S in S_all))) < 1e-12


def test_full_order_identity_three_bodies():
    """Summing every increment reproduces the full correlation energy."""
    p = synthetic.chain(3, seed=21, order=3)
    res = ifci.run(p)
    full = res["E"][(0, 1, 2)]
    assert abs(res["total"] - full) < 1e-12
    assert abs(math.fsum(res["eps"].values()) - (full - res["e_ref"])) < 1e-12


@pytest.mark.slow
def test_full_order_identity_four_bodies():
    p = synthetic.chain(4, seed=22, order=4)
    res = ifci.run(p)
    full = res["E"][(0, 1, 2, 3)]
    assert abs(res["total"] - full) < 1e-12


def test_separable_bodies():
    """Non-interacting bodies: every increment of two or more bodies vanishes,
    and the total is E_ref plus each body's 2o2e closed-form correlation."""
    p = synthetic.separable(4, seed=5, order=3)
    res = ifci.run(p)
    for S, e in res["eps"].items():
        if len(S) >= 2:
            assert abs(e) < 1e-12, S
    corr = 0.0
    for orbs in p.bodies:
        ix = np.ix_(orbs, orbs)
        hb = p.h[ix]
        gb = p.eri[np.ix_(orbs, orbs, orbs, orbs)]
        sing, trip, a, *_ = _two_orbital(hb, gb)
        assert sing[0] < trip
        corr += sing[0] - a
    assert abs(res["total"] - (res["e_ref"] + corr)) < 1e-12


def test_variational_and_monotone():
    p = synthetic.chain(4, seed=9, order=3)
    res = ifci.run(p)
    for S, e in res["E"].items():
        assert e <= res["e_ref"] + 1e-12
        for k in range(1, len(S)):
            for T in itertools.combinations(S, k):
                assert e <= res["E"][T] + 1e-12


def test_frozen_bodies_do_not_change_core_energy_with_all_bodies():
    """With S = every body the space is the whole half-filled FCI space of the
    chain; its energy equals a one-body problem over the same orbitals."""
    p = synthetic.chain(2, seed=4, order=2)
    e_all = fci.solve_increment(p, (0, 1))["E"]
    q = synthetic.Problem(p.h, p.eri, [p.bodies[0][:1] + p.bodies[1][:1] + p.bodies[0][1:] + p.bodies[1][1:]],
                          [2], 1)
    assert abs(fci.solve_increment(q, (0,))["E"] - e_all) < 1e-12


# ------------------------------------------------------------------ RDMs
def test_rdm_traces_energy_and_symmetry():
    p = synthetic.chain(3, seed=2, order=2)
    p.e_const = 0.125
    r = fci.solve_increment(p, (0, 2))
    g, G = rdm.densities(r["c"], r["dets"], p.n_orb)
    N = 6
    assert abs(np.trace(g) - N) < 1e-12
    assert abs(np.einsum("pprr->", G) - N * (N - 1)) < 1e-11
    E = np.sum(p.h * g) + 0.5 * np.sum(p.eri * G) + p.e_const
    assert abs(E - r["E"]) < 1e-12
    w = np.linalg.eigvalsh(g)
    assert w.min() > -1e-12 and w.max() < 2 + 1e-12
    assert np.abs(g - g.T).max() < 1e-13
    assert np.abs(G - G.transpose(2, 3, 0, 1)).max() < 1e-12
    assert np.abs(G - G.transpose(1, 0, 3, 2)).max() < 1e-12


def _orbit(p, q, r, s):
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def test_ifci_gradient_matches_central_differences():
    """Hellmann-Feynman gradient of the truncated expansion vs central
    differences of the oracle energy, step 1e-5."""
    p = synthetic.chain(3, seed=13, order=2)
    E0, dh, dg = rdm.ifci_gradient(p)
    assert abs(E0 - ifci.run(p)["total"]) < 1e-12
    step = 1e-5

    def energy(h, g):
        q = synthetic.Problem(h, g, p.bodies, p.nocc, p.order)
        return ifci.run(q)["total"]

    for (a, b) in [(0, 0), (1, 3), (2, 5), (4, 4)]:
        hp, hm = p.h.copy(), p.h.copy()
        for (x, y) in {(a, b), (b, a)}:
            hp[x, y] += step
            hm[x, y] -= step
        fd = (energy(hp, p.eri) - energy(hm, p.eri)) / (2 * step)
        an = dh[a, b] + (dh[b, a] if a != b else 0.0)
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (a, b)
    for idx in [(0, 0, 0, 0), (0, 1, 2, 3), (1, 1, 4, 4), (0, 2, 0, 2), (3, 5, 1, 4)]:
        orb = _orbit(*idx)
        gp, gm = p.eri.copy(), p.eri.copy()
        for t in orb:
            gp[t] += step
            gm[t] -= step
        fd = (energy(p.h, gp) - energy(p.h, gm)) / (2 * step)
        an = sum(dg[t] for t in orb)
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), idx


# ------------------------------------------------------------------ certifier
def test_sigma_rows_equal_dense_product():
    p = synthetic.chain(3, seed=1, order=3)
    dets, n_str, act = fci.increment_dets(p.n_orb, p.bodies, p.nocc, (0, 1, 2))
    H = hamiltonian.build(dets, p.h, p.eri, act)
    c = synthetic.random_vector(len(dets), 5)
    rows = list(range(0, len(dets), 37))
    got = certify.sigma_rows(rows, dets, c, p.h, p.eri, act)
    assert np.abs(got - (H @ c)[rows]).max() < 1e-12
    e, v, gap = fci.lowest_symmetric(H, n_str)
    r = H @ v - e * v
    assert certify.residual_bound(np.linalg.norm(r), gap) < 1e-12


def test_sigma_rows_strings_equal_dense_product():
    """String-addressed rows (no determinant list) against the dense
    Slater-Condon product of a single body with no core."""
    p = synthetic.single(6, 12, 11)
    dets, n_str, act = fci.increment_dets(p.n_orb, p.bodies, p.nocc, (0,))
    H = hamiltonian.build(dets, p.h, p.eri, act)
    c = synthetic.random_vector(len(dets), 6)
    rows = list(range(0, len(dets), 13))
    got = certify.sigma_rows_strings(rows, 3, c, p.h, p.eri)
    assert np.abs(got - (H @ c)[rows]).max() < 1e-12
    assert np.abs(got - certify.sigma_rows(rows, dets, c, p.h, p.eri, act)).max() < 1e-12
