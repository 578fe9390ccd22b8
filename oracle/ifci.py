"""Incremental expansion (test infrastructure only).

Paper, Methods ("Incremental Full Configuration Interaction"):
* eq. 1: E_c = sum_i eps_i + sum_{i>j} eps_ij + sum_{i>j>k} eps_ijk + ...
* eqs. 2-5: eps_i = E_c(i); eps_ij = E_c(ij) - eps_i - eps_j; eps_ijk and
  eps_ijkl subtract every increment of every proper non-empty subset.
* E_c(S) is the correlation energy of the calculation that includes only the
  bodies of S; the reference energy is that of one determinant in the
  localized basis (GVB-PP paragraph).  E_c(empty) = 0.

Truncating eq. 1 at order n gives E = E_ref + sum_{|S| <= n} eps_S.  Every
E_c(T) enters that sum with a weight w_|T| that depends only on |T|, the
number of bodies N_b and n; `weights` computes it from the recursion itself
and `weights_closed` from the inclusion-exclusion count
w_k = sum_{m=0}^{n-k} (-1)^m C(N_b - k, m).
"""
from __future__ import annotations

import itertools
import math

from . import fci


def increments(n_bodies: int, order: int):
    """Every body set S with 1 <= |S| <= order, by size then lexicographic."""
    out = []
    for k in range(1, order + 1):
        out += list(itertools.combinations(range(n_bodies), k))
    return out


def closed_shell_energy(h, eri, occ, e_const: float = 0.0) -> float:
    """Energy of the determinant with the orbitals `occ` doubly occupied:
    e_const + sum_i 2 h_ii + sum_ij [2 (ii|jj) - (ij|ji)]."""
    terms = [e_const]
    terms += [2.0 * h[i, i] for i in occ]
    terms += [2.0 * eri[i, i, j, j] - eri[i, j, j, i] for i in occ for j in occ]
    return math.fsum(terms)


def reference_energy(problem) -> float:
    occ = [o for b, orbs in enumerate(problem.bodies) for o in orbs[: problem.nocc[b]]]
    return closed_shell_energy(problem.h, problem.eri, occ, problem.e_const)


def increments_from_energies(E: dict, e_ref: float, order: int):
    """eqs. 2-5: eps_S = E_c(S) - sum over proper non-empty subsets T of eps_T,
    with E_c(S) = E(S) - E_ref.  Returns (eps, order sums, E_total)."""
    eps = {}
    for S in sorted(E, key=lambda s: (len(s), s)):
        sub = [eps[T] for k in range(1, len(S)) for T in itertools.combinations(S, k)]
        eps[S] = math.fsum([E[S] - e_ref] + [-x for x in sub])
    by_order = [math.fsum(eps[S] for S in eps if len(S) == k) for k in range(1, order + 1)]
    total = math.fsum([e_ref] + by_order)
    return eps, by_order, total


def weights(n_bodies: int, order: int):
    """w_k obtained by running the recursion of eqs. 2-5 on symbolic unit
    energies: the coefficient of E_c(T) (any |T| = k) in sum_{|S|<=n} eps_S."""
    # eps_S as a vector of coefficients over subsets; by symmetry only |T| matters
    coef = {}
    for S in increments(n_bodies, order):
        c = {S: 1}
        for k in range(1, len(S)):
            for T in itertools.combinations(S, k):
                for U, v in coef[T].items():
                    c[U] = c.get(U, 0) - v
        coef[S] = c
    total = {}
    for S, c in coef.items():
        for U, v in c.items():
            total[U] = total.get(U, 0) + v
    return [total[tuple(range(k))] for k in range(1, order + 1)]


def weights_closed(n_bodies: int, order: int):
    return [sum((-1) ** m * math.comb(n_bodies - k, m) for m in range(order - k + 1))
            for k in range(1, order + 1)]


def run(problem, keep_vectors: bool = False):
    """The whole expansion up to problem.order with exact FCI per increment."""
    e_ref = reference_energy(problem)
    E, gap, vec = {}, {}, {}
    for S in increments(problem.n_bodies, problem.order):
        r = fci.solve_increment(problem, S)
        E[S] = r["E"]
        gap[S] = r["gap"]
        if keep_vectors:
            vec[S] = r
    eps, by_order, total = increments_from_energies(E, e_ref, problem.order)
    return dict(E=E, eps=eps, by_order=by_order, total=total, e_ref=e_ref, gap=gap, vec=vec)
