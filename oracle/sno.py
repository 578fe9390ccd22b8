"""Summation natural orbitals (SNO): the virtual space of each increment
(test infrastructure only).

Paper, Methods ("Incremental Full Configuration Interaction", the SNO
paragraph, eq. 6): here a body is one occupied orbital i and all bodies share
the virtual orbitals V.  For each one-body term the CISD one-particle density
of the two electrons of i in {i} + V (CISD is exact for two electrons: the FCI
of that space, every other occupied orbital frozen) gives rho_i, its block
over V; an n-body term S takes rho_S = sum over i in S of rho_i (eq. 6),
keeps the natural orbitals of rho_S (its eigenvectors over V) whose
occupation numbers are at least 10^-eta, discards the others, and solves
the increment in S's occupied orbitals plus the kept natural orbitals, the
other occupied orbitals frozen.  The paper solves that increment with HBCI;
here with exact FCI (the same reading as for every increment).

Orbitals of the rotated increment problem, in order: S's occupied
orbitals, the kept natural orbitals (largest occupation first), the other
occupied orbitals (frozen core).
"""
from __future__ import annotations

import numpy as np

from . import fci, ifci, rdm


class _P:
    """The minimal problem record the oracle's FCI reads."""

    def __init__(self, h, eri, bodies, nocc, order, e_const=0.0):
        self.h, self.eri, self.bodies, self.nocc, self.order, self.e_const = h, eri, bodies, nocc, order, e_const
        self.n_orb = h.shape[0]
        self.n_bodies = len(bodies)


def one_body_density(h, eri, occ, vir, i, e_const=0.0):
    """rho_i over V: the virtual block of the one-particle density of the
    FCI of the two electrons of occupied orbital i in {i} + V."""
    others = [j for j in occ if j != i]
    p = _P(h, eri, [[i] + list(vir)] + [[j] for j in others], [1] * len(occ), 1, e_const)
    d = rdm.increment_densities(p, (0,))
    return d["gamma"][np.ix_(vir, vir)], d


def natural_orbitals(rho_sum, eta):
    """(U, occupations): the eigenvectors of rho_S with occupation >= 10^-eta,
    largest first (columns of U over V)."""
    w, U = np.linalg.eigh(rho_sum)
    order = np.argsort(-w, kind="stable")
    w, U = w[order], U[:, order]
    keep = w >= 10.0 ** (-eta)
    return U[:, keep], w[keep]


def rotated_problem(h, eri, occ, vir, S_occ, U, e_const=0.0):
    """The increment's problem in the rotated basis: orbitals (S's occupied,
    the natural orbitals U over V, the other occupied), one active body of
    the first two groups (its occupied orbitals first) and one frozen body
    per other occupied orbital."""
    n = h.shape[0]
    others = [j for j in occ if j not in S_occ]
    cols = []
    for i in S_occ:
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(e)
    for k in range(U.shape[1]):
        c = np.zeros(n)
        c[list(vir)] = U[:, k]
        cols.append(c)
    for j in others:
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(e)
    C = np.array(cols).T
    h2 = C.T @ h @ C
    eri2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", eri, C, C, C, C, optimize=True)
    na = len(S_occ) + U.shape[1]
    bodies = [list(range(na))] + [[na + t] for t in range(len(others))]
    return _P(h2, eri2, bodies, [len(S_occ)] + [1] * len(others), 1, e_const)


def sno_expansion(h, eri, occ, vir, order, eta, e_const=0.0):
    """Every increment's SNO energy and the expansion of eqs. 1-5:
    dict(E, n_keep, eps, by_order, total, e_ref)."""
    rho = {i: one_body_density(h, eri, occ, vir, i, e_const)[0] for i in occ}
    E, n_keep = {}, {}
    for S in ifci.increments(len(occ), order):
        S_occ = [occ[b] for b in S]
        U, _ = natural_orbitals(sum(rho[i] for i in S_occ), eta)
        p = rotated_problem(h, eri, occ, vir, S_occ, U, e_const)
        E[S] = fci.solve_increment(p, (0,))["E"]
        n_keep[S] = U.shape[1]
    e_ref = ifci.closed_shell_energy(h, eri, occ, e_const)
    eps, by_order, total = ifci.increments_from_energies(E, e_ref, order)
    return dict(E=E, n_keep=n_keep, eps=eps, by_order=by_order, total=total, e_ref=e_ref)
