"""Density matrices and the analytic gradient of the iFCI energy
(test infrastructure only).

For a normalised state Psi over full-space determinants:
  gamma_pq    = <Psi| E_pq |Psi>
  Gamma_pqrs  = <Psi| E_pq E_rs |Psi> - delta_qr gamma_ps      (spin-summed,
                                                                 chemists' order)
so that E = sum_pq h_pq gamma_pq + 1/2 sum_pqrs (pq|rs) Gamma_pqrs + e_const.
Both are built by applying the second-quantised E_pq to the determinants of
Psi (full space, core orbitals included), never from any factorised form.

Gradient (Hellmann-Feynman, each tensor entry an independent variable):
dE/dh_pq = gamma_pq and dE/d(pq|rs) = 1/2 Gamma_pqrs for every exact
eigenstate.  For the truncated expansion E = E_ref + sum_T w_|T| (E(T) - E_ref)
(eqs. 1-5), dE/dx = (1 - sum_T w_|T|) dE_ref/dx + sum_T w_|T| dE(T)/dx.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fci, hamiltonian, ifci


def _E_on(det: int, p: int, q: int, n: int):
    out = []
    for s in (0, 1):
        r = hamiltonian.apply_string(det, [("+", p + s * n), ("-", q + s * n)])
        if r is not None:
            out.append(r)
    return out


def densities(c: np.ndarray, dets, n_orb: int):
    """(gamma, Gamma) of the state sum_i c_i |dets[i]>, normalised here."""
    c = np.asarray(c, dtype=np.float64)
    c = c / np.sqrt(c @ c)
    n = n_orb
    col = {}
    rows, cols, vals = [], [], []
    for i, d in enumerate(dets):
        if c[i] == 0.0:
            continue
        for r in range(n):
            for s in range(n):
                for sign, d1 in _E_on(d, r, s, n):
                    j = col.setdefault(d1, len(col))
                    rows.append(r * n + s)
                    cols.append(j)
                    vals.append(sign * c[i])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n * n, len(col)))   # rows: E_rs |Psi>
    G = (M @ M.T).toarray()                                            # G[qp, rs] = <E_qp Psi|E_rs Psi>
    psi = np.zeros(len(col))
    for i, d in enumerate(dets):
        if d in col:
            psi[col[d]] = c[i]
    gamma = (M @ psi).reshape(n, n)                                   # <Psi|E_pq Psi>
    G4 = G.reshape(n, n, n, n)                                        # [q, p, r, s]
    Gamma = G4.transpose(1, 0, 2, 3).copy()                           # [p, q, r, s]
    for q in range(n):
        Gamma[:, q, q, :] -= gamma
    return gamma, Gamma


def reference_densities(problem):
    """gamma, Gamma of the reference determinant (all bodies at reference)."""
    occ = [o for b, orbs in enumerate(problem.bodies) for o in orbs[: problem.nocc[b]]]
    n = problem.n_orb
    m = sum(1 << o for o in occ)
    return densities(np.array([1.0]), [m | (m << n)], n)


def increment_densities(problem, S):
    r = fci.solve_increment(problem, S)
    g, G = densities(r["c"], r["dets"], problem.n_orb)
    return dict(E=r["E"], gamma=g, Gamma=G, gap=r["gap"])


def accumulate_gradient(problem, densities_in_order, weights_by_size=None):
    """(E_iFCI, dE/dh, dE/d(pq|rs)) from the densities of every increment.

    densities_in_order yields (S, increment_densities(problem, S)) for every
    increment S of ifci.increments(n_bodies, order), in that order; the sums
    are taken in that order too, so a caller that computes the densities in
    parallel gets the same numbers as the serial `ifci_gradient`."""
    import math
    nb, order = problem.n_bodies, problem.order
    w = weights_by_size or ifci.weights_closed(nb, order)
    g_ref, G_ref = reference_densities(problem)
    e_ref = ifci.reference_energy(problem)
    dh = np.zeros_like(problem.h)
    deri = np.zeros_like(problem.eri)
    w_sum = 0.0
    terms = [e_ref]
    expect = iter(ifci.increments(nb, order))
    for S, d in densities_in_order:
        if tuple(S) != next(expect):
            raise ValueError("densities must come in increment order")
        wt = w[len(S) - 1]
        dh += wt * d["gamma"]
        deri += 0.5 * wt * d["Gamma"]
        terms.append(wt * (d["E"] - e_ref))
        w_sum += wt
    if next(expect, None) is not None:
        raise ValueError("densities missing for some increments")
    dh += (1.0 - w_sum) * g_ref
    deri += 0.5 * (1.0 - w_sum) * G_ref
    return math.fsum(terms), dh, deri


def ifci_gradient(problem, weights_by_size=None):
    """(E_iFCI, dE/dh, dE/d(pq|rs)) of the expansion truncated at problem.order."""
    gen = ((S, increment_densities(problem, S)) for S in ifci.increments(problem.n_bodies, problem.order))
    return accumulate_gradient(problem, gen, weights_by_size)
