"""Determinant space of one increment and its lowest root (test infrastructure only).

Reading of the paper (Methods, iFCI): the correlation energy E_c(S) of an
increment comes from a calculation restricted to the occupied orbitals of
S.  Here a body is a group of orbitals (its occupied orbitals and the virtual
orbitals that belong to it); the calculation for a set S of bodies correlates
every orbital of those bodies, keeps the occupied orbitals of all other
bodies doubly occupied and leaves their virtual orbitals empty.  The paper's
solver (HBCI) approximates FCI in that space; this oracle gives its exact
limit.

Target root: the lowest eigenvalue of H restricted to the space, searched in
the sector whose coefficient matrix C[alpha string, beta string] is symmetric
(C = C^T).  With equal alpha and beta counts this sector holds exactly the
states of even total spin, which contains the closed-shell singlet the
reference describes; the antisymmetric sector (odd spin, e.g. triplets) is
excluded even when it lies lower.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian, strings


def increment_orbitals(bodies, nocc, S):
    """(active, core, deleted) spatial orbital lists of increment S."""
    active, core, deleted = [], [], []
    for b, orbs in enumerate(bodies):
        if b in S:
            active += list(orbs)
        else:
            core += list(orbs[: nocc[b]])
            deleted += list(orbs[nocc[b]:])
    return sorted(active), sorted(core), sorted(deleted)


def increment_dets(n_orb, bodies, nocc, S):
    """Full-space determinants of increment S, alpha string major.

    Returns (dets, n_str, active) where dets[i * n_str + j] combines the
    i-th and j-th active strings (increasing active bitmask order) with the
    core orbitals doubly occupied."""
    active, core, _ = increment_orbitals(bodies, nocc, S)
    n_el = sum(nocc[b] for b in S)
    core_mask = sum(1 << c for c in core)
    full = []
    for s in strings.strings(len(active), n_el):
        m = core_mask
        for i, p in enumerate(active):
            if s >> i & 1:
                m |= 1 << p
        full.append(m)
    dets = [a | (b << n_orb) for a in full for b in full]
    return dets, len(full), active


def sector_basis(n_str: int) -> np.ndarray:
    """Orthonormal basis of symmetric coefficient matrices, as columns of an
    (n_str^2, n_str (n_str + 1) / 2) matrix: |a,a> and (|a,b> + |b,a>)/sqrt 2."""
    cols = []
    for a in range(n_str):
        for b in range(a, n_str):
            v = np.zeros(n_str * n_str)
            if a == b:
                v[a * n_str + a] = 1.0
            else:
                v[a * n_str + b] = v[b * n_str + a] = 1.0 / np.sqrt(2.0)
            cols.append(v)
    return np.array(cols).T


def normalise_sign(c: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry (lowest index on ties) positive."""
    i = int(np.argmax(np.abs(c)))
    return c if c[i] > 0 else -c


def lowest_symmetric(H: np.ndarray, n_str: int):
    """Lowest eigenpair of H in the C = C^T sector: (E, c, gap) with c over
    the full determinant list and gap to the next root of the sector."""
    P = sector_basis(n_str)
    w, v = np.linalg.eigh(P.T @ H @ P)
    c = normalise_sign(P @ v[:, 0])
    gap = float(w[1] - w[0]) if len(w) > 1 else float("inf")
    return float(w[0]), c, gap


def solve_increment(problem, S):
    """Exact E(S) (total energy, e_const included), its vector, the gap and
    the determinant list of increment S."""
    dets, n_str, active = increment_dets(problem.n_orb, problem.bodies, problem.nocc, S)
    H = hamiltonian.build(dets, problem.h, problem.eri, active, problem.e_const)
    e, c, gap = lowest_symmetric(H, n_str)
    return dict(E=e, c=c, gap=gap, dets=dets, n_str=n_str, active=active, H=H)


def spin_squared(c: np.ndarray, dets, n_orb: int) -> float:
    """<S^2> of the vector c over `dets` (diagnostic: 0 for a singlet)."""
    index = {d: i for i, d in enumerate(dets)}
    n_a = bin(dets[0] & ((1 << n_orb) - 1)).count("1")
    n_b = bin(dets[0] >> n_orb).count("1")
    sz = 0.5 * (n_a - n_b)
    # S^2 = S_- S_+ + S_z (S_z + 1); S_+ = sum_p a+_pa a_pb
    plus = {}
    for i, d in enumerate(dets):
        if c[i] == 0.0:
            continue
        for p in range(n_orb):
            r = hamiltonian.apply_string(d, [("+", p), ("-", p + n_orb)])
            if r is not None:
                plus[r[1]] = plus.get(r[1], 0.0) + r[0] * c[i]
    norm_plus = sum(v * v for v in plus.values())
    nrm = float(c @ c)
    del index
    return norm_plus / nrm + sz * (sz + 1)
