"""Heat-bath selected CI with Epstein-Nesbet second-order correction (HBCI)
for one increment (test infrastructure only).

Paper, Methods ("Incremental Full Configuration Interaction", the HBCI
paragraph): each increment energy is computed by a selected CI.  A set of
important determinants is chosen for a variational treatment, the space
outside it is then reached by second-order Epstein-Nesbet perturbation
theory, and two thresholds steer the two steps (eps1 for the variational
selection, eps2 for the perturbative one; 1 mEh and 1 uEh in the paper).
The paper gives no more than that; the method it cites is heat-bath CI
(Holmes, Tubman and Umrigar, J. Chem. Theory Comput. 12, 3674 (2016)),
whose definitions are restated here.

Selection.  With a variational space V and its lowest eigenvector c (unit
norm), the determinants added are every a outside V with
max over i in V of |H_ai c_i| > eps1.  The heat-bath algorithm finds them by
walking integrals sorted by magnitude; the set is the same, so the oracle
tests every pair directly on the dense Hamiltonian.

Iteration.  V starts as the increment's reference determinant (the closed
shell that defines E_ref, c = 1).  Each step adds the selected determinants
and re-solves for the lowest root in V; it ends when a step adds nothing or
after max_iter steps.

Readings (the paper is silent on them):
* spin: V is kept closed under exchanging the alpha and beta strings (every
  added determinant brings its spin-flipped partner), and the root is taken
  in the sector symmetric under that exchange, as for the exact increments;
* PT2 (deterministic, screened as in heat-bath CI): for a outside V,
  N_a = sum over i in V with |H_ai c_i| > eps2 of H_ai c_i, and
  E_PT2 = sum_a N_a^2 / (E_var - H_aa).

Parity: pinned by tests/test_oracle_hbci.py (eps1 = 0 gives the exact
increment energy; the two-orbital two-electron closed forms of the
variational root, of the selection threshold and of the second-order energy;
E_PT2 as the second derivative of an exactly diagonalised Epstein-Nesbet
partitioned Hamiltonian; the variational bound).
"""
from __future__ import annotations

import math

import numpy as np

from . import fci, hamiltonian


def flip(det: int, n_orb: int) -> int:
    """The determinant with its alpha and beta strings exchanged."""
    mask = (1 << n_orb) - 1
    return (det >> n_orb) | ((det & mask) << n_orb)


def reference_det(problem, S) -> int:
    """The closed shell of increment S: the core and S's occupied orbitals
    doubly occupied (the determinant of the reference energy)."""
    occ = [o for b, orbs in enumerate(problem.bodies) for o in orbs[: problem.nocc[b]]]
    a = sum(1 << o for o in occ)
    return a | (a << problem.n_orb)


class Space:
    """The increment's full determinant list and dense Hamiltonian (the
    oracle's Slater-Condon build), with the flip permutation."""

    def __init__(self, problem, S):
        r = fci.increment_dets(problem.n_orb, problem.bodies, problem.nocc, S)
        self.dets, self.n_str, self.active = r
        self.n_orb = problem.n_orb
        self.H = hamiltonian.build(self.dets, problem.h, problem.eri, self.active, problem.e_const)
        self.index = {d: i for i, d in enumerate(self.dets)}
        self.flip = np.array([self.index[flip(d, self.n_orb)] for d in self.dets])
        self.ref = self.index[reference_det(problem, S)]


def lowest_in(H: np.ndarray, V: list[int], flip_idx: np.ndarray):
    """(E, c) of the lowest root of H over V in the flip-symmetric sector;
    V is closed under flip.  c is over V's order, unit norm."""
    pos = {d: t for t, d in enumerate(V)}
    cols = []
    for t, d in enumerate(V):
        f = int(flip_idx[d])
        if f == d:
            v = np.zeros(len(V))
            v[t] = 1.0
            cols.append(v)
        elif d < f:
            v = np.zeros(len(V))
            v[t] = v[pos[f]] = 1.0 / math.sqrt(2.0)
            cols.append(v)
    B = np.array(cols).T
    Hv = H[np.ix_(V, V)]
    w, u = np.linalg.eigh(B.T @ Hv @ B)
    return float(w[0]), fci.normalise_sign(B @ u[:, 0])


def select(H: np.ndarray, V: list[int], c: np.ndarray, eps1: float, flip_idx: np.ndarray) -> list[int]:
    """Determinants outside V with max_i |H_ai c_i| > eps1, and their flip
    partners, in increasing list order."""
    inV = np.zeros(H.shape[0], dtype=bool)
    inV[V] = True
    outside = np.flatnonzero(~inV)
    couple = np.abs(H[np.ix_(outside, V)] * c[None, :])       # |H_ai c_i|, a outside V
    hit = outside[(couple > eps1).any(axis=1)]
    out = set(int(a) for a in hit)
    out |= {int(flip_idx[a]) for a in hit if not inV[flip_idx[a]]}
    return sorted(out)


def pt2(H: np.ndarray, V: list[int], c: np.ndarray, e_var: float, eps2: float):
    """(E_PT2, number of external determinants with a nonzero N_a)."""
    inV = np.zeros(H.shape[0], dtype=bool)
    inV[V] = True
    outside = np.flatnonzero(~inV)
    hc = H[np.ix_(outside, V)] * c[None, :]                   # H_ai c_i
    keep = np.abs(hc) > eps2
    terms = []
    for row, a in enumerate(outside):
        parts = hc[row, keep[row]]
        if parts.size == 0:
            continue
        n_a = math.fsum(parts)
        terms.append(n_a * n_a / (e_var - H[a, a]))
    return math.fsum(terms), len(terms)


def solve(space: Space, eps1: float, eps2: float, max_iter: int = 32):
    """HBCI of one increment: dict(E_var, E_pt2, E, V, c, n_iter, converged)."""
    H, fl = space.H, space.flip
    V = [space.ref]
    e_var, c = float(H[space.ref, space.ref]), np.ones(1)
    n_iter, converged = 0, False
    while n_iter < max_iter:
        new = select(H, V, c, eps1, fl)
        n_iter += 1
        if not new:
            converged = True
            break
        V = V + new
        e_var, c = lowest_in(H, V, fl)
    e2, n_ext = pt2(H, V, c, e_var, eps2)
    return dict(E_var=e_var, E_pt2=e2, E=e_var + e2, V=V, c=c, n_iter=n_iter, converged=converged,
                n_ext=n_ext)


def solve_increment(problem, S, eps1: float, eps2: float, max_iter: int = 32):
    """HBCI of increment S of `problem` (total energy, e_const included)."""
    sp = Space(problem, S)
    r = solve(sp, eps1, eps2, max_iter)
    r["dets"] = [sp.dets[i] for i in r["V"]]
    r["space"] = sp
    return r
