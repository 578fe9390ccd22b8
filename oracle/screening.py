"""Connected n-body (CnB) screening of the incremental expansion (test
infrastructure only).

Paper, Methods ("Incremental Full Configuration Interaction", the CnB
paragraph): increments of three or more bodies whose bodies are not
connected are dropped, with a screening parameter C = 10^-4.6 Eh applied at
n = 3 and 4; the criterion itself is given in the paper's Supplementary
Information and its references, which are not available here.  The reading
taken (the same on the device path):

* two bodies i and j are connected when their pair increment satisfies
  |eps_ij| >= C, eps_ij = E_c(ij) - E_c(i) - E_c(j) (eq. 3);
* an increment S with |S| >= 3 is kept when its bodies form a connected
  graph under that relation; every increment of one or two bodies is kept;
* a dropped increment contributes eps_S = 0, and a kept one is the
  recursion of eqs. 2-5 over its subsets, with the dropped subsets at zero:
  eps_S = E_c(S) - sum over proper non-empty subsets T of eps_T.

With C = 0 nothing is dropped and the sums are those of eqs. 1-5.
"""
from __future__ import annotations

import itertools
import math

from . import ifci


def pair_increments(E: dict, e_ref: float, n_bodies: int):
    """{(i, j): eps_ij} for every pair, from the increment energies E(S)."""
    return {(i, j): (E[(i, j)] - e_ref) - (E[(i,)] - e_ref) - (E[(j,)] - e_ref)
            for i, j in itertools.combinations(range(n_bodies), 2)}


def connected(S, linked) -> bool:
    """Whether the bodies of S form one connected graph, `linked(i, j)`
    telling whether an edge joins i < j (breadth-first search from S[0])."""
    seen = {S[0]}
    todo = [S[0]]
    while todo:
        a = todo.pop()
        for b in S:
            if b not in seen and linked(min(a, b), max(a, b)):
                seen.add(b)
                todo.append(b)
    return len(seen) == len(S)


def cnb_keep(E: dict, e_ref: float, n_bodies: int, order: int, threshold: float):
    """The increments kept by the screening, in increment order (needs E for
    every increment of one and two bodies)."""
    eps2 = pair_increments(E, e_ref, n_bodies)
    keep = []
    for S in ifci.increments(n_bodies, order):
        if len(S) <= 2 or connected(S, lambda i, j: abs(eps2[(i, j)]) >= threshold):
            keep.append(S)
    return keep


def screened_expansion(E: dict, e_ref: float, order: int, keep):
    """(eps, order sums, E_total) of the screened expansion: eps_S of a kept
    S by the recursion over its subsets (dropped subsets at zero), 0 for a
    dropped one.  E needs the kept increments only."""
    kept = set(keep)
    eps = {}
    for S in sorted(kept, key=lambda s: (len(s), s)):
        sub = [eps.get(T, 0.0) for k in range(1, len(S)) for T in itertools.combinations(S, k)]
        eps[S] = math.fsum([E[S] - e_ref] + [-x for x in sub])
    by_order = [math.fsum(eps[S] for S in eps if len(S) == k) for k in range(1, order + 1)]
    total = math.fsum([e_ref] + by_order)
    return eps, by_order, total


def screened_coefficients(keep, order: int):
    """{T: c_T} with sum over kept S of eps_S = sum_T c_T E_c(T): the
    screened expansion applied to symbolic unit energies (the weight of each
    increment's density in the gradient)."""
    kept = sorted(set(keep), key=lambda s: (len(s), s))
    coef = {}
    for S in kept:
        c = {S: 1}
        for k in range(1, len(S)):
            for T in itertools.combinations(S, k):
                for U, v in coef.get(T, {}).items():
                    c[U] = c.get(U, 0) - v
        coef[S] = c
    total = {}
    for c in coef.values():
        for U, v in c.items():
            total[U] = total.get(U, 0) + v
    return total
