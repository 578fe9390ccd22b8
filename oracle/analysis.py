"""Grouped contributions of the incremental expansion (test infrastructure
only).

Paper, Results (the PFAS bond-breaking simulation, Fig. 4): the localized
orbitals are grouped by chemical character; the increment of a set of
orbitals then belongs to the combination of their groups (for instance a
two-body increment of one fluorine lone pair and one C-F sigma bond is an
lp_F / sigma_CF term), the contribution of a combination is the sum of the
increments eps_S that belong to it, and comparing two calculations with
comparable orbitals (two geometries) gives per combination the sum of the
changes of eps_S.

A combination is written as the sorted tuple of the group labels of the
increment's bodies (a multiset: two bodies of one group appear twice).
"""
from __future__ import annotations

import math


def combination(S, group_of_body):
    return tuple(sorted(group_of_body[b] for b in S))


def group_sums(eps: dict, group_of_body):
    """{combination: sum of eps_S over its increments}, with math.fsum."""
    terms = {}
    for S, e in eps.items():
        terms.setdefault(combination(S, group_of_body), []).append(e)
    return {c: math.fsum(v) for c, v in terms.items()}


def group_differences(eps_a: dict, eps_b: dict, group_of_body):
    """{combination: sum of (eps_S in b - eps_S in a)} over the increments
    both calculations share, with math.fsum."""
    terms = {}
    for S in eps_a:
        if S in eps_b:
            terms.setdefault(combination(S, group_of_body), []).extend([eps_b[S], -eps_a[S]])
    return {c: math.fsum(v) for c, v in terms.items()}
