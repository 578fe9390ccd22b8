"""Hamiltonian matrix elements between determinants (test infrastructure only).

Determinants are integers over 2n spin-orbital bits: bit P < n is spatial
orbital P with spin alpha, bit n + p is orbital p with spin beta.  The
determinant is (prod over set alpha bits, ascending, of a+) times (prod over
set beta bits, ascending, of a+) acting on the vacuum, so alpha operators come
first.  The Hamiltonian is the non-relativistic electronic Hamiltonian in a
real orthonormal orbital basis,

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps) + e_const,

with E_pq = sum_spin a+_p a_q (spin-summed) and (pq|rs) in chemists' order.

Two independent constructions are provided:

* `build` uses the Slater-Condon rules in spin-orbital form with
  antisymmetrised integrals <PQ||RS> = <PQ|RS> - <PQ|SR>, <PQ|RS> = (pr|qs)
  when the spins of P,R and of Q,S match;
* `build_by_operators` applies the second-quantised operator above to every
  basis determinant (used on small spaces to check `build`).
"""
from __future__ import annotations

import numpy as np


def _sign_below(det: int, P: int) -> int:
    return -1 if bin(det & ((1 << P) - 1)).count("1") & 1 else 1


def annihilate(det: int, P: int):
    if not det >> P & 1:
        return None
    return _sign_below(det, P), det & ~(1 << P)


def create(det: int, P: int):
    if det >> P & 1:
        return None
    return _sign_below(det, P), det | (1 << P)


def apply_string(det: int, ops):
    """Apply operators right-to-left; ops is a list of ('+', P) / ('-', P)
    written left-to-right as in the operator product.  Returns (sign, det) or None."""
    sign = 1
    for kind, P in reversed(ops):
        r = create(det, P) if kind == "+" else annihilate(det, P)
        if r is None:
            return None
        sign *= r[0]
        det = r[1]
    return sign, det


class SpinOrbitalIntegrals:
    """h and (pq|rs) viewed through spin orbitals 0..2n-1."""

    def __init__(self, h, eri):
        self.h = np.asarray(h, dtype=np.float64)
        self.eri = np.asarray(eri, dtype=np.float64)
        self.n = self.h.shape[0]

    def sp(self, P):
        return P % self.n, P // self.n      # spatial index, spin (0 alpha, 1 beta)

    def one(self, P, Q):
        p, sp = self.sp(P)
        q, sq = self.sp(Q)
        return self.h[p, q] if sp == sq else 0.0

    def two(self, P, Q, R, S):
        """Physicists' <PQ|RS> = (pr|qs) delta(spin P, spin R) delta(spin Q, spin S)."""
        p, sp = self.sp(P)
        q, sq = self.sp(Q)
        r, sr = self.sp(R)
        s, ss = self.sp(S)
        if sp != sr or sq != ss:
            return 0.0
        return self.eri[p, r, q, s]

    def anti(self, P, Q, R, S):
        return self.two(P, Q, R, S) - self.two(P, Q, S, R)


def occupied_spin_orbitals(det: int, n: int):
    return [P for P in range(2 * n) if det >> P & 1]


def diagonal(ints: SpinOrbitalIntegrals, det: int) -> float:
    """<I|H|I> = sum_P h_PP + 1/2 sum_PQ <PQ||PQ> over occupied spin orbitals."""
    n = ints.n
    occ = occupied_spin_orbitals(det, n)
    sp = np.array([P % n for P in occ])
    spin = np.array([P // n for P in occ])
    e1 = ints.h[sp, sp].sum()
    coul = ints.eri[sp[:, None], sp[:, None], sp[None, :], sp[None, :]]        # (pp|qq)
    exch = ints.eri[sp[:, None], sp[None, :], sp[None, :], sp[:, None]]        # (pq|qp)
    same = spin[:, None] == spin[None, :]
    return float(e1 + 0.5 * (coul.sum() - (exch * same).sum()))


def single(ints: SpinOrbitalIntegrals, det: int, P: int, A: int):
    """Element <J|H|I> for J = a+_A a_P I (same spin).  Returns (J, value)."""
    r = apply_string(det, [("+", A), ("-", P)])
    if r is None:
        return None
    sign, J = r
    n = ints.n
    occ = occupied_spin_orbitals(det, n)
    val = ints.one(A, P) + sum(ints.anti(A, Q, P, Q) for Q in occ)
    return J, sign * val


def double(ints: SpinOrbitalIntegrals, det: int, P: int, Q: int, A: int, B: int):
    """Element <J|H|I> for J = a+_A a+_B a_Q a_P I.  Returns (J, value)."""
    r = apply_string(det, [("+", A), ("+", B), ("-", Q), ("-", P)])
    if r is None:
        return None
    sign, J = r
    return J, sign * ints.anti(A, B, P, Q)


def connected(ints: SpinOrbitalIntegrals, det: int, active: list[int]):
    """All (J, <J|H|I>) for J != I reachable by single and double
    replacements among the spin orbitals of `active` spatial orbitals
    (spin conserved).  Each J is produced once."""
    n = ints.n
    act = [p for p in active] + [p + n for p in active]
    occ = [P for P in act if det >> P & 1]
    vir = [P for P in act if not det >> P & 1]
    out = []
    for P in occ:
        for A in vir:
            if P // n == A // n:
                r = single(ints, det, P, A)
                if r is not None and r[1] != 0.0:
                    out.append(r)
    for i, P in enumerate(occ):
        for Q in occ[i + 1:]:
            for j, A in enumerate(vir):
                for B in vir[j + 1:]:
                    if sorted((P // n, Q // n)) != sorted((A // n, B // n)):
                        continue
                    r = double(ints, det, P, Q, A, B)
                    if r is not None and r[1] != 0.0:
                        out.append(r)
    return out


def build(dets, h, eri, active, e_const: float = 0.0) -> np.ndarray:
    """Dense H over the list `dets` by the Slater-Condon rules.  Every
    replacement among `active` orbitals must map the list into itself."""
    ints = SpinOrbitalIntegrals(h, eri)
    index = {d: i for i, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for i, d in enumerate(dets):
        H[i, i] = diagonal(ints, d) + e_const
        for J, v in connected(ints, d, active):
            H[index[J], i] = v
    return H


# --------------------------------------------------------------- operator algebra
def _E(det: int, p: int, q: int, n: int):
    """Spin-summed E_pq on a determinant: list of (sign, det')."""
    out = []
    for s in (0, 1):
        r = apply_string(det, [("+", p + s * n), ("-", q + s * n)])
        if r is not None:
            out.append(r)
    return out


def build_by_operators(dets, h, eri, e_const: float = 0.0) -> np.ndarray:
    """Dense H over `dets` from H = sum h_pq E_pq + 1/2 sum (pq|rs)(E_pq E_rs -
    delta_qr E_ps) applied to each determinant.  Cost O(n^4) per determinant;
    meant for small n."""
    h = np.asarray(h)
    eri = np.asarray(eri)
    n = h.shape[0]
    index = {d: i for i, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for i, d in enumerate(dets):
        col = {}
        for p in range(n):
            for q in range(n):
                for s1, d1 in _E(d, p, q, n):
                    col[d1] = col.get(d1, 0.0) + h[p, q] * s1
                    # -1/2 sum_r (pr|rq) E_pq : the delta_qr term regrouped
                    col[d1] = col.get(d1, 0.0) - 0.5 * s1 * sum(eri[p, r, r, q] for r in range(n))
        for r in range(n):
            for s in range(n):
                first = _E(d, r, s, n)
                if not first:
                    continue
                for p in range(n):
                    for q in range(n):
                        g = eri[p, q, r, s]
                        if g == 0.0:
                            continue
                        for s1, d1 in first:
                            for s2, d2 in _E(d1, p, q, n):
                                col[d2] = col.get(d2, 0.0) + 0.5 * g * s1 * s2
        for d2, v in col.items():
            if d2 in index:
                H[index[d2], i] += v
        H[i, i] += e_const
    return H
