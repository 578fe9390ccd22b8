"""Matrix-free checks for spaces too large to diagonalise densely
(test infrastructure only).

* sigma_rows: rows of H c computed one at a time from the Slater-Condon rules
  (every connected determinant of row I is generated explicitly);
* residual_bound: for a normalised c and E = c.Hc, some eigenvalue lies within
  ||Hc - E c|| of E (Bauer-Fike for symmetric matrices); if the next root of
  the sector is at least `gap` away, |E - lambda| <= ||r||^2 / gap
  (Kato-Temple).
"""
from __future__ import annotations

import math

import numpy as np

from . import hamiltonian, strings


def sigma_rows(rows, dets, c, h, eri, active, e_const: float = 0.0):
    """[(H c)_I for I in rows] with H over the determinant list `dets`."""
    ints = hamiltonian.SpinOrbitalIntegrals(h, eri)
    index = {d: i for i, d in enumerate(dets)}
    out = []
    for I in rows:
        d = dets[I]
        acc = [(hamiltonian.diagonal(ints, d) + e_const) * c[I]]
        for J, v in hamiltonian.connected(ints, d, active):
            acc.append(v * c[index[J]])
        out.append(float(np.sum(acc)))
    return np.array(out)


def sigma_rows_strings(rows, n_el: int, c, h, eri, e_const: float = 0.0):
    """(H c)_I for I in rows over every determinant of the len(h) orbitals of
    h with n_el electrons of each spin and no core.  Determinant I is
    address(alpha) * N_str + address(beta) (strings in increasing bitmask
    order), so no list of all determinants is formed: each row is built from
    the Slater-Condon rules over its connected determinants."""
    ints = hamiltonian.SpinOrbitalIntegrals(h, eri)
    n = ints.n
    S = strings.strings(n, n_el)
    ns = len(S)
    mask = (1 << n) - 1
    active = list(range(n))
    out = []
    for I in rows:
        a, b = divmod(int(I), ns)
        det = S[a] | (S[b] << n)
        acc = [(hamiltonian.diagonal(ints, det) + e_const) * c[I]]
        for J, v in hamiltonian.connected(ints, det, active):
            acc.append(v * c[strings.address(J & mask) * ns + strings.address(J >> n)])
        out.append(math.fsum(acc))
    return np.array(out)


def residual_bound(r_norm: float, gap: float | None = None) -> float:
    if gap is None:
        return r_norm
    return min(r_norm, r_norm * r_norm / gap)
