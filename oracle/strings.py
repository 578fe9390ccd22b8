"""One-spin occupation strings (test infrastructure only).

A string is a bitmask over k spatial orbitals: bit p set means orbital p holds
an electron of this spin.  The determinant space of an increment with k active
orbitals and n electrons of each spin is the product of two copies of
strings(k, n) (Knowles-Handy determinant FCI; the paper gives only the size of
such spaces, Table 1 "FCI Determinants").

Conventions:
* strings are listed in increasing integer order of the bitmask;
* the address of a string is its position in that list;
* E_pq = a+_p a_q acting on a string gives sign * |J> with sign = (-1)^(number of
  occupied orbitals strictly between p and q), or zero.
"""
from __future__ import annotations

from math import comb


def popcount(x: int) -> int:
    return bin(x).count("1")


def strings(k: int, n: int) -> list[int]:
    """All bitmasks over k bits with n bits set, increasing."""
    return [m for m in range(1 << k) if popcount(m) == n]


def occupied(mask: int) -> list[int]:
    return [p for p in range(mask.bit_length()) if mask >> p & 1]


def address(mask: int) -> int:
    """Rank of `mask` among equal-popcount masks in increasing order.

    With the occupied orbitals o_0 < o_1 < ... this is sum_m C(o_m, m + 1)
    (the combinatorial number system; colexicographic order of subsets equals
    increasing order of their bitmasks)."""
    return sum(comb(p, m + 1) for m, p in enumerate(occupied(mask)))


def excite(mask: int, p: int, q: int):
    """Apply E_pq = a+_p a_q to one string.  Returns (sign, new_mask) or None."""
    if not mask >> q & 1:
        return None
    rest = mask & ~(1 << q)
    if rest >> p & 1:
        return None
    lo, hi = (p, q) if p < q else (q, p)
    between = popcount(rest & ((1 << hi) - 1) & ~((1 << (lo + 1)) - 1))
    return (-1 if between & 1 else 1), rest | (1 << p)


def link_table(k: int, n: int):
    """Single replacements of every string.

    Returns a list (one entry per string, in string order) of lists of tuples
    (p, q, J, sign) meaning E_pq |I> = sign |J>, with q running over the
    occupied orbitals of I in increasing order and, for each q, p running in
    increasing order over the orbitals empty in I with q removed (p = q
    included)."""
    strs = strings(k, n)
    out = []
    for s in strs:
        row = []
        for q in occupied(s):
            for p in range(k):
                r = excite(s, p, q)
                if r is not None:
                    row.append((p, q, address(r[1]), r[0]))
        out.append(row)
    return out
