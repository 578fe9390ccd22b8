"""Seeded synthetic iFCI problems: integrals, bodies and reference occupations.

This module only draws random numbers and arranges them; it contains none of
the method's arithmetic (no Hamiltonian, no energies).  Both the CPU oracle
tests and the device path take their inputs from here, so neither side ever
feeds the other.

Recipe (the paper's molecular integrals of PFAS in cc-pVDZ are not available;
these stand in for them with the same structure: a localized basis split into
"bodies", each body a GVB-pair-like group of one occupied and one virtual
orbital, couplings that decay with distance between bodies):

* one-electron h: symmetric; diagonal drawn uniform in [-1.5, 0.5] Eh, upper
  off-diagonal (row-major) drawn N(0, 0.05) and mirrored;
* two-electron (pq|rs) = sum_k L^k_pq L^k_rs with K symmetric factors L^k whose
  upper triangles (diagonal included, row-major) are drawn N(0, 0.15); this
  keeps the 8-fold permutational symmetry and makes the n^2 x n^2 matrix PSD;
* optional body-local decay d_pq = exp(-0.5 |b(p) - b(q)|) with b(p) the body
  of orbital p, applied to the off-diagonal of h and to every L^k_pq;
* the reference-occupied orbitals of a body are its lowest-h_pp orbitals
  (ties broken by lower index) and are listed first in the body.

Random draws happen in this order: h diagonal, h upper triangle, then
L^1 .. L^K upper triangles; the generator is numpy's PCG64 (default_rng).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """An iFCI problem as the paper states it: integrals in a localized
    orbital basis, a partition of the orbitals into bodies with their
    reference occupations, and the truncation order n of the expansion."""

    h: np.ndarray                 # (n, n) float64, symmetric
    eri: np.ndarray               # (n, n, n, n) float64, chemist order (pq|rs)
    bodies: list                  # list of lists of orbital indices; occupied first
    nocc: list                    # doubly occupied orbitals per body
    order: int                    # truncation order n
    e_const: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n_orb(self) -> int:
        return self.h.shape[0]

    @property
    def n_bodies(self) -> int:
        return len(self.bodies)

    def sha256(self) -> str:
        m = hashlib.sha256()
        m.update(np.ascontiguousarray(self.h).tobytes())
        m.update(np.ascontiguousarray(self.eri).tobytes())
        m.update(repr((self.bodies, self.nocc, self.order, self.e_const)).encode())
        return m.hexdigest()


def _sym_upper(rng, n, scale, include_diag):
    """Symmetric n x n matrix from an upper triangle drawn row-major."""
    a = np.zeros((n, n))
    for p in range(n):
        for q in range(p if include_diag else p + 1, n):
            a[p, q] = rng.normal(0.0, scale)
    return a + np.triu(a, 1).T


def integrals(n_orb: int, n_chol: int, seed: int, body_of=None, decay: bool = False, rate: float = 0.5):
    """Draw (h, eri) as described in the module docstring.

    body_of: array of body labels per orbital (used only for the decay);
    rate: the decay factor is exp(-rate |body distance|)."""
    rng = np.random.default_rng(seed)
    diag = rng.uniform(-1.5, 0.5, size=n_orb)
    off = _sym_upper(rng, n_orb, 0.05, include_diag=False)
    h = off.copy()
    h[np.diag_indices(n_orb)] = diag
    L = np.stack([_sym_upper(rng, n_orb, 0.15, include_diag=True) for _ in range(n_chol)])
    if decay:
        b = np.asarray(body_of)
        d = np.exp(-rate * np.abs(b[:, None] - b[None, :]))
        h = h * np.where(np.eye(n_orb, dtype=bool), 1.0, d)
        L = L * d[None]
    eri = np.einsum("kpq,krs->pqrs", L, L)
    return h, eri


def _order_body(h, orbs, nocc):
    """Occupied (lowest h_pp, ties by index) orbitals first, then the rest."""
    ranked = sorted(orbs, key=lambda p: (h[p, p], p))
    occ = sorted(ranked[:nocc])
    vir = sorted(ranked[nocc:])
    return occ + vir


def chain(n_bodies: int, orbs_per_body: int = 2, nocc_per_body: int = 1, n_chol: int = 12,
          seed: int = 0, order: int = 1, decay: bool = True, rate: float = 0.5) -> Problem:
    """A 1-D chain of equal bodies {b*m, ..., b*m + m - 1}; with decay the
    couplings between bodies fall off as exp(-rate |body distance|)."""
    n_orb = n_bodies * orbs_per_body
    body_of = np.arange(n_orb) // orbs_per_body
    h, eri = integrals(n_orb, n_chol, seed, body_of=body_of, decay=decay, rate=rate)
    bodies = [_order_body(h, list(range(b * orbs_per_body, (b + 1) * orbs_per_body)), nocc_per_body)
              for b in range(n_bodies)]
    meta = dict(kind="chain", n_bodies=n_bodies, orbs_per_body=orbs_per_body, n_chol=n_chol, seed=seed,
                decay=decay)
    if rate != 0.5:
        meta["rate"] = rate
    return Problem(h, eri, bodies, [nocc_per_body] * n_bodies, order, meta=meta)


def single(n_orb: int, n_chol: int, seed: int) -> Problem:
    """One body holding every orbital, half filled: a plain FCI problem."""
    h, eri = integrals(n_orb, n_chol, seed)
    nocc = n_orb // 2
    return Problem(h, eri, [_order_body(h, list(range(n_orb)), nocc)], [nocc], 1,
                   meta=dict(kind="single", n_orb=n_orb, n_chol=n_chol, seed=seed))


def separable(n_bodies: int, n_chol: int = 12, seed: int = 0, order: int = 2) -> Problem:
    """Chain of 2-orbital bodies that do not interact at all: h is block
    diagonal and every (pq|rs) with p, q, r, s not all in one body is zero
    (each body gets its own Cholesky-like factors).  Occupied-orbital
    energies are drawn in [-1.1, -0.9] Eh and virtual ones in [0.3, 0.5] Eh,
    so each body's closed-shell singlet lies far below its triplet and below
    any charge-transfer configuration."""
    n_orb = 2 * n_bodies
    rng = np.random.default_rng(seed)
    h = np.zeros((n_orb, n_orb))
    eri = np.zeros((n_orb,) * 4)
    for b in range(n_bodies):
        o, v = 2 * b, 2 * b + 1
        h[o, o] = rng.uniform(-1.1, -0.9)
        h[v, v] = rng.uniform(0.3, 0.5)
        h[o, v] = h[v, o] = rng.normal(0.0, 0.05)
        L = np.stack([_sym_upper(rng, 2, 0.15, include_diag=True) for _ in range(n_chol)])
        blk = np.einsum("kpq,krs->pqrs", L, L)
        eri[o:v + 1, o:v + 1, o:v + 1, o:v + 1] = blk
    bodies = [[2 * b, 2 * b + 1] for b in range(n_bodies)]
    return Problem(h, eri, bodies, [1] * n_bodies, order,
                   meta=dict(kind="separable", n_bodies=n_bodies, n_chol=n_chol, seed=seed))


def local_chain(n_bodies: int, seed: int = 0, order: int = 1, rate: float = 1.0, coupling: float = 0.3,
                n_chol: int = 4) -> Problem:
    """Chain of 2-orbital bodies whose every interaction falls off with the
    distance along the chain, also the integrals (ia|jb) that correlate two
    bodies (in the chain above they do not decay).  Each body is drawn as
    in `separable`; on top, every body centre c carries n_chol shared factors
    M[p][q] = coupling * g_pq * exp(-rate (|b(p) - c| + |b(q) - c|)), g
    symmetric N(0, 0.15), added to the eri as sum M (x) M (so it stays
    8-fold symmetric and positive semidefinite), and h couples bodies I, J by
    N(0, 0.05) * exp(-rate |I - J|)."""
    p = separable(n_bodies, seed=seed, order=order)
    n_orb = 2 * n_bodies
    rng = np.random.default_rng(seed + 7919)
    b = np.arange(n_orb) // 2
    h = p.h.copy()
    off = _sym_upper(rng, n_orb, 0.05, include_diag=False)
    dist = np.abs(b[:, None] - b[None, :])
    h = h + np.where(dist > 0, off * np.exp(-rate * dist), 0.0)
    eri = p.eri.copy()
    for c in range(n_bodies):
        f = np.exp(-rate * np.abs(b - c))
        for _ in range(n_chol):
            M = coupling * _sym_upper(rng, n_orb, 0.15, include_diag=True) * f[:, None] * f[None, :]
            eri += np.einsum("pq,rs->pqrs", M, M)
    bodies = [_order_body(h, [2 * i, 2 * i + 1], 1) for i in range(n_bodies)]
    return Problem(h, eri, bodies, [1] * n_bodies, order,
                   meta=dict(kind="local_chain", n_bodies=n_bodies, seed=seed, rate=rate, coupling=coupling,
                             n_chol=n_chol))


class SnoProblem:
    """Occupied orbitals (each a body, doubly occupied in the reference) and
    virtual orbitals shared by every body, over one set of integrals."""

    def __init__(self, h, eri, occ, vir, order, e_const=0.0, meta=None):
        self.h, self.eri = h, eri
        self.occ, self.vir = list(occ), list(vir)
        self.order = order
        self.e_const = e_const
        self.n_orb = h.shape[0]
        self.meta = meta or {}

    def sha256(self) -> str:
        m = hashlib.sha256()
        m.update(np.ascontiguousarray(self.h).tobytes())
        m.update(np.ascontiguousarray(self.eri).tobytes())
        m.update(repr((self.occ, self.vir, self.order, self.e_const)).encode())
        return m.hexdigest()


def merged(p: Problem) -> Problem:
    """The same integrals with every orbital in one body (the whole system as
    a single increment): the bodies' occupied orbitals first, in body order,
    then their virtual orbitals."""
    occ = [o for b, orbs in enumerate(p.bodies) for o in orbs[: p.nocc[b]]]
    vir = [o for b, orbs in enumerate(p.bodies) for o in orbs[p.nocc[b]:]]
    return Problem(p.h, p.eri, [occ + vir], [len(occ)], 1, p.e_const, meta=dict(p.meta, merged=True))


def sno_system(n_occ: int, n_vir: int, seed: int, order: int = 2, n_chol: int = 12) -> SnoProblem:
    """Integrals as in the module docstring (no decay) over n_occ + n_vir
    orbitals; the n_occ orbitals of lowest h_pp (ties by index) are
    occupied, the others virtual."""
    n = n_occ + n_vir
    h, eri = integrals(n, n_chol, seed)
    ranked = sorted(range(n), key=lambda p: (h[p, p], p))
    occ, vir = sorted(ranked[:n_occ]), sorted(ranked[n_occ:])
    return SnoProblem(h, eri, occ, vir, order, meta=dict(kind="sno", n_occ=n_occ, n_vir=n_vir, seed=seed,
                                                         n_chol=n_chol))


def random_vector(n: int, seed: int, symmetric_dim: int | None = None) -> np.ndarray:
    """Seeded N(0,1) vector; with symmetric_dim = m it is reshaped to m x m
    and symmetrised (C = C^T), then flattened row-major."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=n)
    if symmetric_dim is not None:
        m = symmetric_dim
        c = v.reshape(m, m)
        v = (0.5 * (c + c.T)).reshape(-1)
    return v


# ---------------------------------------------------------------- workloads
def workload(cfg: int, replicate: int = 0) -> Problem:
    """The five synthetic workloads (seed = 1000 * cfg + replicate).

    0: 6 orbitals / 6 electrons, K = 12, one body, order 1.
    1: 10 bodies of 2 orbitals / 2 electrons (20 orbitals), K = 12, decay, order 3.
    2: 16 bodies (32 orbitals), K = 12, decay, order 4.
    3: 12 bodies (24 orbitals), K = 12, decay, order 5.
    4: one body of 14 orbitals / 14 electrons, K = 28.
    """
    seed = 1000 * cfg + replicate
    if cfg == 0:
        return single(6, 12, seed)
    if cfg == 1:
        return chain(10, seed=seed, order=3)
    if cfg == 2:
        return chain(16, seed=seed, order=4)
    if cfg == 3:
        return chain(12, seed=seed, order=5)
    if cfg == 4:
        return single(14, 28, seed)
    raise ValueError(f"unknown workload {cfg}")
