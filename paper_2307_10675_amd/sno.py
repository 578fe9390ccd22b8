"""iFCI with summation natural orbitals (paper, Methods, the SNO paragraph,
eq. 6) on the device: argument marshalling and the order of the steps; every
step runs in the library.

1. For each occupied orbital i, the FCI of its two electrons in {i} plus
   every virtual (the other occupied orbitals frozen) and its one-particle
   density (ifci_rdm with weight one on that increment).
2. For each increment S, the natural orbitals of rho_S = sum of its members'
   virtual blocks, those of occupation >= 10^-eta kept (ifci_sno_orbitals).
3. Each increment's integrals in its rotated basis (ifci_sno_transform) and
   its FCI; all increments in one batched solve (ifci_davidson_group).
4. The expansion's energy sums (ifci_energy of a plan whose bodies are the
   occupied orbitals).
"""
from __future__ import annotations

import ctypes
import itertools

from . import ifci


class _Record:
    """What Plan reads of a problem: orbital count, bodies, occupations, order."""

    def __init__(self, n_orb, bodies, nocc, order, e_const=0.0):
        self.n_orb, self.bodies, self.nocc, self.order, self.e_const = n_orb, bodies, nocc, order, e_const


def _increments(n_bodies, order):
    return [S for k in range(1, order + 1) for S in itertools.combinations(range(n_bodies), k)]


def solve_sno(problem, eta: float, precision=ifci.FP64, device: int = 0, **opts):
    """SNO expansion of a synthetic.SnoProblem: dict(E, n_keep, eps, total,
    e_ref, by_order, seconds_by_step)."""
    import time

    import torch
    dev = torch.device("cuda", device)
    L = ifci.lib()
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    h = torch.as_tensor(problem.h, dtype=torch.float64, device=dev).contiguous()
    eri = torch.as_tensor(problem.eri, dtype=torch.float64, device=dev).contiguous()
    occ, vir, n = list(problem.occ), list(problem.vir), problem.n_orb
    n_occ, n_vir, order = len(occ), len(vir), problem.order
    timing = {}
    t0 = time.perf_counter()
    # 1. one-body densities
    one = []
    for i in occ:
        others = [j for j in occ if j != i]
        rec = _Record(n, [[i] + vir] + [[j] for j in others], [1] * n_occ, 1, problem.e_const)
        one.append(ifci.Plan(rec, precision=precision, device=device, **opts).attach(h, eri))
    ifci.davidson_group(one)
    gamma = torch.empty((n_occ, n, n), dtype=torch.float64, device=dev)
    for t, p in enumerate(one):
        w = torch.zeros(p.n_inc, dtype=torch.float64, device=dev)
        w[0] = 1.0
        dh, _ = p.rdm(weights=w, with_eri=False)
        gamma[t].copy_(dh)
    torch.cuda.synchronize(dev)
    timing["one_body"] = time.perf_counter() - t0
    # 2. natural orbitals per increment
    t0 = time.perf_counter()
    incs = _increments(n_occ, order)
    inc_occ = torch.tensor([list(S) + [-1] * (order - len(S)) for S in incs], dtype=torch.int32, device=dev)
    vir_d = torch.tensor(vir, dtype=torch.int32, device=dev)
    rot = torch.empty((len(incs), n_vir, n_vir), dtype=torch.float64, device=dev)
    n_keep_d = torch.empty(len(incs), dtype=torch.int32, device=dev)
    ifci._check(L.ifci_sno_orbitals(ifci._ptr(gamma), n, ifci._ptr(vir_d), n_vir, ifci._ptr(inc_occ), len(incs),
                                    order, float(eta), ifci._ptr(rot), ifci._ptr(n_keep_d), sp))
    n_keep = n_keep_d.cpu().numpy()
    timing["orbitals"] = time.perf_counter() - t0
    # 3. rotated integrals and the increments' FCI
    t0 = time.perf_counter()
    # C (n x m) and two quarter-transform buffers (n^3 m each), m <= n
    work = torch.empty(n * n + 2 * n ** 4, dtype=torch.float64, device=dev)
    plans = []
    for s, S in enumerate(incs):
        S_occ = [occ[b] for b in S]
        oth = [j for j in occ if j not in S_occ]
        m = len(S_occ) + int(n_keep[s]) + len(oth)
        col = torch.tensor(S_occ + oth, dtype=torch.int32, device=dev)
        h2 = torch.empty((m, m), dtype=torch.float64, device=dev)
        e2 = torch.empty((m, m, m, m), dtype=torch.float64, device=dev)
        ifci._check(L.ifci_sno_transform(ifci._ptr(h), ifci._ptr(eri), n, ifci._ptr(vir_d), n_vir, ifci._ptr(col),
                                         len(S_occ), len(oth), ifci._ptr(rot[s]), int(n_keep[s]), ifci._ptr(work),
                                         work.numel(), ifci._ptr(h2), ifci._ptr(e2), sp))
        na = len(S_occ) + int(n_keep[s])
        rec = _Record(m, [list(range(na))] + [[na + t] for t in range(len(oth))], [len(S_occ)] + [1] * len(oth), 1,
                      problem.e_const)
        plans.append(ifci.Plan(rec, precision=precision, device=device, **opts).attach(h2, e2))
    outs = ifci.davidson_group(plans)
    E = torch.stack([o[0][0] for o in outs])
    st = torch.stack([o[1][0] for o in outs])
    torch.cuda.synchronize(dev)
    timing["increments"] = time.perf_counter() - t0
    # 4. the expansion
    asm = ifci.Plan(_Record(n, [[i] for i in occ], [1] * n_occ, order, problem.e_const), precision=precision,
                    device=device, **opts).attach(h, eri)
    en = asm.energy(E, st)
    return dict(E=E, status=st, n_keep=n_keep, increments=incs, seconds_by_step=timing, **en)
