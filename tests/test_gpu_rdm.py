"""GPU parity of the RDM adjoint (dE/dh = gamma_w, dE/d(pq|rs) = Gamma_w / 2)
against the oracle's operator-applied densities, Hellmann-Feynman against
central finite differences of the GPU energy, and the autograd wrapper."""
import itertools

import numpy as np
import pytest

from oracle import ifci as oifci, rdm as ordm
from paper_2307_10675_amd import ifci, synthetic

pytestmark = pytest.mark.gpu


def _gpu_grad(p, **opts):
    import torch
    plan, res = ifci.solve(p, **opts)
    dh, dg = plan.rdm()
    torch.cuda.synchronize()
    return plan, res, dh.cpu().numpy(), dg.cpu().numpy()


@pytest.mark.parametrize("nb,order,seed", [(3, 2, 21), (3, 3, 22), (4, 2, 23), (4, 4, 1100)])
def test_rdm_matches_oracle(nb, order, seed):
    print(f"[rdm] chain({nb}) order {order} seed {seed}", flush=True)
    p = synthetic.chain(nb, seed=seed, order=order)
    plan, res, dh, dg = _gpu_grad(p, r_tol=1e-10, max_iter=500)
    e_o, dh_o, dg_o = ordm.ifci_gradient(p)
    assert abs(res["total"] - e_o) <= 1e-9
    assert np.abs(dh - dh_o).max() <= 1e-8
    assert np.abs(dg - dg_o).max() <= 1e-8
    # Euler: E is homogeneous of degree one in (h, eri) when e_const = 0
    e_euler = float((p.h * dh).sum() + (p.eri * dg).sum())
    assert abs(e_euler - res["total"]) <= 1e-9


def test_rdm_explicit_weights_equal_default():
    import torch
    p = synthetic.chain(4, seed=31, order=3)
    plan, res, dh, dg = _gpu_grad(p, r_tol=1e-10)
    w_k = plan.weights()
    w = np.array([w_k[len(i.bodies) - 1] for i in plan.increments()], dtype=np.float64)
    dh2, dg2 = plan.rdm(weights=w)
    torch.cuda.synchronize()
    assert np.array_equal(dh, dh2.cpu().numpy())
    assert np.array_equal(dg, dg2.cpu().numpy())


def test_rdm_single_increment_weights():
    """Weight 1 on one increment, 0 elsewhere: the gradient is that
    increment's own density embedded in the full space."""
    import torch
    p = synthetic.chain(3, seed=41, order=2)
    plan, res, _, _ = _gpu_grad(p, r_tol=1e-10)
    incs = [i.bodies for i in plan.increments()]
    S = (0, 2)
    w = np.zeros(len(incs))
    w[incs.index(S)] = 1.0
    dh, dg = plan.rdm(weights=w)
    torch.cuda.synchronize()
    d = ordm.increment_densities(p, S)
    assert np.abs(dh.cpu().numpy() - d["gamma"]).max() <= 1e-8
    assert np.abs(dg.cpu().numpy() - 0.5 * d["Gamma"]).max() <= 1e-8
    n_el = 2 * sum(p.nocc)
    assert abs(np.trace(dh.cpu().numpy()) - n_el) <= 1e-9


def test_rdm_mixed_vs_fp64():
    p = synthetic.chain(4, seed=51, order=3)
    _, _, dh64, dg64 = _gpu_grad(p, r_tol=1e-9)
    _, _, dh32, dg32 = _gpu_grad(p, precision=ifci.MIXED, r_tol=1e-6, r_tol_inner=1e-5)
    assert np.abs(dh32 - dh64).max() <= 1e-4
    assert np.abs(dg32 - dg64).max() <= 1e-4


def _orbit(p, q, r, s):
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def test_hellmann_feynman_finite_differences():
    """Central differences (step 1e-5) of the GPU energy on seeded h pairs and
    eri orbits against the GPU adjoint."""
    p = synthetic.chain(3, seed=61, order=3)
    _, res, dh, dg = _gpu_grad(p, r_tol=1e-11, max_iter=500)
    rng = np.random.default_rng(7)
    n = p.n_orb
    step = 1e-5

    def energy(h, eri):
        q = synthetic.Problem(h, eri, p.bodies, p.nocc, p.order)
        _, r = ifci.solve(q, r_tol=1e-11, max_iter=500)
        return r["total"]

    for _ in range(4):
        a, b = sorted(rng.choice(n, 2, replace=True))
        hp, hm = p.h.copy(), p.h.copy()
        for (x, y) in {(a, b), (b, a)}:
            hp[x, y] += step
            hm[x, y] -= step
        fd = (energy(hp, p.eri) - energy(hm, p.eri)) / (2 * step)
        an = sum(dh[x, y] for (x, y) in {(a, b), (b, a)})
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (a, b, fd, an)
    for _ in range(4):
        idx = tuple(int(v) for v in rng.choice(n, 4, replace=True))
        orb = _orbit(*idx)
        gp, gm = p.eri.copy(), p.eri.copy()
        for t in orb:
            gp[t] += step
            gm[t] -= step
        fd = (energy(p.h, gp) - energy(p.h, gm)) / (2 * step)
        an = sum(dg[t] for t in orb)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (idx, fd, an)


def test_autograd_function():
    import torch
    from paper_2307_10675_amd.autograd import ifci_energy
    p = synthetic.chain(3, seed=71, order=2)
    dev = torch.device("cuda", 0)
    h = torch.tensor(p.h, dtype=torch.float64, device=dev, requires_grad=True)
    eri = torch.tensor(p.eri, dtype=torch.float64, device=dev, requires_grad=True)
    e = ifci_energy(h, eri, p, r_tol=1e-10)
    e.backward()
    e_o, dh_o, dg_o = ordm.ifci_gradient(p)
    assert abs(float(e.detach()) - e_o) <= 1e-9
    assert np.abs(h.grad.cpu().numpy() - dh_o).max() <= 1e-8
    assert np.abs(eri.grad.cpu().numpy() - dg_o).max() <= 1e-8
