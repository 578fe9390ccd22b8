"""Increments beyond dense-oracle size (10, 12 and 14 active orbitals), on the
device-wide path, checked row by row: the oracle builds single rows of H c
from the Slater-Condon rules (no determinant list), so sigma and the
residual of the converged vector are compared on seeded row samples at the
full size.  Also the six-body full-order expansion (up to 12o12e)."""
import numpy as np
import pytest

from oracle import certify, ifci as oifci
from paper_2307_10675_amd import ifci, synthetic

pytestmark = pytest.mark.gpu

# (orbitals, Cholesky factors, seed): 63,504 / 853,776 / 11,778,624 determinants
SIZES = [(10, 20, 4010), (12, 24, 4012), (14, 28, 4000)]


def _rows(n_det, seed, count=40):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_det, count, replace=False))


@pytest.mark.parametrize("n,K,seed", SIZES)
def test_plain_sigma_sampled_rows(n, K, seed):
    import torch
    print(f"[large] sigma {n}o{n}e", flush=True)
    p = synthetic.single(n, K, seed)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    nd = plan.increment(0).n_det
    c = synthetic.random_vector(nd, seed + 1)
    got = plan.sigma(0, torch.tensor(c, device="cuda")).cpu().numpy()
    rows = _rows(nd, seed + 2)
    want = certify.sigma_rows_strings(rows, n // 2, c, p.h, p.eri)
    scale = np.abs(want).max()
    assert np.abs(got[rows] - want).max() <= 1e-12 * max(1.0, scale) * n
    # FP32 contraction on the same vector
    got32 = plan.sigma(0, torch.tensor(c, device="cuda"), precision=ifci.MIXED).cpu().numpy()
    assert np.abs(got32[rows] - want).max() <= 2e-5 * max(1.0, scale)


@pytest.mark.parametrize("n,K,seed", SIZES)
def test_large_solve_residual_rows(n, K, seed):
    """FP64 solve to ||r|| <= 1e-8: sampled rows of H c - E c from the oracle
    stay within that bound; E is below the reference energy; mixed precision
    agrees with FP64 to 1 uEh."""
    import torch
    print(f"[large] solve {n}o{n}e", flush=True)
    p = synthetic.single(n, K, seed)
    plan, res = ifci.solve(p, r_tol=1e-8, max_iter=400)
    torch.cuda.synchronize()
    assert int(res["status"][0]) == ifci.INC_DONE
    E = float(res["E"][0])
    assert E < oifci.reference_energy(p)
    c = plan.vector(0).cpu().numpy()
    assert abs(np.linalg.norm(c) - 1.0) < 1e-10
    nd = len(c)
    rows = _rows(nd, seed + 3)
    r = certify.sigma_rows_strings(rows, n // 2, c, p.h, p.eri) - E * c[rows]
    assert np.abs(r).max() <= 2e-8
    _, res32 = ifci.solve(p, precision=ifci.MIXED, r_tol=3e-5, r_tol_inner=1e-5, max_iter=400)
    assert int(res32["status"][0]) == ifci.INC_DONE
    assert abs(float(res32["E"][0]) - E) <= 1e-6


def test_full_order_six_bodies():
    """Six bodies to full order (63 increments up to 12o12e, batched and
    device-wide paths together): the expansion total equals the FCI energy of
    the whole system, whose residual is checked on oracle rows."""
    import torch
    print("[large] six-body full order", flush=True)
    p = synthetic.chain(6, seed=1101, order=6)
    plan, res = ifci.solve(p, r_tol=1e-9, max_iter=400)
    torch.cuda.synchronize()
    assert (res["status"].cpu().numpy() == ifci.INC_DONE).all()
    E = res["E"].cpu().numpy()
    assert len(E) == 63
    assert abs(res["total"] - float(E[-1])) <= 1e-9
    last = plan.increments()[-1]
    assert last.bodies == tuple(range(6)) and last.n_act == 12
    c = plan.vector(62).cpu().numpy()
    rows = _rows(len(c), 7)
    r = certify.sigma_rows_strings(rows, 6, c, p.h, p.eri) - float(E[-1]) * c[rows]
    assert np.abs(r).max() <= 2e-9


def test_rdm_ten_orbital_increment():
    """Density matrices of a 10o10e increment (device-wide path): traces,
    the Euler identity E = sum h gamma + sum (pq|rs) Gamma / 2, the pair
    symmetries of Gamma, and central finite differences of the GPU energy
    for two h entries."""
    import torch
    print("[large] rdm 10o10e", flush=True)
    p = synthetic.single(10, 20, 4110)
    plan, res = ifci.solve(p, r_tol=1e-10, max_iter=400)
    dh, dg = plan.rdm()
    torch.cuda.synchronize()
    g1 = dh.cpu().numpy()
    g2 = 2.0 * dg.cpu().numpy()
    n_el = 10
    assert abs(np.trace(g1) - n_el) < 1e-9
    assert abs(np.einsum("pprr->", g2) - n_el * (n_el - 1)) < 1e-8
    assert np.abs(g1 - g1.T).max() < 1e-10
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() < 1e-10
    assert np.abs(g2 - g2.transpose(1, 0, 3, 2)).max() < 1e-10
    E = float(res["E"][0])
    assert abs((p.h * g1).sum() + 0.5 * (p.eri * g2).sum() - E) < 1e-9
    w = np.linalg.eigvalsh(g1)
    assert w.min() > -1e-10 and w.max() < 2 + 1e-10
    step = 1e-5
    for (a, b) in ((0, 0), (2, 7)):
        hp, hm = p.h.copy(), p.h.copy()
        for (x, y) in {(a, b), (b, a)}:
            hp[x, y] += step
            hm[x, y] -= step
        ep = ifci.solve(synthetic.Problem(hp, p.eri, p.bodies, p.nocc, p.order), r_tol=1e-10, max_iter=400)[1]["total"]
        em = ifci.solve(synthetic.Problem(hm, p.eri, p.bodies, p.nocc, p.order), r_tol=1e-10, max_iter=400)[1]["total"]
        fd = (ep - em) / (2 * step)
        an = sum(g1[x, y] for (x, y) in {(a, b), (b, a)})
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (a, b, fd, an)


def test_full_order_six_bodies_three_vector_option():
    """max_space = 3 selects the three-vector iteration on chip; the 10o and
    12o increments of the six-body expansion then run the device-wide
    Davidson with its default subspace (their blocks are laid out for it).
    Every increment converges, the total equals the default run's, and the
    12o12e vector read back through the block layout has small residual
    rows."""
    import torch
    print("[large] six-body full order, max_space 3", flush=True)
    p = synthetic.chain(6, seed=1101, order=6)
    plan, res = ifci.solve(p, r_tol=1e-9, max_iter=400, max_space=3)
    torch.cuda.synchronize()
    assert (res["status"].cpu().numpy() == ifci.INC_DONE).all()
    _, ref = ifci.solve(p, r_tol=1e-9, max_iter=400)
    assert abs(res["total"] - ref["total"]) <= 1e-9
    E = res["E"].cpu().numpy()
    c = plan.vector(62).cpu().numpy()
    rows = _rows(len(c), 11)
    r = certify.sigma_rows_strings(rows, 6, c, p.h, p.eri) - float(E[-1]) * c[rows]
    assert np.abs(r).max() <= 2e-9


def test_solve_sixteen_orbitals():
    """16o16e FCI (165,636,900 determinants) on the device-wide path (split
    column sigma), in mixed precision and in FP64: both converged, below the
    reference energy, within 1e-6 of each other, and the oracle's
    Slater-Condon rows of H c - E c on 16 sampled determinants within the
    residual-norm bound for each."""
    import torch
    p = synthetic.single(16, 32, 4016)
    E = {}
    for name, prec in (("mixed", ifci.MIXED), ("fp64", ifci.FP64)):
        print(f"[large] solve 16o16e {name}", flush=True)
        plan, res = ifci.solve(p, precision=prec, r_tol=1e-5, r_tol_inner=1e-5, max_iter=400)
        torch.cuda.synchronize()
        assert int(res["status"][0]) == ifci.INC_DONE
        E[name] = float(res["E"][0])
        assert E[name] < oifci.reference_energy(p)
        c = plan.vector(0).cpu().numpy()
        assert abs(np.linalg.norm(c) - 1.0) < 1e-9
        rows = _rows(len(c), 16016, count=16)
        r = certify.sigma_rows_strings(rows, 8, c, p.h, p.eri) - E[name] * c[rows]
        assert np.abs(r).max() <= 1e-5
        plan.close()
        del plan, res, c
        torch.cuda.empty_cache()
    assert abs(E["mixed"] - E["fp64"]) <= 1e-6
