"""Differentiation at the size of the 12-body workload (12 bodies of 2
orbitals / 2 electrons, 24 orbitals, decay): the expansion gradient
dE/dh = gamma_w and dE/d(pq|rs) = Gamma_w / 2 (Hellmann-Feynman, weighted
as eqs. 1-5 weight each increment energy).

Order 4 (793 increments up to 8o8e): every increment energy, eps_S, the
total and the gradient against the oracle's operator-applied densities
(tests/golden/oracle_w3o4.json, written by make_oracle_refs.py from
oracle/ only); mixed precision (FP64 residual 1e-7) against FP64; central finite differences of
the GPU energy on 16 seeded h pairs and 16 seeded eri orbits.

Order 5 (1585 increments, adding 792 x 10o10e on the device-wide solver):
no dense oracle gradient at this size, so the checks are what holds at any
size -- the trace identities, Euler's identity for a function homogeneous
of degree one in (h, eri), mixed against FP64 -- and central finite
differences on seeded h pairs and eri orbits."""
import numpy as np
import pytest

from paper_2307_10675_amd import ifci, synthetic
from tests.helpers import load_golden

pytestmark = pytest.mark.gpu

STEP = 1e-5


def _orbit(p, q, r, s):
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def _solve_grad(p, h, eri, **opts):
    import torch
    plan = ifci.Plan(p, **opts).attach(h, eri)
    e, st, it, rs = plan.davidson()
    en = plan.energy(e, st)
    dh, dg = plan.rdm()
    torch.cuda.synchronize()
    out = dict(E=e.cpu().numpy(), status=st.cpu().numpy(), dh=dh.cpu().numpy(), dg=dg.cpu().numpy(), **en)
    plan.close()
    return out


def _device(p):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.tensor(p.h, dtype=torch.float64, device=dev),
            torch.tensor(p.eri, dtype=torch.float64, device=dev).contiguous())


def _invariants(p, r, tol):
    n_el = 2 * sum(p.nocc)
    assert abs(np.trace(r["dh"]) - n_el) <= tol * n_el
    n = p.n_orb
    g2 = sum(r["dg"][a, a, b, b] for a in range(n) for b in range(n))
    assert abs(g2 - 0.5 * n_el * (n_el - 1)) <= tol * n_el * n_el
    e_euler = float((p.h * r["dh"]).sum() + (p.eri * r["dg"]).sum())
    assert abs(e_euler - r["total"]) <= tol * max(1.0, abs(r["total"]))


def _finite_differences(p, r, n_h, n_eri, seed, opts, tol, richardson=False):
    rng = np.random.default_rng(seed)
    n = p.n_orb

    def energy(h, eri):
        q = synthetic.Problem(h, eri, p.bodies, p.nocc, p.order)
        _, res = ifci.solve(q, **opts)
        assert (res["status"].cpu().numpy() == ifci.INC_DONE).all()
        return res["total"]

    def central(f, step):
        return (f(step) - f(-step)) / (2 * step)

    def derivative(f):
        # central differences at steps d and 2d, Richardson-extrapolated:
        # the step^2 term (large where an increment is nearly degenerate)
        # cancels, leaving step^4
        return (4 * central(f, STEP) - central(f, 2 * STEP)) / 3 if richardson else central(f, STEP)

    for _ in range(n_h):
        a, b = sorted(int(v) for v in rng.choice(n, 2, replace=True))

        def f_h(d):
            hd = p.h.copy()
            for (x, y) in {(a, b), (b, a)}:
                hd[x, y] += d
            return energy(hd, p.eri)

        fd = derivative(f_h)
        an = sum(r["dh"][x, y] for (x, y) in {(a, b), (b, a)})
        assert abs(fd - an) <= tol * max(1.0, abs(an)), ("h", a, b, fd, an)
    for _ in range(n_eri):
        idx = tuple(int(v) for v in rng.choice(n, 4, replace=True))
        orb = _orbit(*idx)

        def f_g(d):
            gd = p.eri.copy()
            for t in orb:
                gd[t] += d
            return energy(p.h, gd)

        fd = derivative(f_g)
        an = sum(r["dg"][t] for t in orb)
        assert abs(fd - an) <= tol * max(1.0, abs(an)), ("eri", idx, fd, an)


@pytest.fixture(scope="module")
def order4():
    p = synthetic.chain(12, seed=3000, order=4)
    g = load_golden("w3o4")
    assert p.sha256() == g["sha256"], "synthetic generator changed; regenerate tests/golden"
    h, eri = _device(p)
    print("[w3] order 4 fp64", flush=True)
    r64 = _solve_grad(p, h, eri, r_tol=1e-10, max_iter=600)
    print("[w3] order 4 mixed", flush=True)
    r32 = _solve_grad(p, h, eri, precision=ifci.MIXED, r_tol=1e-7, r_tol_inner=1e-5, max_iter=600)
    return p, g, r64, r32


def test_order4_energies_against_oracle(order4):
    p, g, r64, r32 = order4
    assert (r64["status"] == ifci.INC_DONE).all() and (r32["status"] == ifci.INC_DONE).all()
    ref = np.array([x["E"] for x in g["increments"]])
    assert len(ref) == 793 and len(r64["E"]) == 793
    assert np.abs(r64["E"] - ref).max() <= 1e-9
    assert np.abs(r32["E"] - ref).max() <= 1e-6
    sizes = np.array([len(x["bodies"]) for x in g["increments"]])
    eps = np.array(r64["eps"].cpu().numpy())
    assert (np.abs(eps - np.array(g["eps"])) <= 1e-9 * 2.0 ** sizes).all()
    assert abs(r64["total"] - g["total"]) <= 1e-8
    assert abs(r64["total"] - g["gradient"]["e_total"]) <= 1e-8


def test_order4_gradient_against_oracle(order4):
    """gamma_w (every entry) and Gamma_w / 2 (4096 seeded entries and the
    norm of the whole array) against the oracle's densities; mixed
    precision against FP64 at 1e-4."""
    p, g, r64, r32 = order4
    gr = g["gradient"]
    n = p.n_orb
    dh_o = np.array(gr["dE_dh"]).reshape(n, n)
    assert np.abs(r64["dh"] - dh_o).max() <= 1e-8
    idx = np.array(gr["dE_deri_index"])
    assert np.abs(r64["dg"].ravel()[idx] - np.array(gr["dE_deri_value"])).max() <= 1e-8
    assert abs(np.linalg.norm(r64["dg"]) - gr["dE_deri_norm"]) <= 1e-8 * gr["dE_deri_norm"]
    assert np.abs(r32["dh"] - r64["dh"]).max() <= 1e-4
    assert np.abs(r32["dg"] - r64["dg"]).max() <= 1e-4
    _invariants(p, r64, 1e-10)


def test_order4_finite_differences(order4):
    """Central differences (steps 1e-5 and 2e-5, Richardson-extrapolated) of
    the FP64 GPU energy on 16 seeded h pairs and 16 seeded eri orbits
    against the GPU adjoint."""
    p, g, r64, r32 = order4
    print("[w3] order 4 finite differences", flush=True)
    _finite_differences(p, r64, 16, 16, 3001, dict(r_tol=1e-10, max_iter=600), 1e-7, richardson=True)


def test_order5_invariants_mixed_and_finite_differences():
    """Order 5 (1585 increments, 792 x 10o10e): every increment converged,
    trace and Euler identities of the gradient, mixed against FP64 (energies
    within 1e-6, gradient within 1e-4), and central differences on 4 h
    pairs and 4 eri orbits."""
    p = synthetic.workload(3)
    h, eri = _device(p)
    print("[w3] order 5 fp64", flush=True)
    r64 = _solve_grad(p, h, eri, r_tol=1e-9, max_iter=600)
    print("[w3] order 5 mixed", flush=True)
    r32 = _solve_grad(p, h, eri, precision=ifci.MIXED, r_tol=1e-7, r_tol_inner=1e-5, max_iter=600)
    assert len(r64["E"]) == 1585
    assert (r64["status"] == ifci.INC_DONE).all() and (r32["status"] == ifci.INC_DONE).all()
    assert np.abs(r32["E"] - r64["E"]).max() <= 1e-6
    _invariants(p, r64, 1e-10)
    _invariants(p, r32, 1e-6)
    assert np.abs(r32["dh"] - r64["dh"]).max() <= 1e-4
    assert np.abs(r32["dg"] - r64["dg"]).max() <= 1e-4
    print("[w3] order 5 finite differences", flush=True)
    _finite_differences(p, r64, 4, 4, 3005, dict(r_tol=1e-9, max_iter=600), 5e-7)
