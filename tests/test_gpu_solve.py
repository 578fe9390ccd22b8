"""GPU parity of the increment solver and the energy assembly against oracle
energies (written by tests/golden/make_oracle_refs.py from oracle/ only)."""
import math

import numpy as np
import pytest

from oracle import fci, ifci as oifci
from paper_2307_10675_amd import ifci, synthetic
from tests.helpers import active_hamiltonian, load_golden

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
# max_space 12: thick-restart Davidson; max_space 3: the {x, w, p} solver;
# each started from the lowest determinant with the diagonal preconditioner
# (n_guess 0) or from the lowest eigenvector of the 64-determinant P-space
# block with that block's exact inverse as preconditioner (the default)
SPACES = [pytest.param(dict(max_space=12, n_guess=0), id="davidson12"),
          pytest.param(dict(max_space=12), id="davidson12_pspace"),
          pytest.param(dict(max_space=3, n_guess=0), id="3vec"),
          pytest.param(dict(max_space=3), id="3vec_pspace")]


def _check_sha(problem, g):
    assert problem.sha256() == g["sha256"], "synthetic generator changed; regenerate tests/golden"


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("rep", range(10))
def test_workload0_fp64_davidson(rep, space):
    """6 orbitals / 6 electrons: lowest even-spin root to residual 1e-10."""
    import torch
    p = synthetic.workload(0, rep)
    g = load_golden(f"w0_r{rep}")
    _check_sha(p, g)
    print(f"[solve] workload 0 replicate {rep} {space}", flush=True)
    plan, res = ifci.solve(p, r_tol=1e-10, **space, max_iter=500)
    torch.cuda.synchronize()
    assert int(res["status"][0]) == ifci.INC_DONE
    assert float(res["resid"][0]) <= 1e-10
    assert abs(float(res["E"][0]) - g["increments"][0]["E"]) <= TOL64


@pytest.mark.parametrize("solver,space", [(ifci.BATCHED, dict(max_space=12)), (ifci.BATCHED, dict(max_space=3)),
                                          (ifci.BATCHED, dict(max_space=3, n_guess=0)),
                                          (ifci.PLAIN, dict(max_space=12))])
def test_workload1_all_increments(solver, space):
    """10 bodies, order 3: all 175 increments, eps_S and the total."""
    import torch
    p = synthetic.workload(1)
    g = load_golden("w1")
    _check_sha(p, g)
    print(f"[solve] workload 1 solver {solver} {space}", flush=True)
    plan, res = ifci.solve(p, solver=solver, r_tol=1e-8, **space, max_iter=500)
    torch.cuda.synchronize()
    E = res["E"].cpu().numpy()
    st = res["status"].cpu().numpy()
    assert (st == ifci.INC_DONE).all()
    ref = np.array([x["E"] for x in g["increments"]])
    assert [tuple(x["bodies"]) for x in g["increments"]] == [i.bodies for i in plan.increments()]
    assert np.abs(E - ref).max() <= TOL64
    eps = res["eps"].cpu().numpy()
    sizes = np.array([len(x["bodies"]) for x in g["increments"]])
    assert (np.abs(eps - np.array(g["eps"])) <= TOL64 * 2.0 ** sizes).all()
    assert abs(res["e_ref"] - g["e_ref"]) <= 1e-12
    for k in range(3):
        assert abs(res["by_order"][k] - g["by_order"][k]) <= TOL64 * 2 ** (k + 1) * math.comb(10, k + 1)
    assert abs(res["total"] - g["total"]) <= 1e-8


@pytest.mark.parametrize("space", SPACES)
def test_full_order_identity(space):
    """Four bodies to full order: the expansion total equals the 8o8e FCI energy."""
    import torch
    p = synthetic.chain(4, seed=1100, order=4)
    g = load_golden("chain4_full")
    _check_sha(p, g)
    plan, res = ifci.solve(p, r_tol=1e-9, **space, max_iter=500)
    torch.cuda.synchronize()
    E = res["E"].cpu().numpy()
    assert np.abs(E - np.array([x["E"] for x in g["increments"]])).max() <= TOL64
    assert abs(res["total"] - float(E[-1])) <= 1e-10
    assert abs(res["total"] - g["total"]) <= 1e-9


@pytest.mark.parametrize("space", SPACES)
def test_workload2_all_increments(space):
    """16 bodies, order 4: every one of the 2516 increments against the
    oracle's exact energy.  FP64 to residual 1e-8 within 1e-9 (eps_S within
    2^|S| x 1e-9, order sums and total within 1e-8); mixed precision at the
    benchmark's tolerances (FP32 stage to residual 1e-5, then the FP64
    residual test at 1e-5) within 1e-6 on every increment."""
    import torch
    p = synthetic.workload(2)
    g = load_golden("w2")
    _check_sha(p, g)
    print(f"[solve] workload 2 fp64 {space}", flush=True)
    plan64, r64 = ifci.solve(p, r_tol=1e-8, max_iter=600, **space)
    print(f"[solve] workload 2 mixed {space}", flush=True)
    plan32, r32 = ifci.solve(p, precision=ifci.MIXED, r_tol=1e-5, r_tol_inner=1e-5, max_iter=600,
                             **space)
    torch.cuda.synchronize()
    assert [tuple(x["bodies"]) for x in g["increments"]] == [i.bodies for i in plan64.increments()]
    ref = np.array([x["E"] for x in g["increments"]])
    E64 = r64["E"].cpu().numpy()
    E32 = r32["E"].cpu().numpy()
    assert (r64["status"].cpu().numpy() == ifci.INC_DONE).all()
    assert (r32["status"].cpu().numpy() == ifci.INC_DONE).all()
    assert np.abs(E64 - ref).max() <= TOL64
    assert np.abs(E32 - ref).max() <= 1e-6
    sizes = np.array([len(x["bodies"]) for x in g["increments"]])
    assert (np.abs(r64["eps"].cpu().numpy() - np.array(g["eps"])) <= TOL64 * 2.0 ** sizes).all()
    assert np.abs(np.array(r64["by_order"]) - np.array(g["by_order"])).max() <= 1e-8
    assert abs(r64["total"] - g["total"]) <= 1e-8


@pytest.mark.parametrize("space", SPACES)
def test_mixed_uses_fp32_stage_and_refines(space):
    """Mixed precision: FP32 sigma stage, then FP64 refinement to 1e-9 Eh."""
    import torch
    p = synthetic.workload(0, 3)
    g = load_golden("w0_r3")
    plan, res = ifci.solve(p, precision=ifci.MIXED, r_tol=1e-7, r_tol_inner=1e-5, **space, max_iter=500)
    torch.cuda.synchronize()
    assert int(res["status"][0]) == ifci.INC_DONE
    assert abs(float(res["E"][0]) - g["increments"][0]["E"]) <= 1e-9


def test_vector_matches_oracle():
    import torch
    p = synthetic.chain(3, seed=5, order=3)
    plan, res = ifci.solve(p, r_tol=1e-10)
    incs = [i.bodies for i in plan.increments()]
    for S in [(0, 1), (0, 1, 2)]:
        i = incs.index(S)
        H, n_str, s = active_hamiltonian(p, S)
        r = fci.solve_increment(p, S)
        want = fci.normalise_sign(s * r["c"])
        got = fci.normalise_sign(plan.vector(i).cpu().numpy())
        assert r["gap"] > 1e-6
        assert np.abs(got - want).max() < 1e-8
        C = got.reshape(n_str, n_str)
        assert np.abs(C - C.T).max() == 0.0


@pytest.mark.parametrize("space", SPACES)
def test_eviction_requeue_bitwise(space):
    """Failure injection: evicted increments report EVICTED; solving them
    again gives bitwise the energies of an undisturbed run."""
    import torch
    p = synthetic.workload(1)
    plan, clean = ifci.solve(p, r_tol=1e-8, **space, max_iter=500)
    n = plan.n_inc
    mask = np.zeros(n, dtype=np.uint8)
    mask[::7] = 1
    plan2 = ifci.Plan(p, r_tol=1e-8, **space, max_iter=500).attach(p.h, p.eri)
    e, st, it, rs = plan2.davidson(evict=mask)
    st = st.cpu().numpy()
    assert (st[mask == 1] == ifci.INC_EVICTED).all()
    assert (st[mask == 0] == ifci.INC_DONE).all()
    e = e.cpu().numpy()
    for i in np.nonzero(mask)[0]:
        e1, st1, _, _ = plan2.davidson(first=int(i), count=1)
        assert int(st1[0]) == ifci.INC_DONE
        e[i] = float(e1[0])
    torch.cuda.synchronize()
    assert np.array_equal(e, clean["E"].cpu().numpy())


def test_not_converged_status():
    import torch
    p = synthetic.workload(0, 1)
    plan = ifci.Plan(p, max_iter=2, r_tol=1e-12).attach(p.h, p.eri)
    e, st, it, rs = plan.davidson()
    assert int(st[0]) == ifci.INC_NOT_CONVERGED
    assert int(it[0]) == 2
    en = plan.energy(e, st)
    assert en["converged"] is False


@pytest.mark.parametrize("space", SPACES)
def test_deterministic_bitwise(space):
    import torch
    p = synthetic.workload(1)
    _, a = ifci.solve(p, r_tol=1e-8, **space, max_iter=500)
    _, b = ifci.solve(p, r_tol=1e-8, **space, max_iter=500)
    assert np.array_equal(a["E"].cpu().numpy(), b["E"].cpu().numpy())
    assert a["total"] == b["total"]


def test_separable_bodies_closed_form():
    import torch
    p = synthetic.separable(6, seed=3, order=3)
    plan, res = ifci.solve(p, r_tol=1e-10)
    eps = res["eps"].cpu().numpy()
    incs = plan.increments()
    for e, inf in zip(eps, incs):
        if len(inf.bodies) >= 2:
            assert abs(e) < 1e-10
    corr = 0.0
    for orbs in p.bodies:
        q = synthetic.Problem(p.h[np.ix_(orbs, orbs)], p.eri[np.ix_(orbs, orbs, orbs, orbs)], [[0, 1]], [1], 1)
        corr += fci.solve_increment(q, (0,))["E"] - oifci.reference_energy(q)
    assert abs(res["total"] - (res["e_ref"] + corr)) < 1e-10


ODD = [
    ("1o", dict(n_bodies=3, orbs_per_body=1, nocc_per_body=1, order=3, seed=311)),
    ("3o1e", dict(n_bodies=3, orbs_per_body=3, nocc_per_body=1, order=2, seed=312)),
    ("3o2e", dict(n_bodies=2, orbs_per_body=3, nocc_per_body=2, order=2, seed=313)),
]


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("name,kw", ODD, ids=[n for n, _ in ODD])
def test_solve_odd_shapes(name, kw, space):
    """The on-chip solvers on odd orbital counts and fillings away from half
    (1-orbital increments with no off-diagonal pair, 3o/6o increments with one
    or two electrons per spin and body), FP64 and mixed, against the oracle's
    exact increment energies."""
    import torch
    print(f"[solve] odd shapes {name} {space}", flush=True)
    p = synthetic.chain(**kw)
    plan64, r64 = ifci.solve(p, r_tol=1e-9, max_iter=500, **space)
    plan32, r32 = ifci.solve(p, precision=ifci.MIXED, r_tol=3e-5, r_tol_inner=1e-5, max_iter=500,
                             **space)
    torch.cuda.synchronize()
    E64 = r64["E"].cpu().numpy()
    E32 = r32["E"].cpu().numpy()
    assert (r64["status"].cpu().numpy() == ifci.INC_DONE).all()
    assert (r32["status"].cpu().numpy() == ifci.INC_DONE).all()
    for i, inc in enumerate(plan64.increments()):
        want = fci.solve_increment(p, inc.bodies)["E"]
        assert abs(E64[i] - want) <= TOL64, (name, inc.bodies, E64[i] - want)
        assert abs(E32[i] - want) <= 1e-6, (name, inc.bodies, E32[i] - want)
