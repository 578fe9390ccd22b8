"""GPU parity of sigma = H c against the oracle's Slater-Condon Hamiltonian,
element by element, through the C ABI."""
import numpy as np
import pytest

from paper_2307_10675_amd import ifci, synthetic
from tests.helpers import active_hamiltonian

pytestmark = pytest.mark.gpu

# one system whose increments span 2o2e .. 8o8e (several MFMA tiles and a ragged tail)
PROBLEM = synthetic.chain(4, seed=77, order=4)
CASES = [(0,), (2,), (0, 1), (1, 3), (0, 1, 2), (1, 2, 3), (0, 1, 2, 3)]


@pytest.fixture(scope="module")
def plan():
    import torch
    print(f"[sigma] plan for chain(4) seed 77, order 4", flush=True)
    p = ifci.Plan(PROBLEM).attach(PROBLEM.h, PROBLEM.eri)
    torch.cuda.synchronize()
    return p


@pytest.fixture(scope="module")
def refs():
    out = {}
    for S in CASES:
        out[S] = active_hamiltonian(PROBLEM, S)
    return out


def _index(plan, S):
    incs = [i.bodies for i in plan.increments()]
    return incs.index(S)


@pytest.mark.parametrize("S", CASES)
def test_sigma_general_fp64(plan, refs, S):
    import torch
    H, n_str, _ = refs[S]
    i = _index(plan, S)
    print(f"[sigma] general fp64 S={S} n_det={H.shape[0]}", flush=True)
    for seed in (1, 2):
        c = synthetic.random_vector(H.shape[0], seed)
        got = plan.sigma(i, torch.tensor(c, device="cuda")).cpu().numpy()
        want = H @ c
        tol = 1e-12 * np.abs(H).max() * np.abs(c).sum()
        assert np.abs(got - want).max() <= tol, (S, np.abs(got - want).max(), tol)


@pytest.mark.parametrize("S", CASES)
def test_sigma_sector_fp64(plan, refs, S):
    import torch
    H, n_str, _ = refs[S]
    i = _index(plan, S)
    print(f"[sigma] sector fp64 S={S}", flush=True)
    c = synthetic.random_vector(H.shape[0], 3, symmetric_dim=n_str)
    got = plan.sigma_sector(i, torch.tensor(c, device="cuda")).cpu().numpy()
    want = H @ c
    tol = 1e-12 * np.abs(H).max() * np.abs(c).sum()
    assert np.abs(got - want).max() <= tol, (S, np.abs(got - want).max(), tol)
    # the product stays in the symmetric sector exactly
    G = got.reshape(n_str, n_str)
    assert np.array_equal(G, G.T)


@pytest.mark.parametrize("S", CASES)
def test_sigma_mixed_precision(plan, refs, S):
    """FP32 arithmetic on both paths: relative error at FP32 level."""
    import torch
    H, n_str, _ = refs[S]
    i = _index(plan, S)
    print(f"[sigma] fp32 S={S}", flush=True)
    c = synthetic.random_vector(H.shape[0], 4, symmetric_dim=n_str)
    want = H @ c
    scale = np.abs(H).max() * np.abs(c).sum()
    for fn in (plan.sigma, plan.sigma_sector):
        got = fn(i, torch.tensor(c, device="cuda"), precision=ifci.MIXED).cpu().numpy()
        err = np.abs(got - want).max()
        assert err <= 2e-6 * scale, (S, err, scale)
        assert err > 0.0  # really computed in FP32


def test_sigma_sector_equals_general_bitwise_symmetry(plan, refs):
    import torch
    S = (0, 1, 2, 3)
    H, n_str, _ = refs[S]
    i = _index(plan, S)
    c = torch.tensor(synthetic.random_vector(H.shape[0], 9, symmetric_dim=n_str), device="cuda")
    a = plan.sigma_sector(i, c).cpu().numpy()
    b = plan.sigma(i, c).cpu().numpy()
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    # repeated calls are bitwise identical (deterministic accumulation)
    assert np.array_equal(a, plan.sigma_sector(i, c).cpu().numpy())


def test_sigma_sector_rejects_large(plan):
    big = synthetic.single(9, 18, 4001)  # 9 orbitals, 4 + 4 electrons: neither on-chip nor column shape
    p = ifci.Plan(big).attach(big.h, big.eri)
    import torch
    c = torch.zeros(p.increment(0).n_det, dtype=torch.float64, device="cuda")
    with pytest.raises(ifci.IfciError) as e:
        p.sigma_sector(0, c)
    assert e.value.code == 2


# Odd orbital counts and fillings away from half: 1-orbital increments (no
# off-diagonal pair, no MFMA row tile), 3- and 6-orbital ones with one or two
# electrons per spin per body.
ODD = [
    ("1o", dict(n_bodies=3, orbs_per_body=1, nocc_per_body=1, order=3, seed=301)),
    ("3o1e", dict(n_bodies=3, orbs_per_body=3, nocc_per_body=1, order=2, seed=302)),
    ("3o2e", dict(n_bodies=2, orbs_per_body=3, nocc_per_body=2, order=2, seed=303)),
]


@pytest.mark.parametrize("name,kw", ODD, ids=[n for n, _ in ODD])
def test_sigma_sector_odd_shapes(name, kw):
    import torch
    print(f"[sigma] odd shapes {name}", flush=True)
    p = synthetic.chain(**kw)
    plan = ifci.Plan(p).attach(p.h, p.eri)
    for i, inc in enumerate(plan.increments()):
        H, n_str, _ = active_hamiltonian(p, inc.bodies)
        c = synthetic.random_vector(H.shape[0], 10 + i, symmetric_dim=n_str)
        want = H @ c
        scale = np.abs(H).max() * np.abs(c).sum()
        got = plan.sigma_sector(i, torch.tensor(c, device="cuda")).cpu().numpy()
        assert np.abs(got - want).max() <= 1e-12 * scale, (name, inc.bodies, np.abs(got - want).max())
        got32 = plan.sigma_sector(i, torch.tensor(c, device="cuda"), precision=ifci.MIXED).cpu().numpy()
        assert np.abs(got32 - want).max() <= 2e-6 * scale, (name, inc.bodies, np.abs(got32 - want).max())
