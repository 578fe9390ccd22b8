"""Fused column sigma of the device-wide path (half-filled increments of 10,
12 and 14 orbitals, symmetric sector): sampled rows against the oracle's
Slater-Condon rows, and agreement with the general device-wide product."""
import numpy as np
import pytest

from oracle import certify
from paper_2307_10675_amd import ifci, synthetic

pytestmark = pytest.mark.gpu

SIZES = [(10, 20, 4210), (12, 24, 4212), (14, 28, 4214)]


def _sym_vectors(n_str, seed):
    """A random symmetric C as its packed scaled vector and its full form."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n_str, n_str))
    C = C + C.T
    C /= np.linalg.norm(C)
    a, b = np.triu_indices(n_str)
    # packed index of (a <= b) is b (b + 1) / 2 + a
    cp = np.empty(n_str * (n_str + 1) // 2)
    cp[b * (b + 1) // 2 + a] = np.where(a == b, 1.0, np.sqrt(2.0)) * C[a, b]
    return cp, C


@pytest.mark.parametrize("n,K,seed", SIZES)
def test_column_sigma_rows(n, K, seed):
    import torch
    print(f"[column] {n}o{n}e rows", flush=True)
    p = synthetic.single(n, K, seed)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(np.sqrt(plan.increment(0).n_det)))
    cp, C = _sym_vectors(n_str, seed + 1)
    rng = np.random.default_rng(seed + 2)
    rows = np.sort(rng.choice(n_str * n_str, 40, replace=False))
    want = certify.sigma_rows_strings(rows, n // 2, C.reshape(-1), p.h, p.eri)
    ra, rb = rows // n_str, rows % n_str
    lo, hi = np.minimum(ra, rb), np.maximum(ra, rb)
    idx = hi * (hi + 1) // 2 + lo
    scale = np.where(ra == rb, 1.0, np.sqrt(2.0))
    ref = scale * want
    big = max(1.0, np.abs(want).max())
    for prec, tol in ((ifci.FP64, 1e-12 * n), (ifci.MIXED, 2e-5)):
        got = plan.sigma_sector(0, torch.tensor(cp, device="cuda"), precision=prec).cpu().numpy()
        assert np.abs(got[idx] - ref).max() <= tol * big, (prec, np.abs(got[idx] - ref).max())


def test_column_sigma_equals_general_path():
    """Packed column sigma equals the general device-wide product (E
    materialised in HBM) on the full symmetric vector, FP64, 10o10e."""
    import torch
    p = synthetic.single(10, 20, 4220)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(np.sqrt(plan.increment(0).n_det)))
    cp, C = _sym_vectors(n_str, 7)
    full = plan.sigma(0, torch.tensor(C.reshape(-1), device="cuda")).cpu().numpy().reshape(n_str, n_str)
    got = plan.sigma_sector(0, torch.tensor(cp, device="cuda")).cpu().numpy()
    a, b = np.triu_indices(n_str)
    ref = np.where(a == b, 1.0, np.sqrt(2.0)) * full[a, b]
    assert np.abs(got[b * (b + 1) // 2 + a] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_column_sigma_repeatable():
    """Two products of the same vector agree to FP64 rounding (the LDS
    accumulation order of the scatter is not fixed)."""
    import torch
    p = synthetic.single(12, 24, 4230)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(np.sqrt(plan.increment(0).n_det)))
    cp, _ = _sym_vectors(n_str, 9)
    c = torch.tensor(cp, device="cuda")
    for prec in (ifci.FP64, ifci.MIXED):
        x = plan.sigma_sector(0, c, precision=prec).cpu().numpy()
        y = plan.sigma_sector(0, c, precision=prec).cpu().numpy()
        assert np.abs(x - y).max() <= 1e-13 * max(1.0, np.abs(x).max())


def test_column_sigma_rows_16_orbitals():
    """16o16e (165,636,900 determinants): the split column kernel (fragments
    in passes, an FP64 accumulator in both precisions) on 24 sampled rows
    against the oracle's Slater-Condon rows, and repeatable to FP64 rounding;
    the general product is unsupported at this size and says so."""
    import torch
    print("[column] 16o16e rows", flush=True)
    n, K, seed = 16, 32, 4216
    p = synthetic.single(n, K, seed)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(np.sqrt(plan.increment(0).n_det)))
    assert n_str == 12870
    cp, C = _sym_vectors(n_str, seed + 1)
    rng = np.random.default_rng(seed + 2)
    rows = np.sort(rng.choice(n_str * n_str, 24, replace=False))
    want = certify.sigma_rows_strings(rows, n // 2, C.reshape(-1), p.h, p.eri)
    del C
    ra, rb = rows // n_str, rows % n_str
    lo, hi = np.minimum(ra, rb), np.maximum(ra, rb)
    idx = hi * (hi + 1) // 2 + lo
    ref = np.where(ra == rb, 1.0, np.sqrt(2.0)) * want
    big = max(1.0, np.abs(want).max())
    c = torch.tensor(cp, device="cuda")
    for prec, tol in ((ifci.FP64, 1e-12 * n), (ifci.MIXED, 2e-5)):
        x = plan.sigma_sector(0, c, precision=prec)
        got = x[torch.tensor(idx, device="cuda")].cpu().numpy()
        assert np.abs(got - ref).max() <= tol * big, (prec, np.abs(got - ref).max())
        # a second product agrees to FP64 rounding (the scatter's order is not fixed)
        y = plan.sigma_sector(0, c, precision=prec)
        assert float((x - y).abs().max()) <= 1e-13 * float(x.abs().max()), prec
        del x, y
    full = torch.zeros(n_str * n_str, dtype=torch.float64, device="cuda")
    with pytest.raises(ifci.IfciError) as e:
        plan.sigma(0, full)
    assert e.value.code == 2
