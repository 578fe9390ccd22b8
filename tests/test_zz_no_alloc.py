"""ifci_sigma_noalloc, the sigma entry point for callers that cannot
allocate (its scratch is a fixed device array), against ifci_sigma through
the C ABI: two calls in a row, the second on a smaller increment, in FP64
and mixed precision.  Both run the same kernels in the same order, so the
products must be identical; a product larger than the fixed array is
refused."""
import numpy as np
import pytest

from paper_2307_10675_amd import ifci, synthetic

pytestmark = pytest.mark.gpu


def test_noalloc_sigma_matches_sigma_twice():
    import torch
    print("[noalloc] sigma vs ifci_sigma, 10o10e then smaller increments", flush=True)
    p = synthetic.chain(5, seed=3005, order=5)
    plan = ifci.Plan(p).attach(p.h, p.eri)
    incs = plan.increments()
    big = max(range(len(incs)), key=lambda i: incs[i].n_det)
    small = [i for i, x in enumerate(incs) if x.n_act == 8][0]
    tiny = [i for i, x in enumerate(incs) if x.n_act == 4][0]
    assert incs[big].n_act == 10
    for prec in (ifci.FP64, ifci.MIXED):
        for inc in (big, small, tiny):
            nd = incs[inc].n_det
            c = torch.tensor(synthetic.random_vector(nd, 7 + inc), device="cuda")
            out = torch.full((nd,), float("nan"), dtype=torch.float64, device="cuda")
            plan.sigma_noalloc(inc, out, c, precision=prec)
            ref = plan.sigma(inc, c, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (prec, inc)
            assert bool(torch.isfinite(out).all())
    plan.close()


def test_noalloc_refuses_products_beyond_its_scratch():
    import torch
    print("[noalloc] 12o12e refused", flush=True)
    p = synthetic.chain(6, seed=1101, order=6)
    plan = ifci.Plan(p).attach(p.h, p.eri)
    last = plan.n_inc - 1
    nd = plan.increment(last).n_det
    c = torch.zeros(nd, dtype=torch.float64, device="cuda")
    out = torch.empty_like(c)
    with pytest.raises(ifci.IfciError) as e:
        plan.sigma_noalloc(last, out, c)
    assert e.value.code == 2
    plan.close()
