"""The entry point that allocates nothing (fmm_evaluate_noalloc) against the
one-shot fmm_evaluate on the same inputs, through the C ABI: two calls in a
row on one device, the second with a smaller input, so the second runs on a
scratch array that still holds the first call's data."""
import numpy as np
import pytest
import torch

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _case(n, seed, dist):
    if dist == "cube":
        x, q, _ = W.uniform_cube(n, seed)
    else:
        x, q, _ = W.plummer(n, seed, charges="unit")
    return x, q


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_evaluate_twice(precision):
    # the largest input the entry point takes (uniform bodies at p = 8), then a
    # smaller adaptive one
    n1 = 1 << 17
    cases = [(_case(n1, 51, "cube"), 8, 0.4, 64), (_case(30_000, 52, "plummer"), 6, 0.4, 32)]
    for (x, q), p, theta, ncrit in cases:
        xt, qt = dev(x), dev(q)
        # the library's own one-shot entry point (plan memory from torch)
        phi_r, E_r = F.evaluate(xt, qt, p=p, theta=theta, ncrit=ncrit, precision=precision)
        # the one that allocates nothing; its outputs are the caller's tensors
        phi = torch.full_like(phi_r, np.nan)
        E = torch.full_like(E_r, np.nan)
        F.evaluate_noalloc(xt, qt, p=p, theta=theta, ncrit=ncrit, precision=precision, out=(phi, E))
        torch.cuda.synchronize()
        # the same kernels on the same tree and lists; the cross-level products
        # may reach a target in more chunks (the scratch keeps their buffer
        # small), so sums can group differently: equal to rounding
        bar = 1e-12 if precision == "fp64" else 1e-6
        assert rel(host(phi), host(phi_r)) < bar and rel(host(E), host(E_r)) < bar, (precision, x.shape[0])
        assert not torch.isnan(phi).any() and not torch.isnan(E).any()
        # and within the bar against the oracle at sampled targets
        tg = W.sample_targets(x.shape[0], 256)
        T = oracle.Tree(x, ncrit, theta, targets=tg)
        po, Eo = T.fmm(q, p, targets=tg)
        tol = 1e-4 if precision == "mixed" else 1e-10
        assert rel(host(phi)[tg], po) < tol and rel(host(E)[tg], Eo) < tol


def test_noalloc_limits_and_errors():
    x, q = _case(1000, 53, "cube")
    # field is optional
    phi, E = F.evaluate_noalloc(dev(x), dev(q), p=4, field=False)
    assert E is None
    phi_r, _ = F.evaluate(dev(x), dev(q), p=4, field=False)
    assert rel(host(phi), host(phi_r)) < 1e-6
    # beyond the stated maximum n: a clear error, nothing runs
    big = torch.zeros(((1 << 17) + 1, 3), dtype=torch.float64, device="cuda:0")
    big[:, 0] = torch.arange(big.shape[0], dtype=torch.float64, device="cuda:0")
    with pytest.raises(F.FMMError) as ei:
        F.evaluate_noalloc(big, torch.ones(big.shape[0], dtype=torch.float64, device="cuda:0"), p=4)
    assert ei.value.code == 4 and "exceeds" in str(ei.value)
    # a plan larger than the scratch (a deep adaptive tree at high order and a
    # tight acceptance criterion): out of scratch, reported, and the next call works
    xp, qp = _case(1 << 17, 54, "plummer")
    with pytest.raises(F.FMMError) as ei:
        F.evaluate_noalloc(dev(xp), dev(qp), p=12, theta=0.3, ncrit=8)
    assert ei.value.code == 2 and "scratch" in str(ei.value)
    phi2, _ = F.evaluate_noalloc(dev(x), dev(q), p=4, field=False)
    assert rel(host(phi2), host(phi_r)) < 1e-6
