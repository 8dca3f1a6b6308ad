"""GPU parity of the virtual-rank evaluation (fmm_let_evaluate) against the
oracle's: partition bit for bit, every rank's local lists and every LET and
remote list through counts and digests, the work counts l_i and r_i exactly,
and potential and field within 1e-10 (float64) / 1e-4 (mixed) relative L2."""
import numpy as np
import pytest
import torch

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _case(name, n, seed):
    if name == "cube":
        x, q, _ = W.uniform_cube(n, seed)
    elif name == "plummer":
        x, _, _ = W.plummer(n, seed)
        q = np.random.default_rng(seed).uniform(0.0, 1.0, n)
    else:
        x, q, _ = W.sphere_surface(n, seed)
    return x, q


@pytest.mark.parametrize("case,n,R,p,theta,ncrit", [
    ("cube", 40000, 4, 6, 0.4, 32),
    ("plummer", 60000, 7, 8, 0.35, 16),
    ("sphere", 30000, 3, 5, 0.4, 64),
    ("plummer", 20000, 16, 4, 0.45, 8),
])
def test_let_matches_oracle(case, n, R, p, theta, ncrit):
    x, q = _case(case, n, 61)
    L = oracle.Let(x, R, ncrit, theta)
    po, Eo = L.fmm(q, p)
    lw, rw = L.work()
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        out = F.let_evaluate(dev(x), dev(q), R, F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision),
                             work=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(out["rank"]).astype(np.int32), L.rank)
        assert np.array_equal(out["pair_stats"], L.pair_stats), (case, precision)
        assert np.array_equal(out["work_local"].cpu().numpy(), lw)
        assert np.array_equal(out["work_remote"].cpu().numpy(), rw)
        ep, eE = rel(host(out["phi"]), po), rel(host(out["E"]), Eo)
        assert ep < tol and eE < tol, (case, precision, ep, eE)
        st = out["stats"]
        assert st["n_m2l_remote"] > 0 and st["let_cells"] > 0


def test_let_one_rank_and_weights():
    x, q = _case("plummer", 30000, 62)
    prm = F.Params(p=6, theta=0.4, ncrit=16, precision="fp64")
    one = F.let_evaluate(dev(x), dev(q), 1, prm, work=True)
    phi, E = F.Plan(dev(x), prm).evaluate(dev(q))
    assert torch.equal(one["phi"], phi) and torch.equal(one["E"], E)
    # a second partition weighted by the first one's work (Eq. (1), alpha = 2)
    w = one["work_local"] + 2 * one["work_remote"]
    L = oracle.Let(x, 5, 16, 0.4, weights=w.cpu().numpy())
    out = F.let_evaluate(dev(x), dev(q), 5, prm, weights=w)
    assert np.array_equal(host(out["rank"]).astype(np.int32), L.rank)
    assert np.array_equal(out["pair_stats"], L.pair_stats)
    po, Eo = L.fmm(q, 6)
    assert rel(host(out["phi"]), po) < 1e-10 and rel(host(out["E"]), Eo) < 1e-10
    # bad weights are rejected
    with pytest.raises(F.FMMError) as ei:
        F.let_evaluate(dev(x), dev(q), 5, prm, weights=-torch.ones_like(w))
    assert ei.value.code == 1
