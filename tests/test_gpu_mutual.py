"""GPU parity of mutual P2P (each unordered pair of different leaves evaluated
once for both leaves, Section II.C) against the oracle, through the C ABI.

In shallow trees no pair of cells is far enough apart for M2L, so the
whole result is the near field, which the oracle's mutual near field (pinned to the
direct sum and to a sum over the exported list) gives; otherwise the oracle
FMM is the reference, at the bars of the one-sided path (FP64 1e-11 or
tighter, mixed 1e-4).  Cases span leaves of 1-16, 17-32, 33-64 and more
than 64 bodies (the kernel's three row layouts and its target chunks), lists
long enough to be cut into several work items, the compensated pass over
touching leaves, and bit-reproducibility.
"""
import numpy as np
import pytest

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _run(x, q, p, theta, ncrit, precision, mutual=True):
    plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision, mutual=mutual))
    phi, E = plan.evaluate(dev(q))
    return plan, host(phi), host(E)


@pytest.mark.parametrize("n,ncrit", [(600, 16), (800, 24), (3000, 64), (5000, 100)])
def test_near_field_only_matches_oracle_mutual(n, ncrit):
    # shallow trees with theta = 0.25: no pair of cells is far enough apart
    # for M2L, so the FMM is its near field
    x, q, _ = W.uniform_cube(n, 31)
    T = oracle.Tree(x, ncrit, 0.25)
    assert T.n_m2l == 0
    po, Eo = T.near_mutual(q)
    pd, Ed = oracle.direct(x, q)
    assert rel(po, pd) < 1e-13 and rel(Eo, Ed) < 1e-13
    plan, ph, Eh = _run(x, q, 4, 0.25, ncrit, "fp64")
    st = plan.stats()
    assert st["n_m2l"] == 0 and st["n_p2p"] == T.n_p2p
    assert st["p2p_mutual_pairs"] == (T.n_p2p - T.nleaf) // 2
    assert rel(ph, po) < 1e-12 and rel(Eh, Eo) < 1e-12, (rel(ph, po), rel(Eh, Eo))
    _, pm, Em = _run(x, q, 4, 0.25, ncrit, "mixed")
    assert rel(pm, po) < 1e-5 and rel(Em, Eo) < 1e-5, (rel(pm, po), rel(Em, Eo))


@pytest.mark.parametrize("case", ["cube", "plummer", "sphere"])
def test_mutual_fmm_matches_oracle(case):
    if case == "cube":
        x, q, _ = W.uniform_cube(30000, 32)
        p, theta, ncrit = 6, 0.4, 32
    elif case == "plummer":
        x, _, rng = W.plummer(40000, 33)
        q = rng.uniform(-1.0, 1.0, 40000)
        p, theta, ncrit = 6, 0.35, 16
    else:
        x, q, _ = W.sphere_surface(30000, 34)
        p, theta, ncrit = 6, 0.4, 64
    T = oracle.Tree(x, ncrit, theta)
    po, Eo = T.fmm(q, p)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        _, p1, E1 = _run(x, q, p, theta, ncrit, precision, mutual=False)
        plan, pm, Em = _run(x, q, p, theta, ncrit, precision)
        assert plan.stats()["p2p_mutual_pairs"] > 0
        assert rel(pm, po) < tol and rel(Em, Eo) < tol, (precision, rel(pm, po), rel(Em, Eo))
        # the same sums as the one-sided path up to rounding order
        assert rel(pm, p1) < tol and rel(Em, E1) < tol


def test_mutual_long_lists_cut_into_items():
    # coarse halo leaves of a Plummer tree hold more than one work item's
    # worth of upper entries
    x, _, _ = W.plummer(50000, 21)
    q = np.random.default_rng(22).uniform(0.0, 1.0, 50000)
    T = oracle.Tree(x, 6, 0.3)
    po, Eo = T.fmm(q, 3)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        plan, ph, Eh = _run(x, q, 3, 0.3, 6, precision)
        assert rel(ph, po) < tol and rel(Eh, Eo) < tol, (precision, rel(ph, po), rel(Eh, Eo))


def test_mutual_nearly_coincident_bodies_across_leaves():
    # pairs 1e-7 apart anywhere in the box, also on either side of a leaf
    # face: the touching leaves' pass forms differences from compensated
    # coordinates on both sides of the pair
    x, q, _ = W.uniform_cube(20000, 21)
    d = np.random.default_rng(22).normal(size=(10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x[1:20:2] = x[0:20:2] + 1e-7 * d
    T = oracle.Tree(x, 64, 0.4)
    po, Eo = T.fmm(q, 6)
    _, pm, Em = _run(x, q, 6, 0.4, 64, "mixed")
    assert rel(pm, po) < 1e-4 and rel(Em, Eo) < 1e-4, (rel(pm, po), rel(Em, Eo))
    near = np.arange(20)
    assert rel(Em[near], Eo[near]) < 1e-4


def test_mutual_duplicates_and_deep_leaves():
    # many copies of a few points: leaves at the deepest level hold more than
    # N_crit (and more than 64) bodies, coincident pairs are skipped
    x, q, _ = W.uniform_cube(6000, 35)
    x[1000:1300] = x[5]
    x[2000:2100] = x[7]
    T = oracle.Tree(x, 16, 0.4)
    po, Eo = T.fmm(q, 5)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        _, pm, Em = _run(x, q, 5, 0.4, 16, precision)
        assert np.isfinite(pm).all() and np.isfinite(Em).all()
        assert rel(pm, po) < tol and rel(Em, Eo) < tol, (precision, rel(pm, po), rel(Em, Eo))


def test_mutual_bits_reproducible_and_adjoint():
    x, _, rng = W.plummer(30000, 11)
    q = rng.uniform(-1, 1, 30000)
    w = rng.uniform(-1, 1, 30000)
    outs = []
    for _ in range(2):
        _, ph, Eh = _run(x, q, 6, 0.4, 32, "mixed")
        outs.append((ph.tobytes(), Eh.tobytes()))
    assert outs[0] == outs[1]
    # the adjoint runs the same P2P on the loss weights
    T = oracle.Tree(x, 32, 0.4)
    _, Eq = T.fmm(q, 6)
    pw, Ew = T.fmm(w, 6)
    plan = F.Plan(dev(x), F.Params(p=6, theta=0.4, ncrit=32, precision="fp64", mutual=True))
    dq, dx = plan.adjoint(dev(q), dev(w))
    assert rel(host(dq), pw) < 1e-11
    assert rel(host(dx), -(w[:, None] * Eq + q[:, None] * Ew)) < 1e-11


def test_mutual_inside_virtual_ranks():
    # every rank's local near field runs mutually; the remote lists stay
    # one-sided: the same sums as the one-sided ranks up to rounding order
    x, _, rng = W.plummer(30000, 41)
    q = rng.uniform(-1.0, 1.0, 30000)
    outs = {}
    for mutual in (False, True):
        prm = F.Params(p=5, theta=0.4, ncrit=16, precision="fp64", mutual=mutual)
        out = F.let_evaluate(dev(x), dev(q), 3, prm)
        outs[mutual] = (host(out["phi"]), host(out["E"]))
    assert rel(outs[True][0], outs[False][0]) < 1e-12
    assert rel(outs[True][1], outs[False][1]) < 1e-12
