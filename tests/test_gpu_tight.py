"""GPU parity of the tight acceptance criterion (cell radii squeezed to the
bodies about the lattice centers, Section II.B, Fig. `orb2'): tree, radii-
dependent lists bit-exact against the oracle, potential and field within
1e-10 (float64) / 1e-4 (mixed), and at the full Plummer sizes the list
counts and digests against the oracle's full walk with the pair reduction
reported."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, host, rel
from test_gpu_fmm import _compare_tree

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case,n,p,theta,ncrit", [
    ("plummer", 40000, 6, 0.35, 16),
    ("sphere", 30000, 8, 0.4, 64),
    ("cube", 20000, 4, 0.45, 24),
    ("plummer", 8000, 10, 0.4, 1),
])
def test_tight_lists_and_values(case, n, p, theta, ncrit):
    if case == "plummer":
        x, _, _ = W.plummer(n, 71)
        q = np.random.default_rng(72).uniform(0.0, 1.0, n)
    elif case == "sphere":
        x, q, _ = W.sphere_surface(n, 71)
    else:
        x, q, _ = W.uniform_cube(n, 71)
    T = oracle.Tree(x, ncrit, theta, tight=True)
    po, Eo = T.fmm(q, p)
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision, tight=True))
        g = plan.export_tree()
        o = T.export()
        for k in ("keys", "perm", "level", "begin", "end", "parent", "child_begin", "nchild"):
            assert np.array_equal(g[k], o[k]), k
        assert np.array_equal(g["m2l"], o["m2l"]) and np.array_equal(g["p2p"], o["p2p"])
        phi, E = plan.evaluate(dev(q))
        ep, eE = rel(host(phi), po), rel(host(E), Eo)
        assert ep < tol and eE < tol, (precision, ep, eE)
        plan.close()


@pytest.mark.parametrize("name,ntarget", [("plummer4m", 64), ("plummer16m", 16)])
def test_tight_full_size(name, ntarget):
    cfg = W.CONFIGS[name]
    x_np, q_np, _ = W.make_config(name)
    n = x_np.shape[0]
    tg = W.sample_targets(n, ntarget)
    say(f"[{name}] oracle: full walk with and without the tight criterion")
    Tc = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], count_only=True)
    Tt = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tg, tight=True)
    po, Eo = Tt.fmm(q_np, cfg["p"], targets=tg) if name == "plummer4m" else (None, None)
    say(f"[{name}] cube radii: M2L {Tc.n_m2l} P2P {Tc.n_p2p}; tight: M2L {Tt.n_m2l} P2P {Tt.n_p2p} "
        f"({Tt.n_m2l / Tc.n_m2l:.3f}, {Tt.n_p2p / Tc.n_p2p:.3f})")
    plan = F.Plan(dev(x_np), F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], tight=True))
    st = plan.stats()
    assert (st["ncell"], st["n_m2l"], st["n_p2p"]) == (Tt.ncell, Tt.n_m2l, Tt.n_p2p)
    assert plan.list_digest() == (Tt.digest_m2l, Tt.digest_p2p)
    assert Tt.n_m2l < Tc.n_m2l and Tt.n_p2p < Tc.n_p2p
    if po is not None:
        phi, E = plan.evaluate(dev(q_np))
        ep, eE = rel(host(phi)[tg], po), rel(host(E)[tg], Eo)
        say(f"[{name}] mixed vs oracle: phi {ep:.3e} E {eE:.3e}")
        assert ep < 1e-4 and eE < 1e-4
    plan.close()
