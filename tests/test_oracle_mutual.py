"""Pins of the oracle's mutual near field (every unordered body pair of the
P2P lists evaluated once, both bodies updated; mutual interactions are among
the features Section II.C lists): against a brute-force sum over the
exported P2P list written here in numpy, against the direct sum when one
leaf holds every body, Newton's third law, and coincident bodies."""
import numpy as np
import pytest

import oracle
from paper_1405_7487_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def _near_from_list(x, q, ex):
    """One-sided near field of every body straight from the exported list:
    for each (target leaf, source leaf) pair every body of the target gains
    every body of the source, coincident bodies skipped."""
    n = x.shape[0]
    perm, beg, end = ex["perm"], ex["begin"], ex["end"]
    xs, qs = x[perm], q[perm]
    phi, E = np.zeros(n), np.zeros((n, 3))
    for a, b in ex["p2p"]:
        ta, sb = slice(beg[a], end[a]), slice(beg[b], end[b])
        d = xs[ta][:, None, :] - xs[sb][None, :, :]
        r2 = (d * d).sum(-1)
        with np.errstate(divide="ignore"):
            ri = np.where(r2 > 0, 1.0 / np.sqrt(np.where(r2 > 0, r2, 1.0)), 0.0)
        w = qs[sb][None, :] * ri
        phi[ta] += w.sum(1)
        E[ta] += ((w * ri * ri)[:, :, None] * d).sum(1)
    out_phi, out_E = np.zeros(n), np.zeros((n, 3))
    out_phi[perm], out_E[perm] = phi, E
    return out_phi, out_E


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("kind,n,ncrit,theta", [("cube", 600, 8, 0.5), ("plummer", 1500, 16, 0.4),
                                                 ("sphere", 800, 12, 0.6)])
def test_mutual_near_field_is_the_list_sum(kind, n, ncrit, theta):
    if kind == "cube":
        x, q, _ = W.uniform_cube(n, seed=3)
    elif kind == "plummer":
        x, q, _ = W.plummer(n, seed=4, charges="unit")
    else:
        x, q, _ = W.sphere_surface(n, seed=5)
    t = oracle.Tree(x, ncrit, theta)
    phi, E = t.near_mutual(q)
    want_phi, want_E = _near_from_list(x, q, t.export())
    assert _rel(phi, want_phi) < 1e-13
    assert _rel(E, want_E) < 1e-13


def test_mutual_single_leaf_is_the_direct_sum():
    x, q, _ = W.uniform_cube(300, seed=7)
    t = oracle.Tree(x, 300, 0.5)
    assert t.nleaf == 1
    phi, E = t.near_mutual(q)
    dphi, dE = oracle.direct(x, q)
    assert _rel(phi, dphi) < 1e-14
    assert _rel(E, dE) < 1e-14


def test_mutual_near_field_obeys_newtons_third_law():
    # each pair adds equal and opposite forces q_i E_i and q_j E_j, so their
    # sum over all bodies vanishes up to rounding
    x, _, rng = W.plummer(2000, seed=9)
    q = rng.uniform(-1.0, 1.0, x.shape[0])
    t = oracle.Tree(x, 16, 0.4)
    _, E = t.near_mutual(q)
    F = q[:, None] * E
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).sum()


def test_mutual_skips_coincident_bodies():
    x, q, _ = W.uniform_cube(400, seed=11)
    x[10] = x[20]
    x[30] = x[31] = x[32]
    t = oracle.Tree(x, 8, 0.5)
    phi, E = t.near_mutual(q)
    assert np.isfinite(phi).all() and np.isfinite(E).all()
    want_phi, want_E = _near_from_list(x, q, t.export())
    assert _rel(phi, want_phi) < 1e-13
    assert _rel(E, want_E) < 1e-13
