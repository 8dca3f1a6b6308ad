"""Pins of the oracle's tight acceptance criterion (cells squeezed to their
bodies, Section II.B, Fig. `orb2'; error O(theta^P), Section III.A).

Each cell keeps its lattice center; its radius is the farthest corner of a
member body's lattice cell, rounded up to units u = S 2^-22.  A pair is
accepted when the cube radii or these radii meet R_A + R_B < theta d.

* radii against a computation in Python integers from the bodies' own
  lattice coordinates, and against the true distances (a bound, at most one
  unit above the cube radius);
* the lists keep their invariants (symmetry, every ordered body pair covered
  once) and their acceptance decisions hold in exact rational arithmetic;
* the error stays inside the a priori bound with the true radii;
* the criterion removes pairs; without it nothing changes.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1405_7487_amd import workloads as W

from test_oracle_fmm import _a_priori_bound
from test_oracle_tree import LEVELS, _decode, _exact_mac, _lattice


def _case(name, n, seed):
    if name == "plummer":
        x, _, _ = W.plummer(n, seed)
        q = np.random.default_rng(seed).uniform(-1, 1, n)
    elif name == "sphere":
        x, q, _ = W.sphere_surface(n, seed)
    else:
        x, q, _ = W.uniform_cube(n, seed)
    return x, q


@pytest.mark.parametrize("case", ["plummer", "sphere", "cube"])
def test_radii(case):
    x, _ = _case(case, 3000, 3)
    T = oracle.Tree(x, 12, 0.4, tight=True)
    e = T.export()
    rad = T.radii()
    ix, lo, S = _lattice(x)
    u = S * 2.0 ** -22
    for c in range(T.ncell):
        l = int(e["level"][c])
        C = [(2 * v + 1) << (LEVELS - l) for v in _decode(int(e["ckey"][c]), l)]
        mem = e["perm"][e["begin"][c]:e["end"][c]]
        best = 0
        for j in mem:
            s = 0
            for d in range(3):
                v = int(ix[j, d])
                s += max(abs(2 * v - C[d]), abs(2 * v + 2 - C[d])) ** 2
            best = max(best, s)
        want = math.isqrt(best)
        if want * want < best:
            want += 1
        assert rad[c] == want, c
        # a bound on the true distances, never much above the cube radius
        ctr = e["centers"][c]
        assert np.max(np.linalg.norm(x[mem] - ctr, axis=1)) <= rad[c] * u * (1 + 1e-12)
        assert rad[c] <= math.sqrt(3) * 2 ** (LEVELS - l) + 1


def _exact_tight(e, rad, a, b, theta):
    la, lb = int(e["level"][a]), int(e["level"][b])
    ca = [(2 * v + 1) << (LEVELS - la) for v in _decode(int(e["ckey"][a]), la)]
    cb = [(2 * v + 1) << (LEVELS - lb) for v in _decode(int(e["ckey"][b]), lb)]
    d2 = sum((ca[k] - cb[k]) ** 2 for k in range(3))
    th = Fraction(theta)
    return (int(rad[a]) + int(rad[b])) ** 2 < th * th * d2


@pytest.mark.parametrize("case,ncrit,theta", [("plummer", 6, 0.45), ("sphere", 10, 0.4)])
def test_list_invariants(case, ncrit, theta):
    x, _ = _case(case, 1500, 5)
    T = oracle.Tree(x, ncrit, theta, tight=True)
    e = T.export()
    rad = T.radii()
    m2l, p2p = e["m2l"], e["p2p"]
    as_set = lambda L: set(map(tuple, L.tolist()))
    assert as_set(m2l) == as_set(m2l[:, ::-1]) and as_set(p2p) == as_set(p2p[:, ::-1])
    n = x.shape[0]
    cov = np.zeros((n, n), np.int16)
    members = [e["perm"][e["begin"][c]:e["end"][c]] for c in range(T.ncell)]
    for a, b in np.concatenate([m2l, p2p]):
        cov[np.ix_(members[a], members[b])] += 1
    assert np.all(cov == 1)
    rs = np.random.default_rng(0)
    n_tight_only = 0
    for a, b in m2l[rs.choice(len(m2l), min(500, len(m2l)), replace=False)]:
        cube = _exact_mac(e, a, b, theta)
        assert cube or _exact_tight(e, rad, a, b, theta)
        n_tight_only += not cube
    assert n_tight_only > 0  # the tight radii accept pairs the cube radii would not
    for a, b in p2p[rs.choice(len(p2p), min(500, len(p2p)), replace=False)]:
        assert not _exact_mac(e, a, b, theta) and not _exact_tight(e, rad, a, b, theta)


@pytest.mark.parametrize("case,p", [("plummer", 5), ("sphere", 4)])
def test_error_within_a_priori_bound(case, p):
    x, q = _case(case, 5000, 7)
    tg = W.sample_targets(x.shape[0], 120)
    T = oracle.Tree(x, 16, 0.4, targets=tg, tight=True)
    e = T.export()
    phi, E = T.fmm(q, p, targets=tg)
    pd, Ed = oracle.direct(x, q, targets=tg)
    bphi, bE = _a_priori_bound(x, q, T, e, p, tg)
    assert np.all(np.abs(phi - pd) <= bphi + 1e-12 * (np.abs(pd) + 1))
    assert np.all(np.linalg.norm(E - Ed, axis=1) <= bE + 1e-12 * (np.linalg.norm(Ed, axis=1) + 1))


def test_fewer_pairs_and_unchanged_without():
    x, q = _case("plummer", 20000, 1)
    Tc = oracle.Tree(x, 16, 0.4)
    Tt = oracle.Tree(x, 16, 0.4, tight=True)
    assert (Tt.ncell, Tt.nleaf) == (Tc.ncell, Tc.nleaf)
    assert Tt.n_m2l < Tc.n_m2l and Tt.n_p2p < Tc.n_p2p
    assert np.all(Tc.radii() == 0)
