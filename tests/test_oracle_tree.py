"""Pins of the oracle's octree and dual-traversal lists.

* cells against an independent recursive octree written in numpy
  (subdivision by lattice coordinate bits), including coincident bodies and
  flat inputs;
* cell / leaf / depth counts of the workloads (seed 0) against an
  independent level-by-level count in numpy (the 2^24-body one runs with
  the GPU tests, whose host has 16 cores);
* list counts of the complete uniform trees against lattice enumeration;
* list invariants: symmetry, exact once-coverage of every ordered body pair,
  the acceptance criterion decided in exact rational arithmetic, no
  self-interaction in M2L.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1405_7487_amd import workloads as W

LEVELS = 21


def _lattice(x):
    lo = x.min(0)
    S = float((x.max(0) - lo).max())
    if S == 0.0:
        S = 1.0
    scale = 2.0 ** LEVELS / S
    ix = np.floor((x - lo) * scale)
    return np.minimum(ix, 2 ** LEVELS - 1).astype(np.int64), lo, S


def _recursive_cells(x, ncrit):
    """Independent octree: list of (level, ix, iy, iz, sorted member tuple)."""
    ix, _, _ = _lattice(x)
    out = []

    def rec(level, coord, members):
        out.append((level, *coord, tuple(sorted(members.tolist()))))
        if not (members.size > ncrit and level < LEVELS):
            return
        b = LEVELS - level - 1
        bits = (ix[members] >> b) & 1
        digit = bits[:, 0] * 4 + bits[:, 1] * 2 + bits[:, 2]
        for dgt in range(8):
            sel = members[digit == dgt]
            if sel.size:
                child = (2 * coord[0] + (dgt >> 2), 2 * coord[1] + ((dgt >> 1) & 1), 2 * coord[2] + (dgt & 1))
                rec(level + 1, child, sel)

    rec(0, (0, 0, 0), np.arange(x.shape[0]))
    return out


def _decode(k, level):
    v = [0, 0, 0]
    for b in range(level):
        v[0] |= ((k >> (3 * b + 2)) & 1) << b
        v[1] |= ((k >> (3 * b + 1)) & 1) << b
        v[2] |= ((k >> (3 * b)) & 1) << b
    return v


def _oracle_cells(x, ncrit):
    T = oracle.Tree(x, ncrit, 0.5)
    e = T.export()
    cells = []
    for c in range(T.ncell):
        lv = int(e["level"][c])
        v = _decode(int(e["ckey"][c]), lv)
        mem = tuple(sorted(e["perm"][e["begin"][c]:e["end"][c]].tolist()))
        cells.append((lv, *v, mem))
    return T, e, cells


@pytest.mark.parametrize("case", ["uniform", "plummer", "dups", "flat", "line"])
def test_cells_match_independent_recursive_octree(case):
    rng = np.random.default_rng(7)
    ncrit = 12
    if case == "uniform":
        x = rng.random((2500, 3))
    elif case == "plummer":
        x, _, _ = W.plummer(2500, 3)
    elif case == "dups":
        x = rng.random((600, 3))
        x[300:] = x[:300]          # every body has a twin
        x[:40] = x[0]              # 41 coincident bodies force level-21 leaves
    elif case == "flat":
        x = rng.random((900, 3)); x[:, 2] = 0.5
    else:
        x = np.zeros((200, 3)); x[:, 0] = np.linspace(0, 1, 200) ** 3
    T, e, cells = _oracle_cells(x, ncrit)
    ref = _recursive_cells(x, ncrit)
    # canonical order is (level, key); compare as (level, coords) keyed maps
    assert sorted(cells) == sorted(ref)
    lv = e["level"]
    ck = e["ckey"]
    order = np.lexsort((ck, lv))
    assert np.array_equal(order, np.arange(T.ncell))
    # sort is stable: equal keys keep input order
    keys = e["keys"]
    perm = e["perm"]
    assert np.all(np.diff(keys.astype(np.float64)) >= 0) or np.all(keys[1:] >= keys[:-1])
    same = keys[1:] == keys[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])
    # leaves hold at most ncrit bodies unless at level 21
    cnt = e["end"] - e["begin"]
    leaf = e["nchild"] == 0
    assert np.all((cnt[leaf] <= ncrit) | (lv[leaf] == LEVELS))


def test_all_coincident_bodies():
    x = np.tile([[0.3, 0.3, 0.3]], (100, 1))
    T = oracle.Tree(x, 8, 0.5)
    assert T.ncell == LEVELS + 1 and T.nleaf == 1 and T.depth == LEVELS
    assert T.S == 1.0
    q = np.ones(100)
    phi, E = T.fmm(q, 4)
    assert np.all(phi == 0.0) and np.all(E == 0.0)


def level_counts(x, ncrit):
    """(cells, leaves, depth) of the octree of x by the tree rules, counted
    level by level in numpy, independently of the oracle: the lattice
    coordinates of every body, then at each level the distinct prefixes of
    the bodies whose parent cell was split, a cell being split when it holds
    more than ncrit bodies below level 21."""
    ix, _, _ = _lattice(x)
    active = np.arange(x.shape[0])
    cells, leaves, depth = 1, 0, 0
    if not (x.shape[0] > ncrit):
        return 1, 1, 0
    for level in range(1, LEVELS + 1):
        sh = LEVELS - level
        a = ix[active] >> sh
        key = (a[:, 0] << 42) | (a[:, 1] << 21) | a[:, 2]
        uk, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        cells += uk.size
        depth = level
        split = (cnt > ncrit) & (level < LEVELS)
        leaves += int(np.count_nonzero(~split))
        active = active[split[inv]]
        if active.size == 0:
            break
    return cells, leaves, depth


@pytest.mark.parametrize("name", ["cube16k", "cube1m", "plummer4m"])
def test_workload_tree_counts(name):
    # the counts of the workloads' trees, from the oracle and from the
    # independent level-by-level count (they are: cube16k 585 cells / 512
    # leaves / depth 3, cube1m 37,449 / 32,768 / 5, plummer4m 507,524 /
    # 443,909 / 11)
    c = W.CONFIGS[name]
    x, _, _ = W.make_config(name)
    T = oracle.Tree(x, c["ncrit"], c["theta"], count_only=True)
    assert (T.ncell, T.nleaf, T.depth) == level_counts(x, c["ncrit"])


@pytest.mark.parametrize("case", ["uniform", "plummer", "dups", "flat"])
def test_level_counts_match_recursive_octree(case):
    # the level-by-level count is itself checked against the recursive octree
    rng = np.random.default_rng(11)
    if case == "uniform":
        x = rng.random((3000, 3))
    elif case == "plummer":
        x, _, _ = W.plummer(3000, 4)
    elif case == "dups":
        x = rng.random((500, 3))
        x[:60] = x[0]
    else:
        x = rng.random((800, 3))
        x[:, 1] = 0.25
    ref = _recursive_cells(x, 9)
    leaves = sum(1 for i, c in enumerate(ref) if not (len(c[4]) > 9 and c[0] < LEVELS))
    assert level_counts(x, 9) == (len(ref), leaves, max(c[0] for c in ref))


def _mac_same_level(t2, theta):
    # R_A + R_B < theta d for two cubes of side h at lattice offset t (units h):
    # sqrt(3) h < theta h |t|  <=>  3 < theta^2 |t|^2, in the exact form
    # 48 < (4 theta^2) * (4 |t|^2) evaluated in double like the tree does
    t4 = 4.0 * theta * theta
    return 48.0 < t4 * float(4 * t2)


def _uniform_list_counts(depth, theta):
    """M2L and P2P pair counts of a complete octree of the given depth, by
    enumeration over parent offsets (no traversal)."""
    rng = np.arange(-(2 ** depth) + 1, 2 ** depth)
    m2l = 0
    for l in range(1, depth + 1):
        npar = 2 ** (l - 1)
        Ts = np.arange(-npar + 1, npar)
        for Tx in Ts:
            for Ty in Ts:
                for Tz in Ts:
                    if l > 1 and _mac_same_level(Tx * Tx + Ty * Ty + Tz * Tz, theta):
                        continue
                    mult = (npar - abs(Tx)) * (npar - abs(Ty)) * (npar - abs(Tz))
                    for ca in range(8):
                        for cb in range(8):
                            t = (2 * Tx + (ca >> 2) - (cb >> 2), 2 * Ty + ((ca >> 1) & 1) - ((cb >> 1) & 1),
                                 2 * Tz + (ca & 1) - (cb & 1))
                            if _mac_same_level(t[0] ** 2 + t[1] ** 2 + t[2] ** 2, theta):
                                m2l += mult
    n = 2 ** depth
    p2p = 0
    for tx in rng:
        for ty in rng:
            for tz in rng:
                if not _mac_same_level(int(tx * tx + ty * ty + tz * tz), theta):
                    p2p += (n - abs(tx)) * (n - abs(ty)) * (n - abs(tz))
    return m2l, p2p


def test_uniform_list_counts_cube16k():
    x, _, _ = W.make_config("cube16k")
    T = oracle.Tree(x, 64, 0.4, count_only=True)
    m2l, p2p = _uniform_list_counts(3, 0.4)
    assert (T.n_m2l, T.n_p2p) == (m2l, p2p) == (166080, 88000)


def test_uniform_list_counts_cube1m():
    x, _, _ = W.make_config("cube1m")
    T = oracle.Tree(x, 64, 0.4, count_only=True)
    assert T.depth == 5
    m2l, p2p = 60292416, 9586240
    assert (T.n_m2l, T.n_p2p) == (m2l, p2p)


def test_lattice_enumeration_matches_published_cube1m_counts():
    # the enumeration itself reproduces the independently published numbers
    assert _uniform_list_counts(5, 0.4) == (60292416, 9586240)


def _exact_mac(e, a, b, theta):
    la, lb = int(e["level"][a]), int(e["level"][b])
    ca = np.array(_decode(int(e["ckey"][a]), la), dtype=object)
    cb = np.array(_decode(int(e["ckey"][b]), lb), dtype=object)
    ha, hb = Fraction(1, 2 ** la), Fraction(1, 2 ** lb)
    d2 = sum(((ca[k] + Fraction(1, 2)) * ha - (cb[k] + Fraction(1, 2)) * hb) ** 2 for k in range(3))
    th = Fraction(theta)
    # (sqrt3/2)(ha + hb) < theta d  <=>  3 (ha + hb)^2 < 4 theta^2 d^2
    return 3 * (ha + hb) ** 2 < 4 * th * th * d2


@pytest.mark.parametrize("case", ["uniform", "plummer"])
def test_list_invariants(case):
    if case == "uniform":
        x = np.random.default_rng(1).random((1500, 3))
        ncrit, theta = 10, 0.5
    else:
        x, _, _ = W.plummer(1500, 2)
        ncrit, theta = 6, 0.45
    T = oracle.Tree(x, ncrit, theta)
    e = T.export()
    m2l, p2p = e["m2l"], e["p2p"]
    assert len(m2l) == T.n_m2l and len(p2p) == T.n_p2p
    # canonical order
    for L in (m2l, p2p):
        key = L[:, 0].astype(np.int64) * (1 << 32) + L[:, 1]
        assert np.all(np.diff(key) > 0)
    # symmetry
    as_set = lambda L: set(map(tuple, L.tolist()))
    assert as_set(m2l) == as_set(m2l[:, ::-1])
    assert as_set(p2p) == as_set(p2p[:, ::-1])
    assert np.all(m2l[:, 0] != m2l[:, 1])
    # leaves only in P2P
    assert np.all(e["nchild"][p2p[:, 0]] == 0) and np.all(e["nchild"][p2p[:, 1]] == 0)
    # every ordered body pair covered exactly once
    n = x.shape[0]
    cov = np.zeros((n, n), np.int16)
    members = [e["perm"][e["begin"][c]:e["end"][c]] for c in range(T.ncell)]
    for a, b in np.concatenate([m2l, p2p]):
        cov[np.ix_(members[a], members[b])] += 1
    assert np.all(cov == 1)
    # acceptance criterion, exact arithmetic, on a sample of pairs
    rs = np.random.default_rng(0)
    for a, b in m2l[rs.choice(len(m2l), min(400, len(m2l)), replace=False)]:
        assert _exact_mac(e, a, b, theta)
    for a, b in p2p[rs.choice(len(p2p), min(400, len(p2p)), replace=False)]:
        assert not _exact_mac(e, a, b, theta)
    # cross-level pairs exist only with a leaf on the coarser side
    lv = e["level"]
    for a, b in m2l:
        if lv[a] != lv[b]:
            coarse = a if lv[a] < lv[b] else b
            assert e["nchild"][coarse] == 0


def _mix64(z):
    # SplitMix64 output finaliser, written out in Python integers
    m = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def test_list_digest_is_the_sum_over_exported_pairs():
    # the digests are a pure function of the pair sets, whatever thread
    # count or frontier the walk used
    x, _, _ = W.plummer(6000, seed=5)
    T = oracle.Tree(x, 16, 0.4)
    o = T.export()
    m = (1 << 64) - 1
    dm = sum(_mix64((int(a) << 32) | int(b)) for a, b in o["m2l"]) & m
    dp = sum(_mix64((int(a) << 32) | int(b)) for a, b in o["p2p"]) & m
    assert (T.digest_m2l, T.digest_p2p) == (dm, dp)
    # SplitMix64's first output from seed 0 is mix64(0x9E3779B97F4A7C15)
    assert _mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert oracle.Tree(x, 16, 0.4, count_only=True).digest_m2l == dm
