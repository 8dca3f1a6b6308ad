"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tree, keys, permutation, cells, centers and lists must be bit-exact; the
FP64 GPU FMM must match the oracle FMM within 1e-6 relative L2 (expected:
roundoff, ~1e-13) and the mixed FP32/MFMA path within 1e-4, on potential and
field.  Sizes span many tiles and leave ragged tails (counts not multiples of
64 targets per tile, leaves with few bodies, cross-level pairs).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, gpu_fmm, host, rel

pytestmark = pytest.mark.gpu


def test_mfma_lane_layout():
    for f64 in (False, True):
        out = np.asarray(F.mfma_layout(f64), dtype=np.float64)
        exp = np.zeros(256)
        for l in range(64):
            for e in range(4):
                # accumulator rows: 4 (l/16) + e for float32, l/16 + 4 e for float64
                i = (l // 16 + 4 * e) if f64 else (4 * (l // 16) + e)
                j = l % 16
                exp[4 * l + e] = (i + 1) * (1 + 1000 * j)
        assert np.array_equal(out, exp), f"f64={f64}"
    # the 4x4x1 blocks of the short last row tile (float32)
    out = np.asarray(F.mfma_layout(False, tail=True), dtype=np.float64)
    exp = np.array([(e + 1 + 16 * (l // 4)) * (1 + 1000 * (l % 4)) for l in range(64) for e in range(4)], float)
    assert np.array_equal(out, exp), "4x4x1"


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_single_leaf_is_direct_sum(precision, tol):
    x, q, _ = W.uniform_cube(1500, 3)
    x[-4:] = x[:4]  # coincident bodies: their pair is skipped
    plan, phi, E = gpu_fmm(x, q, 4, 0.4, 4096, precision)
    st = plan.stats()
    assert st["ncell"] == 1 and st["n_p2p"] == 1 and st["n_m2l"] == 0
    pd, Ed = oracle.direct(x, q)
    assert rel(phi, pd) < tol and rel(E, Ed) < tol


def _compare_tree(plan, x, ncrit, theta):
    g = plan.export_tree()
    T = oracle.Tree(x, ncrit, theta)
    o = T.export()
    for k in ("keys", "perm", "level", "begin", "end", "parent", "child_begin", "nchild"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["ckey"], o["ckey"])
    assert np.array_equal(g["centers"].view(np.uint64), o["centers"].view(np.uint64))
    assert np.array_equal(g["m2l"], o["m2l"]), "m2l lists"
    assert np.array_equal(g["p2p"], o["p2p"]), "p2p lists"
    return T


@pytest.mark.parametrize("case", ["cube16k", "plummer", "sphere", "dups"])
def test_tree_and_lists_bit_exact(case):
    if case == "cube16k":
        x, q, _ = W.make_config("cube16k")
        ncrit, theta = 64, 0.4
    elif case == "sphere":
        x, _, _ = W.sphere_surface(40000, 7)
        ncrit, theta = 64, 0.4
    elif case == "plummer":
        x, _, _ = W.plummer(30000, 5)
        ncrit, theta = 32, 0.35
    else:
        x, _, _ = W.uniform_cube(5000, 6)
        x[2500:] = x[:2500]
        x[:100] = x[0]
        ncrit, theta = 16, 0.5
    plan = F.Plan(dev(x), F.Params(p=4, theta=theta, ncrit=ncrit, precision="fp64"))
    T = _compare_tree(plan, x, ncrit, theta)
    st = plan.stats()
    assert (st["ncell"], st["nleaf"], st["depth"]) == (T.ncell, T.nleaf, T.depth)
    assert (st["n_m2l"], st["n_p2p"]) == (T.n_m2l, T.n_p2p)
    # body pairs of the P2P list: counted on request only, then reported by stats
    assert st["p2p_body_pairs"] == -1
    o = T.export()
    size = (o["end"] - o["begin"]).astype(np.int64)
    want = int(np.sum(size[o["p2p"][:, 0]] * size[o["p2p"][:, 1]]))
    assert plan.body_pairs() == want
    assert plan.stats()["p2p_body_pairs"] == want


def test_float32_coordinates_widen_exactly():
    x, _, _ = W.plummer(8000, 9)
    x32 = x.astype(np.float32)
    plan = F.Plan(dev(x32, torch.float32), F.Params(p=4, theta=0.4, ncrit=24, precision="mixed"))
    _compare_tree(plan, x32.astype(np.float64), 24, 0.4)


@pytest.mark.parametrize("case", ["cube16k", "plummer", "sphere"])
def test_fmm_matches_oracle(case):
    if case == "cube16k":
        x, q, _ = W.make_config("cube16k")
        p, theta, ncrit = 4, 0.4, 64
    elif case == "sphere":
        x, q, _ = W.sphere_surface(40000, 8)
        p, theta, ncrit = 10, 0.4, 128
    else:
        x, _, _ = W.plummer(40000, 2)
        q = np.random.default_rng(3).uniform(-1, 1, 40000)
        p, theta, ncrit = 6, 0.35, 32
    T = oracle.Tree(x, ncrit, theta)
    po, Eo = T.fmm(q, p)
    plan, p64, E64 = gpu_fmm(x, q, p, theta, ncrit, "fp64")
    e64 = (rel(p64, po), rel(E64, Eo))
    assert e64[0] < 1e-6 and e64[1] < 1e-6
    assert e64[0] < 1e-11 and e64[1] < 1e-11, e64  # roundoff only
    if case == "plummer":
        # both pair-list paths run: shared-operator tiles and the generic kernel
        st = plan.stats()
        assert 0 < st["m2l_cross_batched"] < st["n_m2l_cross"] + st["n_m2l_sparse"], st
    _, pm, Em = gpu_fmm(x, q, p, theta, ncrit, "mixed")
    em = (rel(pm, po), rel(Em, Eo))
    assert em[0] < 1e-4 and em[1] < 1e-4, em
    if case == "cube16k":
        # and against the plain definition: the direct sum, all targets
        pd, Ed = oracle.direct(x, q)
        assert rel(p64, pd) < 1e-3 and rel(E64, Ed) < 1e-3


@pytest.mark.parametrize("p", list(range(1, 17)))
def test_orders_and_padding(p):
    # every order the batched M2L is instantiated for: row tiles of 16
    # coefficients, input steps with (p = 5, 6, 7, 9, 10) and without padding
    x, q, _ = W.uniform_cube(9000, 20 + p)
    T = oracle.Tree(x, 40, 0.45)
    po, Eo = T.fmm(q, p)
    _, p64, E64 = gpu_fmm(x, q, p, 0.45, 40, "fp64")
    assert rel(p64, po) < 1e-11 and rel(E64, Eo) < 1e-11
    _, pm, Em = gpu_fmm(x, q, p, 0.45, 40, "mixed")
    assert rel(pm, po) < 1e-4 and rel(Em, Eo) < 1e-4


@pytest.mark.parametrize("p", [6, 7, 9, 10])
def test_short_last_tile(p):
    # p = 6, 7, 9, 10: in float32 the last row tile holds at most 4
    # coefficient rows and runs on 4x4x1 blocks (same-level and pair-list
    # products).  Those rows are top-degree coefficients, which matter only
    # when the acceptance parameter is large: at theta = 0.9 the oracle's
    # p - 1 and p results differ by 1.5e-3 (p = 6) down to 5e-5 (p = 10),
    # while the mixed path's own rounding is 1e-7 to 6e-7 (measured), so the
    # bar of 2e-6 leaves the top-degree rows no room to be wrong
    x, _, _ = W.uniform_cube(20000, 66)
    q = np.random.default_rng(86).uniform(-1.0, 1.0, 20000)
    T = oracle.Tree(x, 32, 0.9)
    po, Eo = T.fmm(q, p)
    _, pm, Em = gpu_fmm(x, q, p, 0.9, 32, "mixed")
    assert rel(pm, po) < 2e-6 and rel(Em, Eo) < 2e-6, (p, rel(pm, po), rel(Em, Eo))


@pytest.mark.parametrize("p,n,ncrit,theta", [(4, 60000, 24, 0.35), (10, 12000, 8, 0.45)])
def test_cross_level_pairs_plummer(p, n, ncrit, theta):
    # adaptive trees with many leaf-against-finer-cell pairs, at a tile width
    # of 128 (p = 4) and 64 (p = 10) pairs
    x, _, _ = W.plummer(n, 13)
    q = np.random.default_rng(14).uniform(0.0, 1.0, n)
    T = oracle.Tree(x, ncrit, theta)
    po, Eo = T.fmm(q, p)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        plan, ph, Eh = gpu_fmm(x, q, p, theta, ncrit, precision)
        st = plan.stats()
        assert st["m2l_cross_batched"] > 0.5 * st["n_m2l_cross"], st
        assert rel(ph, po) < tol and rel(Eh, Eo) < tol, (precision, rel(ph, po), rel(Eh, Eo))


@pytest.mark.parametrize("p,n,ncrit,theta", [(6, 60000, 16, 0.35), (4, 40000, 24, 0.4)])
def test_sparse_rows_run_as_pairs(p, n, ncrit, theta):
    # same-level tile rows with few sources move to the pair list: the lists
    # (as sets) and the values stay those of the oracle for every threshold,
    # at a tile width of 64 (p = 6) and 128 (p = 4)
    x, _, _ = W.plummer(n, 31)
    q = np.random.default_rng(32).uniform(-1.0, 1.0, n)
    T = oracle.Tree(x, ncrit, theta)
    o = T.export()
    po, Eo = T.fmm(q, p)
    moved, rows, vals = [], [], []
    for thr in (0, 24, 64):
        plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision="fp64", m2l_sparse=thr))
        st = plan.stats()
        assert (st["n_m2l_same"], st["n_m2l_cross"]) == (T.n_m2l - st["n_m2l_cross"], st["n_m2l_cross"])
        assert st["n_m2l"] == T.n_m2l and plan.list_digest() == (T.digest_m2l, T.digest_p2p)
        assert np.array_equal(plan.export_tree()["m2l"], o["m2l"]), thr
        assert st["m2l_cross_batched"] <= st["n_m2l_cross"] + st["n_m2l_sparse"]
        moved.append(st["n_m2l_sparse"])
        rows.append(st["m2l_rows"])
        phi, E = plan.evaluate(dev(q))
        vals.append((host(phi), host(E)))
        assert rel(vals[-1][0], po) < 1e-11 and rel(vals[-1][1], Eo) < 1e-11, thr
        plan.close()
        plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision="mixed", m2l_sparse=thr))
        phi, E = plan.evaluate(dev(q))
        assert rel(host(phi), po) < 1e-4 and rel(host(E), Eo) < 1e-4, thr
        plan.close()
    assert moved[0] == 0 and 0 < moved[1] < moved[2] < T.n_m2l
    assert rows[0] > rows[1] > rows[2]
    # only the grouping of the sums differs
    assert rel(vals[1][0], vals[0][0]) < 1e-13 and rel(vals[2][1], vals[0][1]) < 1e-13


def test_nearly_coincident_bodies_keep_their_field():
    # pairs 1e-7 apart inside leaves about 0.06 wide: with float32 offsets from
    # the leaf center alone their separation would carry a 1e-2 error, and
    # these few bodies dominate the L2 norm of E; the own-leaf pass uses
    # compensated coordinates, so all bodies stay within the 1e-4 bar
    x, q, _ = W.uniform_cube(20000, 21)
    d = np.random.default_rng(22).normal(size=(10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x[1:20:2] = x[0:20:2] + 1e-7 * d
    T = oracle.Tree(x, 64, 0.4)
    po, Eo = T.fmm(q, 6)
    _, pm, Em = gpu_fmm(x, q, 6, 0.4, 64, "mixed")
    assert rel(pm, po) < 1e-4 and rel(Em, Eo) < 1e-4, (rel(pm, po), rel(Em, Eo))
    near = np.arange(20)
    assert rel(Em[near], Eo[near]) < 1e-4


def test_many_tiles_plummer():
    # at least 1024 same-level tiles: every stencil chunk runs in a launch of
    # its own and adds straight to the local expansions
    x, q, _ = W.plummer(400_000, 11)
    p, theta, ncrit = 10, 0.35, 8
    tg = W.sample_targets(x.shape[0], 256)
    T = oracle.Tree(x, ncrit, theta, targets=tg)
    po, Eo = T.fmm(q, p, targets=tg)
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision))
        st = plan.stats()
        assert st["m2l_slots"] // (st["m2l_stencil"] * 64) >= 1024  # tiles of 64 targets at p = 10
        assert (st["n_m2l"], st["n_p2p"]) == (T.n_m2l, T.n_p2p)
        assert plan.list_digest() == (T.digest_m2l, T.digest_p2p)
        phi, E = plan.evaluate(dev(q))
        assert rel(host(phi)[tg], po) < tol and rel(host(E)[tg], Eo) < tol, precision
        plan.close()


def test_p2p_long_lists_split_over_work_items():
    # small leaves and a tight acceptance criterion: coarse halo leaves of a
    # Plummer tree carry P2P lists of (nearly) every leaf, which are cut into
    # several work items whose partial sums are reduced in order
    x, _, _ = W.plummer(50000, 21)
    q = np.random.default_rng(22).uniform(0.0, 1.0, 50000)
    T = oracle.Tree(x, 6, 0.3)
    po, Eo = T.fmm(q, 3)
    outs = []
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        plan, ph, Eh = gpu_fmm(x, q, 3, 0.3, 6, precision)
        assert plan.stats()["p2p_cut_leaves"] > 0
        assert rel(ph, po) < tol and rel(Eh, Eo) < tol, (precision, rel(ph, po), rel(Eh, Eo))
        outs.append((ph, Eh))
    plan, ph, Eh = gpu_fmm(x, q, 3, 0.3, 6, "mixed")
    assert ph.tobytes() == outs[1][0].tobytes() and Eh.tobytes() == outs[1][1].tobytes()


def test_coarse_fp64_levels_variants():
    x, _, _ = W.plummer(20000, 4)
    q = np.random.default_rng(1).uniform(-1, 1, 20000)
    T = oracle.Tree(x, 16, 0.4)
    po, Eo = T.fmm(q, 6)
    for cfl in (0, 1, 3, 30 - 8):
        plan = F.Plan(dev(x), F.Params(p=6, theta=0.4, ncrit=16, precision="mixed", coarse_fp64_levels=cfl))
        phi, E = plan.evaluate(dev(q))
        assert rel(host(phi), po) < 1e-4 and rel(host(E), Eo) < 1e-4, cfl


def test_adjoint_matches_oracle_composition():
    x, q, rng = W.uniform_cube(12000, 7)
    w = W.adjoint_weights(rng, 12000)
    p, theta, ncrit = 5, 0.4, 32
    T = oracle.Tree(x, ncrit, theta)
    _, Eq = T.fmm(q, p)
    pw, Ew = T.fmm(w, p)
    dq_ref = pw
    dx_ref = -(w[:, None] * Eq + q[:, None] * Ew)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-4)):
        plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision))
        dq, dx = plan.adjoint(dev(q), dev(w))          # recompute E^q
        assert rel(host(dq), dq_ref) < tol and rel(host(dx), dx_ref) < tol, precision
        _, E = plan.evaluate(dev(q))
        dq2, dx2 = plan.adjoint(dev(q), dev(w), E)     # reuse E^q
        assert rel(host(dq2), dq_ref) < tol and rel(host(dx2), dx_ref) < tol, precision


def test_autograd_function():
    x, q, rng = W.uniform_cube(6000, 8)
    w = W.adjoint_weights(rng, 6000)
    for recompute in (False, True):
        prm = F.Params(p=5, theta=0.4, ncrit=32, precision="fp64")
        prm.recompute = recompute
        xt = dev(x).requires_grad_(True)
        qt = dev(q).requires_grad_(True)
        phi, E = F.FMMFunction.apply(xt, qt, prm)
        L = (dev(w) * phi).sum()
        L.backward()
        T = oracle.Tree(x, 32, 0.4)
        _, Eq = T.fmm(q, 5)
        pw, Ew = T.fmm(w, 5)
        assert rel(host(qt.grad), pw) < 1e-11
        assert rel(host(xt.grad), -(w[:, None] * Eq + q[:, None] * Ew)) < 1e-11


def test_one_body_leaves():
    # N_crit = 1: every leaf holds one body (or coincident ones), the deepest
    # trees and the most cross-level pairs a distribution gives
    x, _, _ = W.plummer(3000, 14)
    q = np.random.default_rng(15).uniform(-1, 1, 3000)
    x[2990:] = x[:10]  # coincident bodies end in shared leaves at level 21
    T = oracle.Tree(x, 1, 0.4)
    po, Eo = T.fmm(q, 5)
    plan, p64, E64 = gpu_fmm(x, q, 5, 0.4, 1, "fp64")
    st = plan.stats()
    assert (st["ncell"], st["depth"], st["n_m2l"], st["n_p2p"]) == (T.ncell, T.depth, T.n_m2l, T.n_p2p)
    assert plan.list_digest() == (T.digest_m2l, T.digest_p2p)
    assert rel(p64, po) < 1e-11 and rel(E64, Eo) < 1e-11
    _, pm, Em = gpu_fmm(x, q, 5, 0.4, 1, "mixed")
    assert rel(pm, po) < 1e-4 and rel(Em, Eo) < 1e-4


def test_deterministic_bits():
    x, _, _ = W.plummer(30000, 11)
    q = np.random.default_rng(0).uniform(-1, 1, 30000)
    outs = []
    for _ in range(2):
        plan, phi, E = gpu_fmm(x, q, 6, 0.4, 32, "mixed")
        outs.append((phi.tobytes(), E.tobytes()))
    assert outs[0] == outs[1]


def test_error_paths():
    x, q, _ = W.uniform_cube(100, 1)
    bad = [dict(p=0), dict(p=17), dict(theta=0.0), dict(theta=1.0), dict(ncrit=0)]
    for kw in bad:
        prm = F.Params(**{**dict(p=4, theta=0.4, ncrit=8), **kw})
        with pytest.raises(F.FMMError) as ei:
            F.Plan(dev(x), prm)
        assert ei.value.code == 1
    xn = x.copy()
    xn[17, 1] = np.nan
    with pytest.raises(F.FMMError) as ei:
        F.Plan(dev(xn), F.Params(p=4))
    assert ei.value.code == 5
    xi = x.copy()
    xi[3, 0] = np.inf
    with pytest.raises(F.FMMError) as ei:
        F.Plan(dev(xi), F.Params(p=4))
    assert ei.value.code == 5
    # empty input is a valid no-op
    plan = F.Plan(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"), F.Params(p=4))
    phi, E = plan.evaluate(torch.zeros(0, dtype=torch.float64, device="cuda:0"))
    assert phi.numel() == 0
    # one body
    plan, phi, E = gpu_fmm(x[:1], q[:1], 4, 0.4, 8, "mixed")
    assert phi[0] == 0.0 and np.all(E == 0.0)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_float32_caller_dtype(precision, tol):
    # float32 coordinates, charges and weights: the outputs come back in
    # float32 and are checked against the oracle on the widened inputs
    x, q, rng = W.plummer(20000, 31, charges="unit")
    w = W.adjoint_weights(rng, 20000)
    x32, q32, w32 = (a.astype(np.float32) for a in (x, q, w))
    xw, qw, ww = (a.astype(np.float64) for a in (x32, q32, w32))
    p, theta, ncrit = 6, 0.4, 24
    T = oracle.Tree(xw, ncrit, theta)
    po, Eo = T.fmm(qw, p)
    pw, Ew = T.fmm(ww, p)
    dx_ref = -(ww[:, None] * Eo + qw[:, None] * Ew)
    plan = F.Plan(dev(x32, torch.float32), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision))
    qt, wt = dev(q32, torch.float32), dev(w32, torch.float32)
    phi, E = plan.evaluate(qt)
    assert phi.dtype == torch.float32 and E.dtype == torch.float32
    assert rel(host(phi), po) < tol and rel(host(E), Eo) < tol
    for field_q in (E, None):
        dq, dx = plan.adjoint(qt, wt, field_q)
        assert dq.dtype == torch.float32 and dx.dtype == torch.float32
        assert rel(host(dq), pw) < tol and rel(host(dx), dx_ref) < tol, (precision, field_q is None)
    plan.close()


@pytest.mark.parametrize("case", ["flat", "line"])
def test_degenerate_boxes(case):
    # all bodies on a plane, or on a line with a graded spacing: the root cube
    # is set by one or two axes, the others keep a single lattice coordinate
    rng = np.random.default_rng(41)
    if case == "flat":
        x = rng.random((12000, 3))
        x[:, 2] = 0.5
        ncrit = 16
    else:
        x = np.zeros((3000, 3))
        x[:, 0] = np.linspace(0.0, 1.0, 3000) ** 3
        x[:, 1] = 0.25
        ncrit = 8
    q = rng.uniform(-1.0, 1.0, x.shape[0])
    theta, p = 0.4, 6
    plan = F.Plan(dev(x), F.Params(p=p, theta=theta, ncrit=ncrit, precision="fp64"))
    T = _compare_tree(plan, x, ncrit, theta)
    po, Eo = T.fmm(q, p)
    phi, E = plan.evaluate(dev(q))
    assert rel(host(phi), po) < 1e-11 and rel(host(E), Eo) < 1e-11
    plan.close()
    _, pm, Em = gpu_fmm(x, q, p, theta, ncrit, "mixed")
    assert rel(pm, po) < 1e-4 and rel(Em, Eo) < 1e-4


def test_close_pairs_across_leaf_faces():
    # pairs 1e-7 apart straddling the faces between leaves: their fields
    # dominate every norm, and the float32 shift between the two leaf centers
    # alone would carry an error of order 1e-9; the touching-leaf pass of P2P
    # uses compensated offsets, so every body stays within the bar
    x, q, _ = W.uniform_cube(20000, 43)
    lo = x.min(0)
    S = float((x.max(0) - lo).max())
    rng = np.random.default_rng(44)
    # bodies that fix no side of the root cube, so moving them keeps it
    extremal = np.concatenate([x.argmin(0), x.argmax(0)])
    idx = np.setdiff1d(np.arange(60), extremal)[:40]
    for k in range(20):
        a, b = idx[2 * k], idx[2 * k + 1]
        axis = k % 3
        face = lo[axis] + (1 + k % 7) * S / 8.0  # a leaf face of the level-3 tree
        x[a] = x[b] = rng.uniform(0.05, 0.95, 3)
        x[a, axis] = face - 5e-8
        x[b, axis] = face + 5e-8
    assert np.array_equal(x.min(0), lo) and float((x.max(0) - lo).max()) == S
    T = oracle.Tree(x, 64, 0.4)
    e = T.export()
    leaf_of = np.empty(x.shape[0], np.int64)
    for c in np.nonzero(e["nchild"] == 0)[0]:
        leaf_of[e["perm"][e["begin"][c]:e["end"][c]]] = c
    assert np.all(leaf_of[idx[0::2]] != leaf_of[idx[1::2]])  # every pair straddles a face
    po, Eo = T.fmm(q, 6)
    _, p64, E64 = gpu_fmm(x, q, 6, 0.4, 64, "fp64")
    _, pm, Em = gpu_fmm(x, q, 6, 0.4, 64, "mixed")
    assert rel(p64, po) < 1e-11 and rel(E64, Eo) < 1e-11
    assert rel(pm, p64) < 1e-4 and rel(Em, E64) < 1e-4, (rel(pm, p64), rel(Em, E64))
    assert rel(Em[idx], E64[idx]) < 1e-4


def test_allocation_failure_reports_nomem_and_releases_everything():
    # a plan allocator that fails on its k-th call: the build reports
    # FMM_ERR_NOMEM and hands back every block it had obtained
    x, q, _ = W.plummer(30000, 45)
    prm = F.Params(p=6, theta=0.4, ncrit=16, precision="mixed")
    live = {}

    def counting(fail_at):
        calls = [0]

        def alloc(nbytes, stream):
            calls[0] += 1
            if calls[0] == fail_at:
                return None
            ptr = torch.cuda.caching_allocator_alloc(nbytes)
            live[ptr] = nbytes
            return ptr

        def free(ptr, stream):
            live.pop(ptr)
            torch.cuda.caching_allocator_delete(ptr)

        return F.CallbackAllocator(alloc, free), calls

    xt, qt = dev(x), dev(q)
    al, calls = counting(0)  # never fails: count the calls of a good build
    plan = F.Plan(xt, prm, allocator=al)
    n_build = calls[0]
    phi, E = plan.evaluate(qt)
    plan.close()
    assert not live and n_build > 10
    for k in sorted({1, 2, 5, n_build // 3, n_build // 2, n_build - 1, n_build}):
        al, calls = counting(k)
        with pytest.raises(F.FMMError) as ei:
            F.Plan(xt, prm, allocator=al)
        assert ei.value.code == 2, (k, ei.value)
        torch.cuda.synchronize()
        assert not live, (k, len(live))
    # a failure in the adjoint's first call (its second right-hand side)
    # leaves the plan usable
    al, calls = counting(n_build + 1)
    plan = F.Plan(xt, prm, allocator=al)
    with pytest.raises(F.FMMError) as ei:
        plan.adjoint(qt, qt, E)
    assert ei.value.code == 2
    phi2, _ = plan.evaluate(qt)
    assert torch.equal(phi2, phi)
    plan.close()
    torch.cuda.synchronize()
    assert not live


def test_binding_checks_shapes_and_outputs():
    x, q, _ = W.uniform_cube(500, 46)
    with pytest.raises(ValueError):
        F.evaluate(dev(x[:, :2]), dev(q))
    plan = F.Plan(dev(x), F.Params(p=4))
    with pytest.raises(ValueError):
        plan.evaluate(dev(q[:-1]))
    with pytest.raises(TypeError):
        plan.evaluate(dev(q), out=(torch.empty(500, dtype=torch.float32, device="cuda:0"), None))
    with pytest.raises(ValueError):
        plan.evaluate(dev(q), out=(torch.empty(500, dtype=torch.float64, device="cuda:0"),
                                   torch.empty((500, 2), dtype=torch.float64, device="cuda:0")))
    with pytest.raises(ValueError):
        strided = torch.empty((500, 2), dtype=torch.float64, device="cuda:0")[:, 0]
        plan.evaluate(dev(q), out=(strided, None))
    phi = torch.empty(500, dtype=torch.float64, device="cuda:0")
    E = torch.empty((500, 3), dtype=torch.float64, device="cuda:0")
    p1, e1 = plan.evaluate(dev(q), out=(phi, E))
    assert p1.data_ptr() == phi.data_ptr() and e1.data_ptr() == E.data_ptr()
    plan.close()
    # a second backward without recomputation has no plan left
    xt = dev(x).requires_grad_(True)
    phi, E = F.FMMFunction.apply(xt, dev(q), F.Params(p=4))
    L = phi.sum()
    L.backward(retain_graph=True)
    with pytest.raises(RuntimeError):
        L.backward()
