"""GPU parity at the full workload sizes, in the configuration the benchmark
times (plan built on torch's allocator, one evaluate, mixed and FP64 paths).

* cube1m     N = 2^20 uniform, P = 8, theta = 0.4, N_crit = 64
* plummer4m  N = 2^22 Plummer, P = 10, theta = 0.35, N_crit = 32
* cube1m_adjoint: the adjoint of L = sum w phi at 2^20
* plummer16m N = 2^24 Plummer, P = 12, theta = 0.3, N_crit = 64
* sphere4m   N = 2^22 on the unit sphere's surface, P = 10, theta = 0.4, N_crit = 512

The oracle cannot evaluate every body at these sizes, so potentials and fields
are compared on sampled targets (the oracle's target-subset mode gives exactly
the full oracle's values there), and the lists through their order-free
digests and counts.  Tolerances: 1e-4 relative L2 for the mixed path and 1e-6
for FP64 (in practice ~1e-14); the FMM's own truncation error is reported
against the direct sum on the same targets.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1405_7487_amd as F
from paper_1405_7487_amd import workloads as W

from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _plan(x, cfg, precision):
    prm = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision=precision)
    return F.Plan(x, prm)


def _check_tree(plan, T):
    st = plan.stats()
    assert (st["ncell"], st["nleaf"], st["depth"]) == (T.ncell, T.nleaf, T.depth)
    assert st["n_m2l"] == T.n_m2l and st["n_p2p"] == T.n_p2p
    assert plan.list_digest() == (T.digest_m2l, T.digest_p2p)
    return st


@pytest.mark.parametrize("name,ntarget", [("cube1m", 512), ("plummer4m", 96), ("sphere4m", 96)])
def test_full_size_parity(name, ntarget):
    cfg = W.CONFIGS[name]
    x_np, q_np, _ = W.make_config(name)
    n = x_np.shape[0]
    tg = W.sample_targets(n, ntarget)
    say(f"[{name}] oracle: full traversal (counts, digests) + FMM at {tg.size} targets")
    T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tg)
    po, Eo = T.fmm(q_np, cfg["p"], targets=tg)
    pd, Ed = oracle.direct(x_np, q_np, targets=tg)
    say(f"[{name}] oracle vs direct: phi {rel(po, pd):.3e} E {rel(Eo, Ed):.3e}")
    x, q = dev(x_np), dev(q_np)
    full = {}
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        say(f"[{name}] GPU {precision}")
        plan = _plan(x, cfg, precision)
        phi, E = plan.evaluate(q)
        torch.cuda.synchronize()
        _check_tree(plan, T)
        full[precision] = (host(phi), host(E))
        phi_h, E_h = full[precision][0][tg], full[precision][1][tg]
        ep, eE = rel(phi_h, po), rel(E_h, Eo)
        say(f"[{name}] {precision}: vs oracle phi {ep:.3e} E {eE:.3e}; vs direct phi {rel(phi_h, pd):.3e}")
        assert ep < tol and eE < tol, (precision, ep, eE)
        plan.close()
    # every body: the mixed path against the FP64 path (itself ~1e-15 from the oracle)
    ap = rel(full["mixed"][0], full["fp64"][0])
    aE = rel(full["mixed"][1], full["fp64"][1])
    say(f"[{name}] mixed vs fp64 GPU, all {n} bodies: phi {ap:.3e} E {aE:.3e}")
    assert ap < 1e-4 and aE < 1e-4


def test_full_size_tree_bit_exact_plummer4m():
    cfg = W.CONFIGS["plummer4m"]
    x_np, _, _ = W.make_config("plummer4m")
    T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], count_only=True)
    o = T.export()
    plan = _plan(dev(x_np), cfg, "mixed")
    g = plan.export_tree(lists=False)
    for k in ("keys", "perm", "level", "begin", "end", "parent", "child_begin", "nchild", "ckey"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["centers"].view(np.uint64), o["centers"].view(np.uint64))
    _check_tree(plan, T)
    plan.close()


def _direct_gradient(x, q, w, idx):
    """dL/dq and dL/dx of L = sum_i w_i phi_i by the direct sum at bodies idx:
    dL/dq_k = phi^w_k, dL/dx_k = -(w_k E^q_k + q_k E^w_k)."""
    _, Eq = oracle.direct(x, q, targets=idx)
    pw, Ew = oracle.direct(x, w, targets=idx)
    return pw, -(w[idx, None] * Eq + q[idx, None] * Ew)


def test_adjoint_against_direct_gradient_and_finite_differences():
    name = "cube1m_adjoint"
    cfg = W.CONFIGS[name]
    x_np, q_np, rng = W.make_config(name)
    n = x_np.shape[0]
    w_np = W.adjoint_weights(rng, n)
    idx_fd, ax_fd = W.fd_coordinates(n)
    tg = W.sample_targets(n, 4096)
    # reference gradient by the direct sum
    dq_ref, dx_ref = _direct_gradient(x_np, q_np, w_np, tg)
    dq_fd_ref, dx_fd_ref = _direct_gradient(x_np, q_np, w_np, idx_fd)
    g_direct = dx_fd_ref[np.arange(idx_fd.size), ax_fd]
    # central differences of L on the direct sum (only terms with body k change)
    h = 1e-4
    g_fd = np.empty(idx_fd.size)
    bound = np.empty(idx_fd.size)
    for s, (k, a) in enumerate(zip(idx_fd, ax_fd)):
        others = np.arange(n) != k
        c = w_np[k] * q_np[others] + w_np[others] * q_np[k]

        def lk(xk):
            r = np.sqrt(((x_np[others] - xk) ** 2).sum(axis=1))
            return float(np.sum(c / r)), r

        xp, xm = x_np[k].copy(), x_np[k].copy()
        xp[a] += h
        xm[a] -= h
        lp, r = lk(xp)
        lm, _ = lk(xm)
        g_fd[s] = (lp - lm) / (2 * h)
        r0 = np.sqrt(((x_np[others] - x_np[k]) ** 2).sum(axis=1))
        # |third derivative of 1/r| <= 6/r^4 on the segment, plus rounding of the two sums
        bound[s] = h * h * np.sum(np.abs(c) / (r0 - h) ** 4) + 8e-16 * np.sum(np.abs(c) / (r0 - h)) / h
    assert np.all(np.abs(g_fd - g_direct) <= bound), np.max(np.abs(g_fd - g_direct) / bound)
    say(f"[adjoint] finite differences vs direct gradient: max |diff| {np.max(np.abs(g_fd - g_direct)):.3e}")

    # GPU adjoint (mixed path), forward field reused, then recomputed
    x, q, w = dev(x_np), dev(q_np), dev(w_np)
    plan = _plan(x, cfg, "mixed")
    phi, E = plan.evaluate(q)
    for field_q in (E, None):
        dq, dx = plan.adjoint(q, w, field_q)
        torch.cuda.synchronize()
        dq_h, dx_h = host(dq), host(dx)
        e_dq = rel(dq_h[tg], dq_ref)
        e_dx = rel(np.concatenate([dx_h[tg].ravel(), dx_h[idx_fd, ax_fd]]),
                   np.concatenate([dx_ref.ravel(), g_direct]))
        e_fd = rel(dx_h[idx_fd, ax_fd], g_fd)
        say(f"[adjoint] field_q={'given' if field_q is not None else 'recomputed'}: "
            f"dq {e_dq:.3e} dx {e_dx:.3e} dx vs FD {e_fd:.3e}")
        assert e_dq < 1e-4 and e_dx < 1e-4
        # per coordinate against the central differences: their own error
        # (within the bound checked above) plus 1e-4 of the gradient (with a
        # floor at 1e-4 of the coordinates' RMS gradient for near-zero entries)
        g_gpu = dx_h[idx_fd, ax_fd]
        allow = bound + 1e-4 * np.maximum(np.abs(g_direct), np.sqrt(np.mean(g_direct ** 2)))
        worst = np.max(np.abs(g_gpu - g_fd) / allow)
        say(f"[adjoint] per-coordinate |g_GPU - g_FD| / allowance: max {worst:.3f}")
        assert np.all(np.abs(g_gpu - g_fd) <= allow)
    plan.close()


def test_plummer16m_tree_and_lists_bit_exact():
    # the largest workload: counts against the independent level-by-level
    # count, keys, permutation, cells and centers bit for bit, and both lists
    # through their counts and digests, against the oracle's full walk
    from test_oracle_tree import level_counts

    name = "plummer16m"
    cfg = W.CONFIGS[name]
    x_np, _, _ = W.make_config(name)
    say(f"[{name}] oracle: tree and full traversal (counts, digests)")
    T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], count_only=True)
    assert (T.ncell, T.nleaf, T.depth) == level_counts(x_np, cfg["ncrit"])
    say(f"[{name}] {T.ncell} cells, {T.nleaf} leaves, depth {T.depth}; M2L {T.n_m2l}, P2P {T.n_p2p}")
    o = T.export()
    say(f"[{name}] GPU build")
    plan = _plan(dev(x_np), cfg, "mixed")
    g = plan.export_tree(lists=False)
    for k in ("keys", "perm", "level", "begin", "end", "parent", "child_begin", "nchild", "ckey"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["centers"].view(np.uint64), o["centers"].view(np.uint64))
    _check_tree(plan, T)
    plan.close()


def test_plummer16m_forward_and_recomputed_adjoint():
    name = "plummer16m"
    cfg = W.CONFIGS[name]
    x_np, q_np, rng = W.make_config(name)
    n = x_np.shape[0]
    w_np = W.adjoint_weights(rng, n)
    tg = W.sample_targets(n, 4096)
    tgo = tg[:32]
    say(f"[{name}] oracle at {tgo.size} targets (pruned walk, which keeps exactly the full walk's pairs "
        f"for these targets)")
    T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tgo, prune=True)
    po, Eo = T.fmm(q_np, cfg["p"], targets=tgo)
    del T
    x, q, w = dev(x_np), dev(q_np), dev(w_np)
    del x_np
    prm64 = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision="fp64")
    prm = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision="mixed")
    prm.recompute = True  # the plan is freed after the forward pass and rebuilt in the backward
    say(f"[{name}] GPU fp64 forward + adjoint")
    p64 = F.Plan(x, prm64)
    phi64, E64 = p64.evaluate(q)
    dq64, dx64 = p64.adjoint(q, w, E64)
    torch.cuda.synchronize()
    phi64_h, E64_h = host(phi64), host(E64)
    dq64_h, dx64_h = host(dq64)[tg], host(dx64)[tg]
    p64.close()
    del phi64, E64, dq64, dx64
    assert rel(phi64_h[tgo], po) < 1e-6 and rel(E64_h[tgo], Eo) < 1e-6
    say(f"[{name}] GPU mixed forward, plan freed, adjoint recomputes its expansions")
    torch.cuda.reset_peak_memory_stats()
    xr = x.clone().requires_grad_(True)
    qr = q.clone().requires_grad_(True)
    phi, E = F.FMMFunction.apply(xr, qr, prm)
    phi_h, E_h = host(phi), host(E)
    L = (phi * w).sum()
    L.backward()
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated()
    ep, eE = rel(phi_h[tg], phi64_h[tg]), rel(E_h[tg], E64_h[tg])
    eo_p, eo_E = rel(phi_h[tgo], po), rel(E_h[tgo], Eo)
    e_dq, e_dx = rel(host(qr.grad)[tg], dq64_h), rel(host(xr.grad)[tg], dx64_h)
    say(f"[{name}] mixed vs fp64 GPU: phi {ep:.3e} E {eE:.3e}; vs oracle phi {eo_p:.3e} E {eo_E:.3e}; "
        f"adjoint dq {e_dq:.3e} dx {e_dx:.3e}; peak torch memory {peak / 2**30:.2f} GiB")
    assert max(ep, eE, eo_p, eo_E, e_dq, e_dx) < 1e-4
