#!/usr/bin/env python
"""Benchmark of the per-rank FMM evaluation on one MI355X.

A step is one pass of the whole hot path over one synthetic body set already
resident in HBM: fmm_build (keys, sort, cells, traversal, lists), the forward
evaluation (P2M, M2M, M2L, L2L, L2P, P2P, unpermute) and the adjoint of
L = sum w phi.  `value` is the forward throughput N / T_forward in
particles/s (potential + field); the adjoint time is reported beside it.

Prints ONE JSON line.  The library evaluates one rank's share on one GPU;
multi-GPU runs are not supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "particles/s (potential+field) at ≤1e-4 rel L2, FP32/MFMA vs FP64 FMM; adjoint/fwd"
PEAK = {"mfma_f32": 157.3, "mfma_f64": 78.6, "valu_f32": 157.3, "valu_f64": 78.6, "hbm": 8000.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = {"k_m2l_batched": "m2l.hip", "k_p2p": "p2p.hip"}


def recorded_traffic(kernel, config, precision):
    """HBM bytes that `kernel` moves in one evaluation (all its launches), from
    the committed counter summary, or None when the kernel's source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", f"hbm_traffic_{config}.md")
    src = os.path.join(HERE, "paper_1405_7487_amd", "csrc", KERNEL_SOURCE[kernel])
    if not os.path.exists(path) or not os.path.exists(src):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        # | kernel | precision | source sha256 | FETCH KiB | WRITE KiB | bytes per launch |
        if len(cols) == 6 and cols[0] == kernel and cols[1] == precision and cols[2] == sha:
            return float(cols[5])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cube1m")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--cpu-sample", type=int, default=12000, help="oracle targets for cpu_baseline (0 = skip)")
    ap.add_argument("--fp64-steps", type=int, default=3, help="FP64 GPU forward runs for the speedup (0 = skip)")
    ap.add_argument("--pool", action="store_true", help="library caching pool instead of torch's allocator")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library evaluates one rank's share on one GPU; --gpus must be 1 "
              "(the multi-GPU LET exchange is out of scope)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1405_7487_amd as F
    from paper_1405_7487_amd import workloads as W

    F.load()
    cfg = W.CONFIGS[args.config]
    n = cfg["n"]
    x_np, q_np, rng = W.make_config(args.config)
    w_np = W.adjoint_weights(rng, n)
    dev = torch.device("cuda:0")
    x = torch.as_tensor(x_np, device=dev)
    q = torch.as_tensor(q_np, device=dev)
    w = torch.as_tensor(w_np, device=dev)
    prm = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision=args.precision)
    log(f"bench: {args.config} n={n} p={cfg['p']} theta={cfg['theta']} ncrit={cfg['ncrit']} {args.precision}")

    stream = torch.cuda.current_stream()

    def step(timed_events=None):
        plan = F.Plan(x, prm, timing=timed_events is not None, torch_allocator=not args.pool)
        if timed_events is not None:
            timed_events[1].record(stream)
        phi, E = plan.evaluate(q)
        if timed_events is not None:
            timed_events[2].record(stream)
        dq, dx = plan.adjoint(q, w, E)
        if timed_events is not None:
            timed_events[3].record(stream)
        return plan, phi, E, dq, dx

    for k in range(args.warmup):
        plan, *_ = step()
        torch.cuda.synchronize()
        plan.close()
        log(f"bench: warmup {k + 1}/{args.warmup} done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    fwd, adj, kern = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        plan, phi, E, dq, dx = step(evs[k])
        st = plan.stats()  # waits on this step's phase events
        kern.append(st)
        plan.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e in evs:
        fwd.append(e[0].elapsed_time(e[2]))
        adj.append(e[2].elapsed_time(e[3]))
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_fwd = float(np.median(fwd))
    t_adj = float(np.median(adj))
    log(f"bench: {args.steps} timed steps: forward {t_fwd:.3f} ms, adjoint {t_adj:.3f} ms, step {ms_step:.3f} ms")

    # evaluation alone on a reused plan; keep its outputs for the accuracy check
    plan = F.Plan(x, prm)
    ev_ms = []
    for k in range(max(3, min(args.steps, 10))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        phi, E = plan.evaluate(q)
        e1.record(stream)
        torch.cuda.synchronize()
        ev_ms.append(e0.elapsed_time(e1))
    t_eval = float(np.median(ev_ms))
    body_pairs = plan.body_pairs()
    stats = plan.stats()
    phi_h = phi.cpu().numpy()
    E_h = E.cpu().numpy()
    plan.close()

    # roofline of the dominant kernel (per-launch means over the timed steps)
    m2l_ms = float(np.mean([s["ms_m2l"] for s in kern]))
    p2p_ms = float(np.mean([s["ms_p2p"] for s in kern]))
    p2 = cfg["p"] ** 2
    m2l_flops = 2.0 * p2 * p2 * stats["n_m2l_same"]
    p2p_flops = 20.0 * body_pairs
    if m2l_ms >= p2p_ms:
        achieved = m2l_flops / (m2l_ms * 1e-3) / 1e12
        peak = PEAK["mfma_f32"] if args.precision == "mixed" else PEAK["mfma_f64"]
        # the phase is the chunk launches of k_m2l_batched (and their ordered
        # partial-sum reductions) of one evaluation, timed by events on its stream
        roof = {"kernel": "k_m2l_batched (same-level M2L, all chunk launches of one evaluation)", "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": recorded_traffic("k_m2l_batched", args.config, args.precision),
                "launch_ms": m2l_ms, "flops_per_launch": m2l_flops}
    else:
        achieved = p2p_flops / (p2p_ms * 1e-3) / 1e12
        peak = PEAK["valu_f32"] if args.precision == "mixed" else PEAK["valu_f64"]
        roof = {"kernel": "k_p2p", "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": recorded_traffic("k_p2p", args.config, args.precision),
                "launch_ms": p2p_ms, "flops_per_launch": p2p_flops}
    other = {"m2l_ms": m2l_ms, "m2l_tflops": m2l_flops / (m2l_ms * 1e-3) / 1e12 if m2l_ms else None,
             "p2p_ms": p2p_ms, "p2p_tflops": p2p_flops / (p2p_ms * 1e-3) / 1e12 if p2p_ms else None,
             "m2l_cross_ms": float(np.mean([s["ms_m2l_cross"] for s in kern])),
             "p2m_ms": float(np.mean([s["ms_p2m"] for s in kern])),
             "l2l_ms": float(np.mean([s["ms_l2l"] for s in kern])),
             "l2p_ms": float(np.mean([s["ms_l2p"] for s in kern])),
             "build_ms": float(np.mean([s["ms_build"] for s in kern])),
             "build_tree_ms": float(np.mean([s["ms_tree"] for s in kern])),
             "build_traverse_ms": float(np.mean([s["ms_traverse"] for s in kern])),
             "build_ops_ms": float(np.mean([s["ms_ops"] for s in kern]))}

    # FP64 GPU baseline (same build + forward)
    fp64_ms = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        prm64 = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision="fp64")
        times = []
        for k in range(args.fp64_steps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            p64 = F.Plan(x, prm64)
            phi64, E64 = p64.evaluate(q)
            e1.record(stream)
            torch.cuda.synchronize()
            if k > 0:
                times.append(e0.elapsed_time(e1))
            p64.close()
        fp64_ms = float(np.mean(times))
        phi64_h, E64_h = phi64.cpu().numpy(), E64.cpu().numpy()
        log(f"bench: fp64 forward {fp64_ms:.3f} ms")
    else:
        phi64_h = E64_h = None

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    err = {}
    if phi64_h is not None:
        err["vs_fp64_gpu_all"] = {"phi": rel(phi_h, phi64_h), "E": rel(E_h, E64_h)}

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        tg = W.sample_targets(n, args.cpu_sample)
        c0 = time.perf_counter()
        T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tg, prune=True)
        po, Eo = T.fmm(q_np, cfg["p"], targets=tg)
        c1 = time.perf_counter()
        err["vs_oracle_sampled"] = {"phi": rel(phi_h[tg], po), "E": rel(E_h[tg], Eo), "targets": int(tg.size)}
        if phi64_h is not None:
            err["fp64_gpu_vs_oracle_sampled"] = {"phi": rel(phi64_h[tg], po), "E": rel(E64_h[tg], Eo)}
        cpu = {"value": tg.size / (c1 - c0), "unit": "particles/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"FP64 oracle FMM (full tree build of all {n} bodies + target-subset evaluation) "
                         f"at {tg.size} sampled targets; {c1 - c0:.2f} s"}
        log(f"bench: oracle sample {tg.size} targets in {c1 - c0:.2f} s; err {err['vs_oracle_sampled']}")

    out = {
        "metric": METRIC,
        "value": n / (t_fwd * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: N={n} {cfg['dist']}, p={cfg['p']}, theta={cfg['theta']}, "
                               f"ncrit={cfg['ncrit']}, forward+adjoint", "n": n, "p": cfg["p"],
                   "theta": cfg["theta"], "ncrit": cfg["ncrit"], "precision": args.precision},
        "forward_ms": t_fwd,
        "forward_ms_mean": float(np.mean(fwd)),
        "evaluate_only_ms": t_eval,
        "adjoint_ms": t_adj,
        "adjoint_over_forward": t_adj / t_fwd,
        "fp64_forward_ms": fp64_ms,
        "speedup_vs_fp64": (fp64_ms / t_fwd) if fp64_ms else None,
        "err": err,
        "phases_ms": other,
        "counts": {k: stats[k] for k in ("ncell", "nleaf", "depth", "n_m2l", "n_m2l_same", "n_m2l_cross", "n_p2p",
                                         "p2p_body_pairs", "m2l_stencil", "m2l_offsets", "device_bytes")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
