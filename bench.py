#!/usr/bin/env python
"""Benchmark of the per-rank FMM evaluation on one MI355X.

A step is one pass of the whole hot path over one synthetic body set already
resident in HBM, as a differentiable caller runs it with expansion
recomputation (the sequence FMMFunction runs with params.recompute = True):

  forward  : fmm_build (keys, sort, cells, traversal, lists, operators) and
             fmm_evaluate_plan (P2M, M2M, M2L, L2L, L2P, P2P, unpermute) for
             potential and field; the plan is then released;
  backward : fmm_build again (same deterministic tree) and fmm_adjoint of
             L = sum w phi with the forward field kept, giving dL/dq, dL/dx.

`value` is the forward throughput N / T_forward in particles/s (potential +
field); the backward time, the FP64 GPU forward time, the memory high-water
mark, per-phase times and roofline fractions are reported beside it.  The
default workload is the largest single-GPU one: 2^24 Plummer bodies, P = 12,
theta = 0.3, N_crit = 64.

Prints ONE JSON line.  The library evaluates one rank's share on one GPU;
multi-GPU runs are not supported.  Exits with status 3 (after printing) when
the mixed path misses 1e-4 relative L2 against the oracle on the sampled
targets.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "particles/s (potential+field) at ≤1e-4 rel L2, FP32/MFMA vs FP64 FMM; adjoint/fwd"
# MI355X published peaks (TFLOP/s, GB/s).  All HIP code is built without
# packed FP32, so scalar FP32 vector code is capped at 78.6 TFLOP/s.
PEAK = {"mfma_f32": 157.3, "mfma_f64": 78.6, "valu_f32": 78.6, "valu_f64": 78.6, "hbm": 8000.0}
# oracle targets (accuracy reference and cpu_baseline sample) per workload
ORACLE_TARGETS = {"plummer16m": 32, "plummer4m": 128, "sphere4m": 256, "cube1m": 4096, "cube1m_adjoint": 4096,
                  "cube16k": 16384}


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
        # | kernel | precision | source sha256 | FETCH KiB | WRITE KiB | bytes per evaluation |
        if len(cols) == 6 and cols[0] == kernel and cols[1] == precision and cols[2] == sha:
            return float(cols[5])
    return None


def rotation_flops(p):
    """Flops of one M2L pair by rotation as the kernel computes it: per
    rotation two products of the degree-n coefficient vectors (complex) with
    the real (2n+1)^2 table (4 flops per entry), two rotations, and the axial
    translation (4 flops per (j, s, n) term)."""
    rot = sum(2 * 4 * (2 * n + 1) ** 2 for n in range(p))
    axial = sum(4 * (p - abs(s)) for j in range(p) for s in range(-j, j + 1))
    return 2 * rot + axial


def roofline_phases(cfg, stats, ph, n, precision, rotation=False):
    """T* = sum over phases of max(flops / peak, bytes / bandwidth), per phase
    and overall, with the algorithmic work of each phase (not what the
    implementation executes)."""
    p2 = cfg["p"] ** 2
    f32 = precision == "mixed"
    mm = PEAK["mfma_f32"] if f32 else PEAK["mfma_f64"]
    va = PEAK["valu_f32"] if f32 else PEAK["valu_f64"]
    bw = PEAK["hbm"] * 1e9
    ncell = stats["ncell"]
    work = {
        # tree build: x, q read (32 B), key (8 B), one sort read + write of
        # (key, index) (24 B), sorted body write (16 B)
        "build": (0.0, 1.0, 80.0 * n),
        # same-level pairs of sparse tile rows run with the cross-level pairs
        "m2l_same": (2.0 * p2 * p2 * (stats["n_m2l_same"] - stats["n_m2l_sparse"]), mm, 8.0 * p2 * ncell),
        "m2l_cross": (2.0 * p2 * p2 * (stats["n_m2l_cross"] + stats["n_m2l_sparse"]), mm, 0.0),
    }
    if rotation:  # every pair in the rotation kernel
        work["m2l_same"] = (0.0, mm, 0.0)
        work["m2l_cross"] = (rotation_flops(cfg["p"]) * stats["n_m2l"], PEAK["valu_f64"], 0.0)
    work |= {
        "p2p": (20.0 * stats["p2p_body_pairs"], va, 32.0 * n),
        "p2m": (5.0 * p2 * n, va, 16.0 * n),
        "l2l": (2.0 * p2 * p2 * ncell, va, 0.0),
        "l2p": (8.0 * p2 * n, va, 32.0 * n),
    }
    out, tstar = {}, 0.0
    for k, (fl, pk, by) in work.items():
        t = max(fl / (pk * 1e12), by / bw)
        tstar += t
        ms = ph.get(k)
        out[k] = {"tstar_ms": t * 1e3, "ms": ms, "frac": (t * 1e3 / ms) if ms else None}
    return out, tstar * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="plummer16m")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--oracle-targets", type=int, default=-1,
                    help="oracle targets for the accuracy check and cpu_baseline (-1: per workload, 0: skip)")
    ap.add_argument("--serial-targets", type=int, default=-1,
                    help="targets of the single-thread oracle run (-1: an eighth of the sample, 0: skip)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed FP64 GPU forward runs (0 = skip)")
    ap.add_argument("--pool", action="store_true", help="library caching pool instead of torch's allocator")
    ap.add_argument("--m2l-sparse", type=int, default=-1,
                    help="same-level tile rows with fewer sources per 64 targets run pair by pair "
                         "(0: never; -1: the library's automatic choice)")
    ap.add_argument("--m2l-rotation", action="store_true",
                    help="every M2L pair by rotation (O(p^3) per pair, float64 on the vector units)")
    ap.add_argument("--mutual", action="store_true",
                    help="mutual P2P: each unordered pair of different leaves once, both leaves updated")
    ap.add_argument("--tight", action="store_true",
                    help="acceptance also by cell radii tight to the bodies (fewer M2L and P2P pairs)")
    ap.add_argument("--let-ranks", default="",
                    help="comma-separated virtual rank counts: also time the evaluation split over that many "
                         "ranks (ORB + LET on this GPU) and report LET sizes and timings per count")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (the reference for HBM counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy > 0:
        import torch
        a = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": a.numel() * 4}), flush=True)
        return
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
    prm = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision=args.precision, tight=args.tight,
                   m2l_sparse=args.m2l_sparse, m2l_rotation=args.m2l_rotation, mutual=args.mutual)
    log(f"bench: {args.config} n={n} p={cfg['p']} theta={cfg['theta']} ncrit={cfg['ncrit']} {args.precision}")
    stream = torch.cuda.current_stream()
    new_plan = lambda timing=False: F.Plan(x, prm, timing=timing, torch_allocator=not args.pool)

    def step(ev=None):
        """Forward with the plan released afterwards, then the backward with
        the plan rebuilt; ev = 4 events (start, after build, after forward,
        after backward).  Returns the two plans' stats and the outputs."""
        if ev is not None:
            ev[0].record(stream)
        plan = new_plan(ev is not None)
        if ev is not None:
            ev[1].record(stream)
        phi, E = plan.evaluate(q)
        if ev is not None:
            ev[2].record(stream)
        st_f = plan.stats() if ev is not None else None
        plan.close()
        plan = new_plan(ev is not None)
        dq, dx = plan.adjoint(q, w, E)
        if ev is not None:
            ev[3].record(stream)
        st_b = plan.stats() if ev is not None else None
        plan.close()
        return st_f, st_b, (phi, E, dq, dx)

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {k + 1}/{args.warmup} done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    stf, stb = [], []
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sf, sb, outs = step(evs[k])
        stf.append(sf)
        stb.append(sb)
        log(f"bench: step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    peak_mem = torch.cuda.max_memory_allocated()
    del outs
    fwd = [e[0].elapsed_time(e[2]) for e in evs]
    bld = [e[0].elapsed_time(e[1]) for e in evs]
    bwd = [e[2].elapsed_time(e[3]) for e in evs]
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_fwd, t_bwd = float(np.median(fwd)), float(np.median(bwd))
    log(f"bench: {args.steps} timed steps: forward {t_fwd:.3f} ms, backward {t_bwd:.3f} ms, step {ms_step:.3f} ms, "
        f"peak memory {peak_mem / 2**30:.2f} GiB")

    # evaluation alone on a reused plan; keep its outputs for the accuracy check
    plan = F.Plan(x, prm)
    ev_ms = []
    for k in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        phi, E = plan.evaluate(q)
        e1.record(stream)
        torch.cuda.synchronize()
        ev_ms.append(e0.elapsed_time(e1))
    t_eval = float(np.median(ev_ms))
    body_pairs = plan.body_pairs()
    stats = plan.stats()
    phi_h, E_h = phi.cpu().numpy(), E.cpu().numpy()
    plan.close()
    del phi, E

    mean = lambda key, src=stf: float(np.mean([s[key] for s in src]))
    ph = {"build": float(np.median(bld)), "build_host_ms": mean("ms_build"), "build_tree": mean("ms_tree"),
          "build_traverse": mean("ms_traverse"), "build_ops": mean("ms_ops"), "p2m": mean("ms_p2m"),
          "m2l_same": mean("ms_m2l"), "m2l_cross": mean("ms_m2l_cross"), "l2l": mean("ms_l2l"),
          "p2p": mean("ms_p2p"), "l2p": mean("ms_l2p"), "evaluate": mean("ms_evaluate"),
          "adjoint": mean("ms_adjoint", stb)}
    stats["p2p_body_pairs"] = body_pairs
    per_phase, tstar_ms = roofline_phases(cfg, stats, ph, n, args.precision, args.m2l_rotation)

    # roofline of the dominant kernel: the same-level M2L (all chunk launches
    # of k_m2l_batched in one evaluation, timed by events on their stream) or P2P
    p2 = cfg["p"] ** 2
    m2l_flops = 2.0 * p2 * p2 * (stats["n_m2l_same"] - stats["n_m2l_sparse"])
    p2p_flops = 20.0 * body_pairs
    if args.m2l_rotation:
        # every M2L pair in the rotation kernel (float64 vector arithmetic)
        rot_flops = rotation_flops(cfg["p"]) * stats["n_m2l"]
        achieved = rot_flops / (ph["m2l_cross"] * 1e-3) / 1e12
        roof = {"kernel": "k_m2l_rot (M2L by rotation, all pairs, one evaluation)", "bound": "alu",
                "achieved": achieved, "peak": PEAK["valu_f64"], "unit": "TFLOP/s", "frac": achieved / PEAK["valu_f64"],
                "traffic": None, "launch_ms": ph["m2l_cross"], "flops_per_launch": rot_flops}
    elif ph["m2l_same"] >= ph["p2p"]:
        peak = PEAK["mfma_f32"] if args.precision == "mixed" else PEAK["mfma_f64"]
        achieved = m2l_flops / (ph["m2l_same"] * 1e-3) / 1e12
        roof = {"kernel": "k_m2l_batched (same-level M2L, all chunk launches of one evaluation)", "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": recorded_traffic("k_m2l_batched", args.config, args.precision),
                "launch_ms": ph["m2l_same"], "flops_per_launch": m2l_flops}
    else:
        peak = PEAK["valu_f32"] if args.precision == "mixed" else PEAK["valu_f64"]
        achieved = p2p_flops / (ph["p2p"] * 1e-3) / 1e12
        roof = {"kernel": "k_p2p", "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": recorded_traffic("k_p2p", args.config, args.precision),
                "launch_ms": ph["p2p"], "flops_per_launch": p2p_flops}
    # all M2L work (both kernels' pairs) against both phases' time
    m2l_all = 2.0 * p2 * p2 * stats["n_m2l"] / ((ph["m2l_same"] + ph["m2l_cross"]) * 1e-3) / 1e12
    roof["m2l_all"] = {"achieved": m2l_all, "frac": m2l_all / (PEAK["mfma_f32"] if args.precision == "mixed"
                                                              else PEAK["mfma_f64"])}
    roof["tstar_forward_ms"] = tstar_ms
    roof["overall_frac"] = tstar_ms / t_fwd
    roof["phases"] = per_phase

    # FP64 GPU baseline (same build + forward), one warm-up run
    fp64_ms, phi64_h, E64_h = None, None, None
    if args.fp64_steps > 0 and args.precision != "fp64":
        prm64 = F.Params(p=cfg["p"], theta=cfg["theta"], ncrit=cfg["ncrit"], precision="fp64", tight=args.tight,
                         m2l_sparse=args.m2l_sparse, m2l_rotation=args.m2l_rotation, mutual=args.mutual)
        times = []
        for k in range(args.fp64_steps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            p64 = F.Plan(x, prm64, torch_allocator=not args.pool)
            phi64, E64 = p64.evaluate(q)
            e1.record(stream)
            torch.cuda.synchronize()
            if k > 0:
                times.append(e0.elapsed_time(e1))
            p64.close()
        fp64_ms = float(np.mean(times))
        phi64_h, E64_h = phi64.cpu().numpy(), E64.cpu().numpy()
        del phi64, E64
        log(f"bench: fp64 forward {fp64_ms:.3f} ms")

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    err = {}
    if phi64_h is not None:
        err["mixed_vs_fp64_gpu_all_bodies"] = {"phi": rel(phi_h, phi64_h), "E": rel(E_h, E64_h)}

    let = []
    for R in [int(v) for v in args.let_ranks.split(",") if v.strip()]:
        out_l = None
        times = []
        for k in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out_l = F.let_evaluate(x, q, R, prm)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        st = out_l["stats"]
        phl, Eal = out_l["phi"].cpu().numpy(), out_l["E"].cpu().numpy()
        let.append({"ranks": R, "ms": times[-1], "particles_per_s": n / (times[-1] * 1e-3),
                    "vs_single_tree_all_bodies": {"phi": float(np.linalg.norm(phl - phi_h) / np.linalg.norm(phi_h)),
                                                  "E": float(np.linalg.norm(Eal - E_h) / np.linalg.norm(E_h))},
                    **{k: st[k] for k in ("let_cells", "let_far", "let_body_leaves", "let_bodies", "let_bytes",
                                          "n_m2l_local", "n_p2p_local", "n_m2l_remote", "n_p2p_remote",
                                          "n_m2p_remote", "device_bytes", "ms_partition", "ms_build", "ms_let",
                                          "ms_evaluate")}})
        log(f"bench: {R} virtual ranks: {times[-1]:.1f} ms, LET {st['let_bytes'] / 2**20:.1f} MiB")
        del out_l

    cpu, bad = None, False
    nt = ORACLE_TARGETS.get(args.config, 256) if args.oracle_targets < 0 else args.oracle_targets
    if nt > 0:
        import oracle
        tg = W.sample_targets(n, nt)
        cores = oracle.num_threads()
        c0 = time.perf_counter()
        T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tg, prune=True, tight=args.tight)
        po, Eo = T.fmm(q_np, cfg["p"], targets=tg)
        c1 = time.perf_counter()
        del T
        err["vs_oracle_sampled"] = {"phi": rel(phi_h[tg], po), "E": rel(E_h[tg], Eo), "targets": int(tg.size)}
        bad = max(err["vs_oracle_sampled"]["phi"], err["vs_oracle_sampled"]["E"]) > (
            1e-4 if args.precision == "mixed" else 1e-6)
        if phi64_h is not None:
            err["fp64_gpu_vs_oracle_sampled"] = {"phi": rel(phi64_h[tg], po), "E": rel(E64_h[tg], Eo)}
        log(f"bench: oracle {tg.size} targets on {cores} threads in {c1 - c0:.2f} s; err {err}")
        cpu = {"value": tg.size / (c1 - c0), "unit": "particles/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 oracle FMM of {args.config}: full tree build of all {n} bodies, P2M/M2M of every "
                         f"cell, pruned traversal and evaluation at {tg.size} sampled targets; {c1 - c0:.2f} s "
                         f"on {cores} threads"}
        ns = max(1, tg.size // 8) if args.serial_targets < 0 else args.serial_targets
        if ns > 0:
            oracle.set_num_threads(1)
            s0 = time.perf_counter()
            T = oracle.Tree(x_np, cfg["ncrit"], cfg["theta"], targets=tg[:ns], prune=True, tight=args.tight)
            T.fmm(q_np, cfg["p"], targets=tg[:ns])
            s1 = time.perf_counter()
            del T
            oracle.set_num_threads(cores)
            cpu["serial"] = {"value": ns / (s1 - s0), "unit": "particles/s", "cores": 1,
                             "sample": f"the same at {ns} sampled targets on 1 thread; {s1 - s0:.2f} s"}
            log(f"bench: serial oracle {ns} targets in {s1 - s0:.2f} s")

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
                               f"ncrit={cfg['ncrit']}{', tight radii' if args.tight else ''}; forward (build + "
                               f"evaluate) and backward (plan rebuilt, adjoint of L = sum w phi)", "n": n,
                   "p": cfg["p"], "theta": cfg["theta"], "ncrit": cfg["ncrit"], "precision": args.precision,
                   "tight": args.tight, "m2l_sparse": args.m2l_sparse, "m2l_rotation": args.m2l_rotation,
                   "mutual": args.mutual},
        "forward_ms": t_fwd,
        "forward_ms_mean": float(np.mean(fwd)),
        "backward_ms": t_bwd,
        "adjoint_over_forward": t_bwd / t_fwd,
        "evaluate_only_ms": t_eval,
        "fp64_forward_ms": fp64_ms,
        "speedup_vs_fp64": (fp64_ms / t_fwd) if fp64_ms else None,
        "memory_high_water_gib": peak_mem / 2**30,
        "memory_inputs_gib": base_mem / 2**30,
        "err": err,
        "phases_ms": ph,
        "counts": {k: stats[k] for k in ("ncell", "nleaf", "depth", "n_m2l", "n_m2l_same", "n_m2l_cross", "n_p2p",
                                         "p2p_body_pairs", "m2l_stencil", "m2l_offsets", "m2l_slots", "m2l_rows",
                                         "n_m2l_sparse", "p2p_mutual_pairs", "device_bytes")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if let:
        out["virtual_ranks"] = let
    print(json.dumps(out), flush=True)
    if bad:
        log("bench: the accuracy bar was missed")
        sys.exit(3)


if __name__ == "__main__":
    main()
