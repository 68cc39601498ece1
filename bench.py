#!/usr/bin/env python3
"""Benchmark of the block-tridiagonal Cholesky hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole hot path over one synthetic instance that is
already resident in HBM: a full refactorization (all levels of the
nested-dissection elimination) followed by a solve (forward and backward
level sweeps).  W untimed steps, then K timed steps bracketed by
device synchronisation.  Prints ONE JSON line.

The roofline object describes the dominant kernel (the level launch with the
largest total time), timed live with HIP events recorded by the library on the
launch stream; its algorithmic bytes and flops per launch are computed from
the level schedule (see ``level_work``).  The CPU baseline runs the FP64
oracle (test infrastructure) single-threaded on the same instance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor+solve/sec & p99 latency, served mixed-prec vs plain FP64 @1e-10 resid"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP64_RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)


def level_work(N: int, n: int, m: int = 1, mixed: bool = False):
    """Algorithmic flops and HBM bytes of every level launch.

    Factor, per node i at level l (stride s), with the block I/O the level step
    of Algorithm 4 defines (each n x n block read or written once):
      reads  S_i, C_{i+s,i} (if right), C_{i,i-s} (if left), T_{i+s/2} (if
             deferred), S_{i+s} (if right), T_{i+3s/2} (if deferred)
      writes L_ii, R_i, T_i, S_{i+s}, fill C_{i+s,i-s} (when present)
      flops  potrf n^3/3, trsm n^3 each, syrk n^3 each, gemm 2n^3
             (cost table of section "Computational Complexity").
    Word sizes: 8 bytes for everything on the FP64 path; on the mixed path the
    Schur complements S and the input blocks are FP64 (8 bytes) and the factor
    blocks L, R, T and the fill couplings FP32 (4 bytes).
    Solve, per node and sweep: reads L_ii, R_i, T_i (when present) plus the
    n x m vectors it touches; flops n^2 m per triangular solve and 2n^2 m per
    block product (Algorithm 6)."""
    out = {"factor": [], "forward": [], "backward": []}
    wS = 8.0
    wF = 4.0 if mixed else 8.0
    nn = n * n
    L = int(np.floor(np.log2(N))) + 1
    for l in range(L):
        s = 1 << l
        h = s >> 1
        i = np.arange(s, N + 1, 2 * s, dtype=np.int64)
        has_r = i + s <= N
        has_l = i > s
        d_self = (i + h <= N) & (l > 0)
        d_sep = (i + 3 * h <= N) & has_r & (l > 0)
        both = has_r & has_l
        wC = 8.0 if l == 0 else wF  # level 0 reads the couplings from the FP64 input
        rd = nn * (wS * (len(i) + has_r.sum()) + wC * (has_r.sum() + has_l.sum())
                   + wF * (d_self.sum() + d_sep.sum()))
        wr = nn * (wS * has_r.sum() + wF * (len(i) + has_r.sum() + has_l.sum() + both.sum()))
        fl = n ** 3 * (len(i) / 3 + 2 * has_r.sum() + has_l.sum() + d_self.sum() + d_sep.sum()
                       + 2 * both.sum())
        out["factor"].append({"bytes": float(rd + wr), "flops": float(fl), "nodes": len(i)})
        vec = wF * n * m
        blocks = len(i) + has_r.sum() + has_l.sum()
        pulls = len(i) * 2 * l  # at most 2 small vectors per lower level
        fwd_b = blocks * nn * wF + vec * (len(i) + pulls) + vec * (len(i) + has_r.sum() + has_l.sum())
        bwd_b = blocks * nn * wF + vec * (len(i) + has_r.sum() + has_l.sum()) + vec * len(i)
        sfl = n * n * m * (len(i) + 2 * has_r.sum() + 2 * has_l.sum())
        out["forward"].append({"bytes": float(fwd_b), "flops": float(sfl), "nodes": len(i)})
        out["backward"].append({"bytes": float(bwd_b), "flops": float(sfl), "nodes": len(i)})
    return out


def cpu_baseline(pr, budget_s: float):
    """FP64 oracle (plain C, one thread) factor + solve on the same instance,
    repeated while within the time budget (at least once)."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    runs = 0
    while True:
        Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
        oracle.solve_nd(Ld, Rb, Tb, pr.B)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 50:
            break
        if el / runs * (runs + 1) > budget_s * 1.5:
            break
    return runs / el, runs, el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fp64-single", choices=["fp64-single"])
    ap.add_argument("--N", type=int, default=4096)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_ir"])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the method factors one block-tridiagonal system "
              "per device here; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_2601_03754_amd import btc, inputs

    N, n, m = args.N, args.n, args.nrhs
    seed = inputs.sweep_seed(N, n)
    pr = inputs.block_tridiag(N, n, c=4.0, seed=seed, nrhs=m)
    dev = torch.device("cuda:0")
    D = torch.from_numpy(pr.D).to(dev)
    E = torch.from_numpy(pr.E).to(dev)
    B = torch.from_numpy(pr.B).to(dev)
    X = torch.empty_like(B)
    stream = torch.cuda.current_stream()
    prec = btc.BTC_FP64 if args.precision == "fp64" else btc.BTC_FP32_IR
    f = btc.Factor(D, E, precision=prec)
    for _ in range(args.warmup):
        f.refactor(D, E)
        f.solve(B, X)
    torch.cuda.synchronize()
    info = f.info
    if info != 0:
        raise RuntimeError("factorization broke down at block %d" % info)

    # timed region: K steps bracketed by synchronisation, no instrumentation
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        f.refactor(D, E)
        f.solve(B, X)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)

    # live kernel timing: the same K steps again with HIP events recorded by the
    # library around every level launch on its launch stream
    btc.btc_profile(f.handle, True)
    for _ in range(args.steps):
        f.refactor(D, E)
        f.solve(B, X)
    torch.cuda.synchronize()
    prof = {ph: btc.btc_profile_read(f.handle, k) for k, ph in enumerate(("factor", "forward", "backward", "refine"))}
    btc.btc_profile(f.handle, False)

    # accuracy of the last step, checked by the oracle's FP64 residual
    relres = oracle.relres(pr.D, pr.E, X.cpu().numpy(), pr.B)
    _, sinfo = f.solve(B, X, want_info=True)

    ms_step = wall * 1e3 / args.steps
    value = args.steps / wall

    work = level_work(N, n, m, mixed=args.precision != "fp64")
    best = None
    for ph in ("factor", "forward", "backward"):
        ms, cnt = prof[ph]
        for l in range(len(ms)):
            if cnt[l] > 0 and (best is None or ms[l] > best[0]):
                best = (ms[l], ph, l, ms[l] / cnt[l])
    _, ph, lvl, avg_ms = best
    wk = work[ph][lvl]
    ai = wk["flops"] / wk["bytes"]
    if ai < FP64_RIDGE:
        roof = {"bound": "hbm", "achieved": wk["bytes"] / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": wk["flops"] / (avg_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = "%s level %d (%d nodes)" % (ph, lvl, wk["nodes"])
    roof["avg_launch_ms"] = avg_ms

    cpu = None
    if not args.no_cpu_baseline:
        rate, runs, el = cpu_baseline(pr, args.cpu_budget)
        cpu = {"value": rate, "unit": "factor+solve/s", "cores": 1, "kind": "oracle",
               "sample": "%d full factor+solve runs of the same instance (N=%d, n=%d, nrhs=%d) in %.1f s"
                         % (runs, N, n, m, el)}

    tot_fl = sum(w["flops"] for w in work["factor"]) + sum(w["flops"] for w in work["forward"]) \
        + sum(w["flops"] for w in work["backward"])
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "factor+solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 factor+solve, single instance, refactor every step",
                   "N": N, "n": n, "nrhs": m, "diag_shift": 4.0, "seed": seed,
                   "precision": args.precision},
        "refine": sinfo,
        "relres": relres,
        "gpu_event_ms_per_step": gpu_ms / args.steps,
        "gflops_per_s": tot_fl / (ms_step * 1e-3) / 1e9,
        "per_level_ms": {ph: [round(float(x) / args.steps, 5) for x in prof[ph][0]] for ph in prof},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    f.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
