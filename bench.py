#!/usr/bin/env python3
"""Benchmark of the block-tridiagonal Cholesky hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload served|single]

Default workload ("served"): 256 clients, each with its own block-tridiagonal
system (N log-uniform in [64, 4096], n uniform in {12..96}, diagonal shift 4,
one right-hand side), served by the library's continuous-batching server.
Every request is either a solve against the client's resident factor with a
new right-hand side (70%) or a refactorization with new matrix values
followed by a solve (30%).  The headline runs the server closed-loop at
saturation: every client always has one request outstanding and submits its
next one as soon as the previous one completes.  A step is 4096 completed
requests (16 per client on average; --step-requests); W untimed steps, then K
timed steps bracketed by device synchronisation.  The mixed-precision path (FP32 factor
and sweeps, FP64 Schur complements, pivot factorizations, residual and
iterative refinement to a 1e-10 relative residual) is the headline; the plain
FP64 path runs the same trace beside it.  Latency (p50/p99) is measured per
request from submission to the observed completion; the open-loop Poisson
runs (--rates) report latency at fixed arrival rates from the scheduled
arrival time.  Every input is drawn on the device before timing starts.

Workload "single": one instance (N, n) refactored and solved every step.

Roofline: the kernel group with the largest total time (found during the
warm-up) is timed live during the timed region with HIP events that the
library records on the stream each launch runs on (independent groups of one
server step run concurrently on up to four streams, so a timed launch may
share the GPU); its algorithmic bytes/flops per launch come from
btc_level_work.  "roofline_aggregate" divides the algorithmic bytes and flops
of every kernel of the timed region by its wall time.  Every completed
request reports its outcome (factor status, converged flag, the FP64
residual of its last convergence test): the line counts them ("verified")
and splits latency by request class ("per_class").  The CPU baseline is
Algorithm 1 of the oracle (plain C, FP64) on every host core over a bounded
sample of the same requests, with the single-threaded nested-dissection
oracle beside it.  "configs" holds the other benchmark configurations: the
FP64 sweep table (N x n: time, GFLOP/s, GB/s, roofline fractions), the
many-instance batch (instances/s, with and without autotuning) and the
latency of every elimination order at N = 16, n = 8.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor+solve/sec & p99 latency, served mixed-prec vs plain FP64 @1e-10 resid"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
OPS = {0: "factor", 1: "forward", 2: "backward", 3: "residual", 4: "refine_init", 5: "refine_test"}
FACTOR_KIND = {0: "fp64 valu", 1: "fp64 mfma", 2: "mixed", 3: "fp64 tiled", 4: "mixed tiled", 5: "mixed bf16",
               6: "mixed bf16 tiled"}
TILED_PART = {1: "k_tiled_syrk_deferred", 2: "k_tiled_potrf_trsm", 3: "k_tiled_update"}
SOLVE_FRAC = 0.7
RELRES_TARGET = 1e-10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else float("nan")


def relres_torch(D, E, X, B):
    """max over columns of ||b - Psi x||_2 / ||b||_2 in FP64 with plain torch
    ops (independent of the library): Psi has the lower triangles of D
    mirrored on the diagonal and E[i-1] at block (i+1, i)."""
    import torch
    Dl = torch.tril(D) + torch.tril(D, -1).transpose(1, 2)
    R = B - torch.bmm(Dl, X)
    if E.shape[0]:
        R[1:] -= torch.bmm(E, X[:-1])
        R[:-1] -= torch.bmm(E.transpose(1, 2).contiguous(), X[1:])
    num = torch.linalg.vector_norm(R, dim=(0, 1))
    den = torch.linalg.vector_norm(B, dim=(0, 1))
    return float((num / den).max())


# HBM traffic of kernel groups measured with rocprofv3 PMC counters
# (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by a plain copy kernel) over
# a whole served run, divided by the algorithmic bytes of the same launches
# (the run's group_totals): rows "| group | measured / algorithmic | sha1 |
# sources |" of the committed summary.  The traffic of a launch is that ratio
# times its algorithmic bytes.  A row counts only while the sha1 of its
# sources (the kernel files, concatenated in the listed order) still matches.
TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "pmc_traffic_served.md")


def committed_traffic(group):
    import hashlib
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2601_03754_amd", "csrc")
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) != 4 or cells[0] != group:
            continue
        try:
            value = float(cells[1])
        except ValueError:
            continue
        h = hashlib.sha1()
        try:
            for f in cells[3].split():
                h.update(open(os.path.join(csrc, f.strip("`")), "rb").read())
        except OSError:
            return None
        return value if h.hexdigest() == cells[2].strip("`") else None
    return None


def roofline_entry(stat):
    """Roofline object for one profiled kernel group."""
    avg_ms = stat["ms"] / stat["launches"]
    bpl = stat["bytes"] / stat["launches"]
    fpl = stat["flops"] / stat["launches"]
    t_hbm = bpl / (HBM_PEAK_GBS * 1e9)
    # FP32 peak for the FP32 kernel families (mixed factor: its products run on
    # FP32 matrix cores; FP32 sweeps), FP64 peak otherwise
    fp32 = (stat["op"] == 0 and stat["kind"] in (2, 4)) or (stat["op"] in (1, 2) and stat["kind"] in (1, 3))
    fpeak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    t_alu = fpl / (fpeak * 1e12)
    if t_hbm >= t_alu:
        r = {"bound": "hbm", "achieved": bpl / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        r = {"bound": "alu", "achieved": fpl / (avg_ms * 1e-3) / 1e12, "peak": fpeak, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = None
    r["avg_launch_ms"] = avg_ms
    r["launches"] = stat["launches"]
    r["algorithmic_bytes_per_launch"] = bpl
    r["algorithmic_flops_per_launch"] = fpl
    kind = FACTOR_KIND.get(stat["kind"], str(stat["kind"])) if stat["op"] == 0 else \
        ("fp32" if stat["kind"] & 1 else "fp64") + (" ranges" if stat["kind"] >= 2 else "") \
        if stat["op"] in (1, 2) else "fp64"
    r["kernel"] = "%s %s np=%d" % (OPS[stat["op"]], kind, stat["np"])
    if stat.get("part"):
        r["kernel"] += " " + TILED_PART[stat["part"]]
    ratio = committed_traffic(r["kernel"])
    r["traffic"] = None if ratio is None else ratio * bpl
    return r


# ---------------------------------------------------------------------------
# served workload

class Clients:
    """Device-resident inputs of every client: two matrix versions (a
    refactorization switches to the other one) and four right-hand sides."""

    def __init__(self, shapes, seed=0):
        import torch
        from paper_2601_03754_amd import inputs
        self.shapes = shapes
        self.mats, self.rhs, self.X = [], [], []
        for c, (N, n) in enumerate(shapes):
            vers = []
            for v in range(2):
                D, E, B = inputs.block_tridiag_device(N, n, 4.0, seed=seed * 100003 + 2 * c + v, nrhs=4)
                vers.append((D, E))
                if v == 0:
                    self.rhs.append([B[:, :, k:k + 1].contiguous() for k in range(4)])
                del B
            self.mats.append(vers)
            self.X.append(torch.zeros((N, n, 1), dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()


class Served:
    """One server (one precision) over the clients, with the bookkeeping of
    the requests a run submits."""

    def __init__(self, btc, clients, precision, seed, sweep_ranges=False, hbm_budget=1 << 46, lanes=0):
        self.btc = btc
        self.cl = clients
        self.srv = btc.Server(precision=precision, hbm_budget=hbm_budget, sweep_ranges=sweep_ranges, lanes=lanes)
        self.ids = [self.srv.add_client(N, n) for N, n in clients.shapes]
        self.rng = np.random.default_rng(seed)
        self.ver = [0] * len(self.ids)
        self.rhs_k = [0] * len(self.ids)
        self.first = [True] * len(self.ids)
        self.last = {}  # client -> (version, rhs index) of its last submitted request

    def submit(self, c, refactor=None):
        if refactor is None:
            refactor = self.first[c] or self.rng.random() >= SOLVE_FRAC
        if refactor and not self.first[c]:
            self.ver[c] ^= 1
        self.first[c] = False
        k = self.rhs_k[c] = (self.rhs_k[c] + 1) % 4
        A = self.cl.mats[c][self.ver[c]] if refactor else None
        t = self.srv.submit(self.ids[c], self.cl.rhs[c][k], self.cl.X[c], A=A)
        self.last[c] = (self.ver[c], k)
        return t

    def closed_loop(self, requests):
        """Every client keeps one request outstanding until `requests` have
        been submitted; returns (completions, wall seconds)."""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sub = 0
        for c in range(len(self.ids)):
            if sub < requests:
                self.submit(c)
                sub += 1
        done = []
        t_step = 0.0
        ticks = 0
        while len(done) < requests:
            ts = time.perf_counter()
            self.srv.step()
            t_step += time.perf_counter() - ts
            ticks += 1
            for d in self.srv.poll():
                done.append(d)
                if sub < requests:
                    self.submit(d["client"])
                    sub += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        self.last_loop = {"ticks": ticks, "host_step_s": t_step, "wall_s": wall}
        return done, wall

    def open_loop(self, rate, requests):
        """Poisson arrivals at `rate` per second over random clients;
        latency from the scheduled arrival to the observed completion."""
        import torch
        rng = np.random.default_rng(int(rate))
        arr = np.cumsum(rng.exponential(1.0 / rate, size=requests))
        who = rng.integers(0, len(self.ids), size=requests)
        torch.cuda.synchronize()
        t0m = time.monotonic()
        sched = {}
        k = 0
        done = []
        while len(done) < requests:
            now = time.monotonic() - t0m
            while k < requests and arr[k] <= now:
                t = self.submit(int(who[k]))
                sched[t] = t0m + arr[k]
                k += 1
            self.srv.step()
            for d in self.srv.poll():
                d["t_sched"] = sched.pop(d["ticket"])
                done.append(d)
        torch.cuda.synchronize()
        wall = time.monotonic() - t0m
        return done, wall

    def verify(self):
        """Relative residual of every client's last result (FP64, torch)."""
        worst = 0.0
        for c, (v, k) in self.last.items():
            D, E = self.cl.mats[c][v]
            worst = max(worst, relres_torch(D, E, self.cl.X[c], self.cl.rhs[c][k]))
        return worst

    def close(self):
        self.srv.close()


def prof_on(btc, rhs, op, kind):
    for r in rhs:
        btc.runner_profile(r, op, kind)


def prof_read(btc, rhs):
    """Launch-profile totals summed over the server's lane runners, largest
    time first."""
    agg = {}
    for r in rhs:
        for st in btc.runner_profile_read(r):
            k = (st["op"], st["kind"], st["np"], st["part"])
            if k in agg:
                for f in ("launches", "items", "ms", "bytes", "flops"):
                    agg[k][f] += st[f]
            else:
                agg[k] = dict(st)
    return sorted(agg.values(), key=lambda st: -st["ms"])


def host_stats(btc, rhs, reset=False):
    tot = {"run_s": 0.0, "wait_s": 0.0, "calls": 0}
    for r in rhs:
        h = btc.runner_host_stats(r, reset=reset)
        for k in tot:
            tot[k] += h[k]
    return tot


def lat_ms(done, key="t_submit", drop=0.05):
    d = done[int(len(done) * drop):]
    return [(x["t_done"] - x[key]) * 1e3 for x in d]


def run_served(args, btc):
    import torch
    from paper_2601_03754_amd import inputs
    shapes = inputs.served_clients(args.clients, seed=0)
    log("generating inputs of %d clients on the device" % len(shapes))
    cl = Clients(shapes)
    per_step = args.step_requests
    paths = {}
    rates_out = []
    roof = None
    for name, prec in (("mixed", btc.BTC_FP32_IR), ("fp64", btc.BTC_FP64)):
        sv = Served(btc, cl, prec, seed=1, sweep_ranges=args.sweep_ranges, lanes=args.lanes)
        rhs = sv.srv.runner_handles()
        # warm-up: first requests factor every client; profile every group
        prof_on(btc, rhs, -1, -1)
        sv.closed_loop(per_step * max(1, args.warmup))
        stats = prof_read(btc, rhs)
        dom = stats[0]
        # timed region: only the dominant group's family carries events
        prof_on(btc, rhs, -1 if args.profile_all else dom["op"], -1 if args.profile_all else dom["kind"])
        host_stats(btc, rhs, reset=True)
        sv.srv.host_stats(reset=True)
        done, wall = sv.closed_loop(per_step * args.steps)
        hstat = host_stats(btc, rhs)
        sstat = sv.srv.host_stats()
        allstats = prof_read(btc, rhs)
        totals = None
        if args.profile_all:
            totals = {}
            for st_ in list(stats) + list(allstats):
                t = totals.setdefault(roofline_entry(st_)["kernel"], {"launches": 0, "bytes": 0.0, "ms": 0.0})
                t["launches"] += st_["launches"]
                t["bytes"] += st_["bytes"]
                t["ms"] += st_["ms"]
        tstats = [s for s in allstats
                  if (s["op"], s["kind"], s["np"], s["part"]) == (dom["op"], dom["kind"], dom["np"], dom["part"])]
        prof_on(btc, rhs, -2, -1)
        lat = lat_ms(done)
        loop = dict(sv.last_loop)
        relres = sv.verify()
        # every completion carries the outcome of its request: the factor's
        # status, and for the mixed path the converged flag and the FP64
        # residual its last convergence test measured
        conv = sum(1 for d in done if d["converged"] and d["info"] == 0)
        dev_rr = [d["relres"] for d in done if d["relres"] >= 0]
        per_class = {}
        for cls, sel in (("solve", False), ("refactor_solve", True)):
            dd = [d for d in done if bool(d["refactored"]) == sel]
            lc = lat_ms(dd)
            per_class[cls] = {"requests": len(dd), "share": len(dd) / max(1, len(done)),
                              "p50_ms": pct(lc, 50), "p99_ms": pct(lc, 99),
                              "steps_max": max([d["steps"] for d in dd], default=0)}
        ent = {"value": len(done) / wall, "ms_per_step": wall * 1e3 / args.steps,
               "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "requests": len(done), "wall_s": wall,
               "refactor_share": float(np.mean([d["refactored"] for d in done])),
               "verified": {"requests": len(done), "converged": conv,
                            "relres_max_device": max(dev_rr) if dev_rr else None,
                            "relres_max_last_torch": relres},
               "per_class": per_class,
               "lanes": len(rhs), "server_ticks": sstat["ticks"], "step_calls": loop["ticks"],
               "host_step_frac": loop["host_step_s"] / loop["wall_s"],
               # where the host's time per tick goes: planning in the server,
               # enqueueing in the runners, and waiting for the device (for
               # the oldest tick in flight, or for a runner's descriptor
               # slot); a host that waits on every tick leaves the device as
               # the bottleneck
               "host_us_per_tick": {
                   "step": loop["host_step_s"] / max(1, sstat["ticks"]) * 1e6,
                   "planning": (loop["host_step_s"] - hstat["run_s"] - sstat["wait_s"])
                   / max(1, sstat["ticks"]) * 1e6,
                   "enqueue": (hstat["run_s"] - hstat["wait_s"]) / max(1, sstat["ticks"]) * 1e6,
                   "device_wait": (hstat["wait_s"] + sstat["wait_s"]) / max(1, sstat["ticks"]) * 1e6,
                   "wall": loop["wall_s"] / max(1, sstat["ticks"]) * 1e6},
               "max_relres_last": relres,
               "warmup_kernel_ms": [{"kernel": roofline_entry(s)["kernel"], "ms": round(s["ms"], 3),
                                     "launches": s["launches"],
                                     "gbs": round(s["bytes"] / (s["ms"] * 1e-3) / 1e9, 1)} for s in stats[:10]]}
        if totals is not None:
            ent["group_totals"] = totals
        if tstats:
            ent["roofline"] = roofline_entry(tstats[0])
        # every kernel of the timed region: algorithmic bytes / flops over its wall time
        tb = sum(s["bytes"] for s in allstats)
        tf = sum(s["flops"] for s in allstats)
        ent["aggregate"] = {"bytes": tb, "flops": tf, "gbs": tb / wall / 1e9, "tflops": tf / wall / 1e12,
                            "hbm_frac": tb / wall / 1e9 / HBM_PEAK_GBS}
        log("%s closed loop: %.0f req/s, p50 %.2f ms, p99 %.2f ms, relres %.2e, %d ticks, host step %.0f%%"
            % (name, ent["value"], ent["p50_ms"], ent["p99_ms"], relres, sstat["ticks"],
               100 * ent["host_step_frac"]))
        for rate in args.rates:
            nreq = int(min(args.rate_requests, max(200, rate * args.rate_seconds)))
            d2, w2 = sv.open_loop(rate, nreq)
            l2 = lat_ms(d2, key="t_sched")
            rates_out.append({"path": name, "rate": rate, "requests": nreq, "achieved": nreq / w2,
                              "p50_ms": pct(l2, 50), "p99_ms": pct(l2, 99)})
            log("%s open loop %d/s: achieved %.0f/s p50 %.2f p99 %.2f ms"
                % (name, rate, nreq / w2, rates_out[-1]["p50_ms"], rates_out[-1]["p99_ms"]))
        sv.close()
        paths[name] = ent
        torch.cuda.synchronize()
    return shapes, paths, rates_out


def cpu_baseline_served(shapes, budget_s, wall_cap_s=90.0):
    """The FP64 oracle (plain C, one thread) on requests of the same mix:
    clients in order; refactor+solve for 30% of them, solve-only otherwise
    (factor time not counted for those), until `budget_s` seconds of oracle
    time are spent (or the wall-clock cap, which includes drawing the inputs
    on the host)."""
    import oracle
    from paper_2601_03754_amd import inputs
    oracle.build()
    rng = np.random.default_rng(5)
    t_work = 0.0
    served = 0
    used = []
    t_start = time.perf_counter()
    for c, (N, n) in enumerate(shapes):
        if t_work >= budget_s or time.perf_counter() - t_start > wall_cap_s:
            break
        pr = inputs.block_tridiag(N, n, c=4.0, seed=c, nrhs=1)
        t0 = time.perf_counter()
        Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
        t1 = time.perf_counter()
        oracle.solve_nd(Ld, Rb, Tb, pr.B)
        t2 = time.perf_counter()
        refactor = rng.random() >= SOLVE_FRAC
        t_work += (t2 - t0) if refactor else (t2 - t1)
        served += 1
        used.append((N, n, bool(refactor)))
    return served / t_work, served, t_work, used


def cpu_baseline_alg1(shapes, budget_s, max_clients=48):
    """The natural-order Algorithm 1 of the oracle (plain C, FP64) on every
    host core over requests of the same mix: the first clients' systems
    (inputs drawn beforehand, not timed), one request each (30% refactor +
    solve, 70% solve against a factor computed beforehand), spread over
    os.cpu_count() threads (the oracle releases the interpreter lock);
    requests per wall second.  Stops early once `budget_s` of wall time is
    spent."""
    import os
    import threading
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from paper_2601_03754_amd import inputs
    oracle.build()
    rng = np.random.default_rng(5)
    cores = os.cpu_count() or 1
    reqs = []
    t_gen = time.perf_counter()
    for c, (N, n) in enumerate(shapes[:max_clients]):
        pr = inputs.block_tridiag(N, n, c=4.0, seed=c, nrhs=1)
        refactor = rng.random() >= SOLVE_FRAC
        fac = None if refactor else oracle.factor_seq(pr.D, pr.E)
        reqs.append((pr, refactor, fac))
        if time.perf_counter() - t_gen > 60.0:
            break
    lock = threading.Lock()
    done = [0]
    t0 = time.perf_counter()
    stop = t0 + budget_s

    def work(k):
        if time.perf_counter() > stop:
            return
        pr, refactor, fac = reqs[k]
        Dh, Eh, info = oracle.factor_seq(pr.D, pr.E) if refactor else fac
        oracle.solve_seq(Dh, Eh, pr.B)
        with lock:
            done[0] += 1

    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(work, range(len(reqs))))
    wall = time.perf_counter() - t0
    return done[0] / wall, done[0], wall, cores


# ---------------------------------------------------------------------------
# benchmark configurations beside the served headline

def sweep_table(btc, Ns=(64, 256, 1024, 4096, 16384), ns=(16, 32, 64, 128), reps=5):
    """FP64 single instance, refactor + solve per call, every (N, n) of the
    sweep: time per call (median over reps, HIP events), GFLOP/s of the
    method's work and algorithmic GB/s (btc_level_work), fraction of the
    FP64 and HBM peaks."""
    import torch
    from paper_2601_03754_amd import inputs
    rows = []
    for N in Ns:
        for n in ns:
            D, E, B = inputs.block_tridiag_device(N, n, 4.0, seed=inputs.sweep_seed(N, n), nrhs=1)
            X = torch.empty_like(B)
            f = btc.Factor(D, E)
            f.solve(B, X)
            L = int(math.floor(math.log2(N))) + 1
            by = fl = 0.0
            for op in (btc.BTC_OP_FACTOR, btc.BTC_OP_FORWARD, btc.BTC_OP_BACKWARD):
                for l in range(L):
                    b_, f_ = btc.btc_level_work(op, 0, N, n, 1, l)
                    by += b_
                    fl += f_
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                f.refactor(D, E)
                f.solve(B, X)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b))
            rr = relres_torch(D, E, X, B)
            f.close()
            ms = float(np.median(ts))
            rows.append({"N": N, "n": n, "ms": round(ms, 4), "gflops": round(fl / (ms * 1e-3) / 1e9, 1),
                         "gbs": round(by / (ms * 1e-3) / 1e9, 1),
                         "fp64_frac": round(fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                         "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "relres": rr})
            del D, E, B, X
            torch.cuda.empty_cache()
    return rows


def batch_rate(btc, count=512, reps=3, tune=False):
    """The many-instance batch: 512 instances (N ~ U{32..2048}, n ~ U{8, 16,
    24, 32, 48}), FP32 factors with FP64 refinement, batched factor + solve
    through one runner (one launch group per level or level range);
    instances per second (median over reps), every result verified."""
    import torch
    from paper_2601_03754_amd import inputs
    shapes = inputs.batch_shapes(count, seed=0)
    mats = [inputs.block_tridiag_device(N, n, 4.0, seed=k, nrhs=1) for k, (N, n) in enumerate(shapes)]
    r = btc.Runner()
    hs = [btc.btc_create(N, n, btc.BTC_FP32_IR) for N, n in shapes]
    Xs = [torch.empty_like(m[2]) for m in mats]
    if tune:
        # the autotuner on the batch itself, as the batched calls run it
        r.autotune(hs, [m[0] for m in mats], [m[1] for m in mats], [m[2] for m in mats], Xs, 1, reps=3)
    ts = []
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.factor_batched(hs, [m[0] for m in mats], [m[1] for m in mats])
        r.solve_batched(hs, [m[2] for m in mats], Xs, 1)
        r.sync()
        if rep:
            ts.append(time.perf_counter() - t0)
    info = r.solve_batched(hs, [m[2] for m in mats], Xs, 1, want_info=True)
    worst = max(relres_torch(m[0], m[1], X, m[2]) for m, X in zip(mats, Xs))
    for h in hs:
        btc.btc_destroy(h)
    r.close()
    t = float(np.median(ts))
    return {"instances": count, "seconds": t, "instances_per_s": count / t,
            "converged": sum(1 for i in info if i["converged"]), "relres_max": worst}


def conditioning_sweep(btc):
    """The conditioning sweep at its own size: N = 4096, n = 64, four
    right-hand sides, the diagonal shifted so that lambda_min(Psi) = c for c
    in {4, 0.1, 0.001} (lambda_min of the unshifted matrix from
    tests/golden/margin_lambda0.json, written by the oracle-based bisection);
    FP32 and BF16 factors with classic FP64 refinement and BF16 with GMRES-
    based refinement: refinement steps, inner GMRES iterations, the device's
    FP64 relative residual, and the solve time."""
    import torch
    from paper_2601_03754_amd import inputs
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                    "margin_lambda0.json")))
    out = []
    for c in (4.0, 0.1, 0.001):
        pr = inputs.block_tridiag(g["N"], g["n"], c=c, seed=g["seed"], nrhs=g["nrhs"], margin=True,
                                  lam0=g["lambda0"])
        D, E, B = (torch.from_numpy(a).to("cuda:0") for a in (pr.D, pr.E, pr.B))
        for name, prec, refine in (("fp32_ir", btc.BTC_FP32_IR, btc.BTC_REFINE_CLASSIC),
                                   ("bf16_ir", btc.BTC_BF16_IR, btc.BTC_REFINE_CLASSIC),
                                   ("bf16_gmres_ir", btc.BTC_BF16_IR, btc.BTC_REFINE_GMRES)):
            f = btc.Factor(D, E, precision=prec, refine=refine)
            f.solve(B, want_info=True)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, info = f.solve(B, want_info=True)
            ms = (time.perf_counter() - t0) * 1e3
            f.close()
            out.append({"c": c, "path": name, "converged": info["converged"], "steps": info["steps"],
                        "inner": info["inner"], "relres": info["relres"], "solve_ms": round(ms, 3)})
        del D, E, B
    return out


def latency_strategies(btc, N=16, n=8, reps=200):
    """The smallest configuration (N = 16, n = 8, FP64): milliseconds per
    refactor + solve of every elimination order, and the one the AUTO
    strategy then takes."""
    import torch
    from paper_2601_03754_amd import inputs
    D, E, B = inputs.block_tridiag_device(N, n, 4.0, seed=0, nrhs=1)
    X = torch.empty_like(B)
    ms = btc.btc_autotune_strategy(D, E, B, X, reps=reps)
    pick = btc.btc_select_strategy(N, n)
    names = ["multistage", "sequential (k=0)", "single-stage (k=1)", "two-stage (k=2)", "partition (p=2)",
             "partition (p=4)"]
    if pick[0] == btc.BTC_STRATEGY_MULTISTAGE:
        auto = names[0]
    elif pick[0] == btc.BTC_STRATEGY_KSTAGE:
        auto = names[1 + pick[1]]
    else:
        auto = "partition (p=%d)" % pick[1]
    return {"N": N, "n": n, "us_per_factor_solve": {names[k]: round(ms[k] * 1e3, 2) for k in range(6) if ms[k] > 0},
            "auto_pick": auto}


# ---------------------------------------------------------------------------
# single-instance workload

def run_single(args, btc):
    import torch
    from paper_2601_03754_amd import inputs
    N, n, m = args.N, args.n, args.nrhs
    seed = inputs.sweep_seed(N, n)
    D, E, B = inputs.block_tridiag_device(N, n, 4.0, seed=seed, nrhs=m)
    X = torch.empty_like(B)
    prec = btc.BTC_FP64 if args.precision == "fp64" else btc.BTC_FP32_IR
    f = btc.Factor(D, E, precision=prec)
    for _ in range(args.warmup):
        f.refactor(D, E)
        f.solve(B, X)
    torch.cuda.synchronize()
    if f.info != 0:
        raise RuntimeError("factorization broke down at block %d" % f.info)
    btc.btc_profile(f.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f.refactor(D, E)
        f.solve(B, X)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {ph: btc.btc_profile_read(f.handle, k) for k, ph in enumerate(("factor", "forward", "backward"))}
    btc.btc_profile(f.handle, False)
    relres = relres_torch(D, E, X, B)
    best = None
    for op, ph in enumerate(("factor", "forward", "backward")):
        ms, cnt = prof[ph]
        for l in range(len(ms)):
            if cnt[l] > 0 and (best is None or ms[l] > best["ms"]):
                b, fl = btc.btc_level_work(op, prec, N, n, m, l)
                best = {"op": op, "kind": 1 if prec else 0, "np": 0, "launches": int(cnt[l]), "ms": ms[l],
                        "bytes": b * cnt[l], "flops": fl * cnt[l], "level": l}
    roof = roofline_entry(best)
    roof["kernel"] = "%s level %d" % (OPS[best["op"]], best["level"])
    # per level step: microseconds per launch and algorithmic GB/s
    levels = {}
    for op, ph in enumerate(("factor", "forward", "backward")):
        ms, cnt = prof[ph]
        row = []
        for l in range(len(ms)):
            if cnt[l] > 0:
                b, _ = btc.btc_level_work(op, prec, N, n, m, l)
                us = ms[l] / cnt[l] * 1e3
                row.append([l, round(us, 1), round(b / (us * 1e-6) / 1e9, 1)])
        levels[ph] = row
    f.close()
    return {"value": args.steps / wall, "ms_per_step": wall * 1e3 / args.steps, "relres": relres,
            "roofline": roof, "seed": seed, "levels": levels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="served", choices=["served", "single", "copy"])
    ap.add_argument("--clients", type=int, default=256)
    ap.add_argument("--rates", default="1000,10000,50000",
                    help="open-loop Poisson arrival rates (req/s), comma separated; empty: none")
    ap.add_argument("--rate-seconds", type=float, default=1.0)
    ap.add_argument("--rate-requests", type=int, default=50000)
    ap.add_argument("--N", type=int, default=4096)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_ir"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-requests", type=int, default=4096,
                    help="served workload: requests per step (16 per client by default)")
    ap.add_argument("--sweep-ranges", action="store_true",
                    help="served workload: one server tick per sweep level range instead of per level")
    ap.add_argument("--lanes", type=int, default=0,
                    help="served workload: server lanes (0: the library's choice, three; 1: one tick over all "
                         "clients; 2..4: clients split by padded block size class, each lane ticking on its "
                         "own stream)")
    ap.add_argument("--profile-all", action="store_true",
                    help="served workload: time every kernel group in the timed region too and report each "
                         "group's launches and algorithmic bytes over the whole run (group_totals), to set "
                         "hardware traffic counters of the same run against")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other configurations (sweep table, batch, latency per strategy)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every instance is factored and solved on a single device; "
              "runs on more than one GPU are not part of this implementation", file=sys.stderr)
        sys.exit(2)
    args.rates = [int(x) for x in args.rates.split(",") if x.strip()]

    import torch
    from paper_2601_03754_amd import btc
    btc.lib()
    assert torch.cuda.is_available(), "a GPU is required"

    if args.workload == "copy":
        # plain device copy of a known size: the reference for scaling HBM
        # traffic counters (FETCH_SIZE / WRITE_SIZE per dispatch)
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": 2 * nbytes * args.steps / wall / 1e9,
                          "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "copy of a 1 GiB FP64 buffer", "bytes_read_per_step": nbytes,
                                     "bytes_written_per_step": nbytes}}))
        return

    if args.workload == "single":
        r = run_single(args, btc)
        cpu = None
        if not args.no_cpu_baseline:
            import oracle
            from paper_2601_03754_amd import inputs
            oracle.build()
            pr = inputs.block_tridiag(args.N, args.n, c=4.0, seed=r["seed"], nrhs=args.nrhs)
            t0 = time.perf_counter()
            runs = 0
            while time.perf_counter() - t0 < args.cpu_budget or runs == 0:
                Ld, Rb, Tb, _ = oracle.factor_nd(pr.D, pr.E)
                oracle.solve_nd(Ld, Rb, Tb, pr.B)
                runs += 1
            el = time.perf_counter() - t0
            cpu = {"value": runs / el, "unit": "factor+solve/s", "cores": 1, "kind": "oracle",
                   "sample": "%d factor+solve runs of the same instance in %.1f s" % (runs, el)}
        line = {"metric": METRIC, "value": r["value"], "unit": "factor+solve/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
                "config": {"workload": "single instance factor+solve, refactor every step", "N": args.N,
                           "n": args.n, "nrhs": args.nrhs, "diag_shift": 4.0, "precision": args.precision},
                "relres": r["relres"], "roofline": r["roofline"], "cpu_baseline": cpu,
                "levels_us_gbs": r["levels"]}
        print(json.dumps(line))
        return

    shapes, paths, rates = run_served(args, btc)
    mixed, fp64 = paths["mixed"], paths["fp64"]
    extras = None
    if not args.no_extras:
        log("other configurations: sweep table, batch, latency per strategy, conditioning sweep")
        extras = {"sweep_fp64": sweep_table(btc),
                  "batch": batch_rate(btc),
                  "batch_autotuned": batch_rate(btc, tune=True),
                  "latency_n16_n8": latency_strategies(btc),
                  "conditioning_n4096_n64": conditioning_sweep(btc)}
        log("batch: %.0f instances/s, autotuned %.0f" % (extras["batch"]["instances_per_s"],
                                                         extras["batch_autotuned"]["instances_per_s"]))
    cpu = None
    if not args.no_cpu_baseline:
        rate, cnt, el, cores = cpu_baseline_alg1(shapes, args.cpu_budget)
        r1, cnt1, el1, _ = cpu_baseline_served(shapes, args.cpu_budget / 3, wall_cap_s=30.0)
        cpu = {"value": rate, "unit": "req/s", "cores": cores, "kind": "oracle",
               "sample": "Algorithm 1 (natural-order block Cholesky, plain C, FP64) over %d requests of the "
                         "same mix (the first clients' systems, seeded host draws; 30%% refactor + solve, 70%% "
                         "solve against a factor computed beforehand), on all %d host threads, %.1f s wall"
                         % (cnt, cores, el),
               "nd_single_core": {"value": r1, "unit": "req/s", "cores": 1,
                                  "sample": "nested-dissection oracle, one thread, %d requests, %.1f s" % (cnt1, el1)}}
    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "req/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "served: 256 clients, N log-uniform [64, 4096], n uniform {12..96}, nrhs 1, "
                               "70% solve on the resident factor / 30% refactor+solve, closed loop at "
                               "saturation; mixed precision with FP64 refinement to 1e-10",
                   "clients": len(shapes), "step_requests": args.step_requests, "diag_shift": 4.0,
                   "relres_target": RELRES_TARGET,
                   "server_sweeps": "one tick per level range" if args.sweep_ranges else "one tick per level",
                   "server_lanes": mixed["lanes"]},
        "p50_ms": mixed["p50_ms"],
        "p99_ms": mixed["p99_ms"],
        "max_relres_last": mixed["max_relres_last"],
        "fp64_path": {k: fp64[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "max_relres_last")},
        "speedup_vs_fp64": mixed["value"] / fp64["value"],
        "open_loop": rates,
        "paths": paths,
        "roofline": mixed.get("roofline"),
        "roofline_aggregate": mixed.get("aggregate"),
        "cpu_baseline": cpu,
        "configs": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
