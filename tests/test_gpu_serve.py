"""Continuous-batching server through the C ABI: every result equals the same
request computed alone (bit for bit: the per-item arithmetic does not depend
on what else shares a launch), requests of one client complete in order, and
an HBM budget smaller than the working set forces evictions and re-admission
without changing any result."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    b.lib()
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def alone(btc, D, E, B, precision):
    f = btc.Factor(D, E, precision=precision)
    X = f.solve(B)
    torch.cuda.synchronize()
    out = X.cpu().numpy()
    f.close()
    return out


def run_trace(btc, precision, budget, seed=0, clients=6, requests=40):
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(16, 300)), int(rng.choice([5, 12, 16, 24, 40, 64]))) for _ in range(clients)]
    mats = [[inputs.block_tridiag(N, n, seed=seed * 100 + c * 10 + v) for v in range(2)]
            for c, (N, n) in enumerate(shapes)]
    dmats = [[(dev(p.D), dev(p.E)) for p in ms] for ms in mats]
    srv = btc.Server(precision=precision, hbm_budget=budget)
    ids = [srv.add_client(N, n) for N, n in shapes]
    current = [None] * clients
    subs = []
    for k in range(requests):
        c = int(rng.integers(0, clients))
        refactor = current[c] is None or rng.random() < 0.3
        if refactor:
            current[c] = int(rng.integers(0, 2))
        p = mats[c][current[c]]
        B = dev(rng.standard_normal((p.N, p.n, 1)))
        X = torch.full_like(B, np.nan)
        t = srv.submit(ids[c], B, X, A=dmats[c][current[c]] if refactor else None)
        subs.append((t, c, current[c], B, X, refactor))
        if k % 3 == 0:
            srv.step()
    done = []
    while srv.step() > 0:
        done += srv.poll()
    done += srv.poll(wait=True)
    stats = srv.stats()
    return srv, subs, done, mats, dmats, stats


@pytest.mark.parametrize("precision", [0, 1])
def test_results_in_the_mix_equal_results_alone(btc, precision):
    srv, subs, done, mats, dmats, stats = run_trace(btc, precision, budget=1 << 40)
    assert len(done) == len(subs)
    assert stats["queued"] == 0 and stats["in_flight"] == 0
    tol = 1e-12 if precision == 0 else 1e-10
    for t, c, v, B, X, _ in subs:
        Xm = X.cpu().numpy()
        Xa = alone(btc, dmats[c][v][0], dmats[c][v][1], B, precision)
        assert np.array_equal(Xm, Xa), (t, c)
        p = mats[c][v]
        assert oracle.relres(p.D, p.E, Xm, B.cpu().numpy()) <= tol
    srv.close()


def test_per_client_order_and_latency_fields(btc):
    srv, subs, done, *_ = run_trace(btc, 0, budget=1 << 40, seed=3)
    by_ticket = {d["ticket"]: d for d in done}
    last = {}
    for t, c, *_ in subs:
        d = by_ticket[t]
        assert d["t_submit"] <= d["t_admit"] <= d["t_done"]
        if c in last:
            assert d["t_admit"] >= by_ticket[last[c]]["t_done"]  # one request in flight per client
        last[c] = t
    srv.close()


def test_small_budget_evicts_and_readmits(btc):
    """A budget that fits about two clients at a time: clients are evicted and
    re-admitted (their solves then refactor with the last matrix), and every
    result still equals the one computed alone."""
    from paper_2601_03754_amd import btc as b
    budget = 2 * b.btc_footprint_bytes(300, 64, 0, 1)
    srv, subs, done, mats, dmats, stats = run_trace(btc, 0, budget=budget, seed=7)
    assert len(done) == len(subs)
    assert stats["resident_bytes"] <= budget
    # every request that brought a matrix refactored; evicted clients refactor again
    assert sum(d["refactored"] for d in done) >= sum(1 for s in subs if s[5])
    for t, c, v, B, X, _ in subs:
        Xa = alone(btc, dmats[c][v][0], dmats[c][v][1], B, 0)
        assert np.array_equal(X.cpu().numpy(), Xa)
    srv.close()
