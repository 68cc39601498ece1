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


def run_trace(btc, precision, budget, seed=0, clients=6, requests=40, n_choices=(5, 12, 16, 24, 40, 64),
              N_max=300, sweep_ranges=False, lanes=0):
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(16, N_max)), int(rng.choice(n_choices))) for _ in range(clients)]
    mats = [[inputs.block_tridiag(N, n, seed=seed * 100 + c * 10 + v) for v in range(2)]
            for c, (N, n) in enumerate(shapes)]
    dmats = [[(dev(p.D), dev(p.E)) for p in ms] for ms in mats]
    srv = btc.Server(precision=precision, hbm_budget=budget, sweep_ranges=sweep_ranges, lanes=lanes)
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


# block sizes of the served workload's kernels: up to the padded-96 pivot
# kernels that carry most of its time, and the padded-128 ones
BIG_BLOCKS = (12, 33, 64, 80, 96, 110, 128)


@pytest.mark.parametrize("precision,n_choices,ranges,lanes", [
    (0, None, False, 1), (1, None, False, 1), (0, BIG_BLOCKS, False, 1),
    (1, BIG_BLOCKS, False, 1), (2, BIG_BLOCKS, False, 1),
    (0, None, True, 1), (1, BIG_BLOCKS, True, 1), (2, BIG_BLOCKS, True, 1),
    # clients split into lanes by block size class, each lane ticking alone
    # (0: the library's default, three lanes)
    (0, BIG_BLOCKS, False, 4), (1, BIG_BLOCKS, False, 4), (1, None, False, 2), (2, BIG_BLOCKS, True, 3),
    (1, BIG_BLOCKS, False, 0)])
def test_results_in_the_mix_equal_results_alone(btc, precision, n_choices, ranges, lanes):
    """Every result equals the same request alone, bit for bit, in both
    server plans (one tick per sweep level range, or per level) and with the
    clients in one lane or several."""
    kw = {} if n_choices is None else {"n_choices": n_choices, "N_max": 140, "requests": 30}
    kw["sweep_ranges"] = ranges
    kw["lanes"] = lanes
    srv, subs, done, mats, dmats, stats = run_trace(btc, precision, budget=1 << 40, seed=11 + precision, **kw)
    assert len(done) == len(subs)
    assert stats["queued"] == 0 and stats["in_flight"] == 0
    tol = 1e-12 if precision == 0 else 1e-10
    by_ticket = {d["ticket"]: d for d in done}
    for t, c, v, B, X, _ in subs:
        Xm = X.cpu().numpy()
        Xa = alone(btc, dmats[c][v][0], dmats[c][v][1], B, precision)
        assert np.array_equal(Xm, Xa), (t, c)
        p = mats[c][v]
        rr = oracle.relres(p.D, p.E, Xm, B.cpu().numpy())
        assert rr <= tol
        d = by_ticket[t]
        assert d["info"] == 0 and d["converged"], d
        if precision == 0:
            assert d["steps"] == 0 and d["relres"] == -1.0
        else:
            # the completion carries the device's FP64 residual of this result
            assert abs(d["relres"] - rr) <= 1e-3 * rr + 1e-16, (d, rr)
    srv.close()


def test_evicted_solve_uses_the_matrix_admitted_before_it(btc):
    """A solve-only request refers to the matrix of the client's previous
    refactorization, also when the client is evicted before the solve is
    admitted and a later refactorization with another matrix is already
    queued.  Budget: one client at a time."""
    from paper_2601_03754_amd import btc as b
    n, N = 16, 40
    budget = b.btc_footprint_bytes(N, n, 0, 1) + 64
    p1, p2, q = (inputs.block_tridiag(N, n, seed=s) for s in (1, 2, 3))
    srv = btc.Server(precision=0, hbm_budget=budget)
    c0, c1 = srv.add_client(N, n), srv.add_client(N, n)
    A1, A2, Aq = ((dev(p.D), dev(p.E)) for p in (p1, p2, q))
    B = dev(np.random.default_rng(0).standard_normal((N, n, 1)))
    X1, X2, X3, Xq = (torch.full_like(B, np.nan) for _ in range(4))
    t1 = srv.submit(c0, B, X1, A=A1)   # admitted; holds the whole budget
    tq = srv.submit(c1, B, Xq, A=Aq)   # waits for memory, then evicts client 0
    t2 = srv.submit(c0, B, X2)         # solve-only: must use A1
    t3 = srv.submit(c0, B, X3, A=A2)   # a newer matrix, submitted before t2 runs
    srv.step()
    while srv.step() > 0:
        pass
    done = {d["ticket"]: d for d in srv.poll(wait=True)}
    assert set(done) == {t1, tq, t2, t3}
    assert done[t2]["refactored"]      # client 0 was evicted in between
    assert np.array_equal(X2.cpu().numpy(), alone(btc, *A1, B, 0))
    assert np.array_equal(X3.cpu().numpy(), alone(btc, *A2, B, 0))
    assert np.array_equal(Xq.cpu().numpy(), alone(btc, *Aq, B, 0))
    srv.close()


def test_admission_limits(btc):
    """A request whose footprint alone exceeds the budget is refused at
    submission; a client that needs a larger workspace (more right-hand
    sides) evicts idle clients instead of waiting for ever."""
    from paper_2601_03754_amd import btc as b
    n, N = 8, 30
    fp = lambda m: b.btc_footprint_bytes(N, n, 0, m)
    # both clients fit with one right-hand side, not with client 0 at two
    budget = 2 * fp(1) + (fp(2) - fp(1)) // 2
    big = next(m for m in range(2, 100) if fp(m) > budget)
    srv = btc.Server(precision=0, hbm_budget=budget)
    c0, c1 = srv.add_client(N, n), srv.add_client(N, n)
    pa, pb = inputs.block_tridiag(N, n, seed=5), inputs.block_tridiag(N, n, seed=6)
    Aa, Ab = (dev(pa.D), dev(pa.E)), (dev(pb.D), dev(pb.E))
    B1 = dev(np.ones((N, n, 1)))
    B2 = dev(np.ones((N, n, 2)))
    B3 = dev(np.ones((N, n, big)))
    with pytest.raises(btc.BtcError) as ei:
        srv.submit(c0, B3, torch.empty_like(B3), A=Aa)
    assert ei.value.code == btc.BTC_ERR_UNSUPPORTED
    Xa, Xb, Xa2 = torch.empty_like(B1), torch.empty_like(B1), torch.empty_like(B2)
    srv.submit(c0, B1, Xa, A=Aa)
    srv.submit(c1, B1, Xb, A=Ab)
    srv.submit(c0, B2, Xa2)   # grows client 0's workspace: client 1 must be evicted
    for _ in range(10000):
        if srv.step() == 0:
            break
    else:
        raise AssertionError("server did not drain")
    done = srv.poll(wait=True)
    assert len(done) == 3 and all(d["converged"] for d in done)
    ref = oracle.solve(pa.D, pa.E, np.ones((N, n, 2)))
    assert np.abs(Xa2.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    srv.close()


@pytest.mark.parametrize("lanes", [1, 0, 4])
def test_per_client_order_and_latency_fields(btc, lanes):
    srv, subs, done, *_ = run_trace(btc, 0, budget=1 << 40, seed=3, lanes=lanes)
    # one runner per lane (0: the library's three); ticks counted over all lanes
    assert len(srv.runner_handles()) == (3 if lanes == 0 else lanes)
    hs = srv.host_stats()
    assert hs["ticks"] > 0 and hs["wait_s"] >= 0.0
    by_ticket = {d["ticket"]: d for d in done}
    last = {}
    for t, c, *_ in subs:
        d = by_ticket[t]
        assert d["t_submit"] <= d["t_admit"] <= d["t_done"]
        if c in last:
            assert d["t_admit"] >= by_ticket[last[c]]["t_done"]  # one request in flight per client
        last[c] = t
    srv.close()


@pytest.mark.parametrize("lanes", [1, 3])
def test_small_budget_evicts_and_readmits(btc, lanes):
    """A budget that fits about two clients at a time: clients are evicted and
    re-admitted (their solves then refactor with the last matrix), and every
    result still equals the one computed alone."""
    from paper_2601_03754_amd import btc as b
    budget = 2 * b.btc_footprint_bytes(300, 64, 0, 1)
    srv, subs, done, mats, dmats, stats = run_trace(btc, 0, budget=budget, seed=7, lanes=lanes)
    assert len(done) == len(subs)
    assert stats["resident_bytes"] <= budget
    # every request that brought a matrix refactored; evicted clients refactor again
    assert sum(d["refactored"] for d in done) >= sum(1 for s in subs if s[5])
    for t, c, v, B, X, _ in subs:
        Xa = alone(btc, dmats[c][v][0], dmats[c][v][1], B, 0)
        assert np.array_equal(X.cpu().numpy(), Xa)
    srv.close()
