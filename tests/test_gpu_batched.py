"""Many instances per launch (runner / batched entry points), through the C ABI.

Every instance in a batch goes through the same kernels with the same
per-item arithmetic as when it is factored alone, so its factor and solution
must equal its single-instance results bit for bit; the single-instance
results themselves are checked against the FP64 oracle."""
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


def single(btc, pr, precision):
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=precision)
    X = f.solve(dev(pr.B))
    torch.cuda.synchronize()
    out = (X.cpu().numpy(), f.export(), f.info)
    f.close()
    return out


def make_batch(count, seed, n_choices=(3, 8, 13, 16, 24, 32, 48, 64), N_max=300, nrhs=1):
    rng = np.random.default_rng(seed)
    prs = []
    for k in range(count):
        N = int(rng.integers(1, N_max + 1))
        n = int(rng.choice(n_choices))
        prs.append(inputs.block_tridiag(N, n, seed=seed * 1000 + k, nrhs=nrhs))
    return prs


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_single_bitwise(btc, precision):
    prs = make_batch(24, seed=5 + precision)
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, precision) for p in prs]
    Ds = [dev(p.D) for p in prs]
    Es = [dev(p.E) for p in prs]
    Bs = [dev(p.B) for p in prs]
    Xs = [torch.empty_like(b) for b in Bs]
    r.factor_batched(hs, Ds, Es)
    r.solve_batched(hs, Bs, Xs, 1)
    r.sync()
    tol = 1e-12 if precision == 0 else 1e-10
    for k, p in enumerate(prs):
        assert btc.btc_status(hs[k]) == 0
        Xb = Xs[k].cpu().numpy()
        Xsng, blocks_s, info_s = single(btc, p, precision)
        assert info_s == 0
        assert np.array_equal(Xb, Xsng), (k, p.N, p.n)
        blocks_b = btc.btc_export_factor(hs[k], p.N, p.n)
        assert all(np.array_equal(a, b) for a, b in zip(blocks_b, blocks_s))
        assert oracle.relres(p.D, p.E, Xb, p.B) <= tol
        if precision == 1:
            info = btc.btc_refine_info(hs[k])
            assert info["converged"], info
    for h in hs:
        btc.btc_destroy(h)
    r.close()


def test_runner_steps_at_different_levels_in_one_launch(btc):
    """Continuous batching: instance B starts its factorization while A is
    mid-tree; each runner call carries one step per instance at different
    levels (and, later, different operations)."""
    pa = inputs.block_tridiag(200, 24, seed=1)
    pb = inputs.block_tridiag(77, 16, seed=2)
    r = btc.Runner()
    ha = btc.btc_create(pa.N, pa.n)
    hb = btc.btc_create(pb.N, pb.n)
    Da, Ea, Ba = dev(pa.D), dev(pa.E), dev(pa.B)
    Db, Eb, Bb = dev(pb.D), dev(pb.E), dev(pb.B)
    Xa, Xb = torch.empty_like(Ba), torch.empty_like(Bb)
    La, Lb = int(np.log2(pa.N)) + 1, int(np.log2(pb.N)) + 1

    def plan(h, D, E, B, X, L):
        s = [btc.step(h, btc.BTC_OP_FACTOR, l, D, E) for l in range(L)]
        s += [btc.step(h, btc.BTC_OP_FORWARD, l, B=B, X=X, nrhs=1) for l in range(L)]
        s += [btc.step(h, btc.BTC_OP_BACKWARD, l, B=B, X=X, nrhs=1) for l in reversed(range(L))]
        return s

    qa = plan(ha, Da, Ea, Ba, Xa, La)
    qb = [None] * 3 + plan(hb, Db, Eb, Bb, Xb, Lb)  # B arrives three ticks later
    btc.runner_host_stats(r.handle, reset=True)
    ticks = max(len(qa), len(qb))
    for t in range(ticks):
        batch = [q[t] for q in (qa, qb) if t < len(q) and q[t] is not None]
        r.run(batch)
    r.sync()
    # the host-time counters: one call per tick, the wait part of the total
    hs = btc.runner_host_stats(r.handle, reset=True)
    assert hs["calls"] == ticks
    assert 0.0 < hs["run_s"] and 0.0 <= hs["wait_s"] <= hs["run_s"]
    assert btc.runner_host_stats(r.handle) == {"run_s": 0.0, "wait_s": 0.0, "calls": 0}
    for p, X, h in ((pa, Xa, ha), (pb, Xb, hb)):
        Xs, _, _ = single(btc, p, 0)
        assert np.array_equal(X.cpu().numpy(), Xs)
        assert oracle.relres(p.D, p.E, X.cpu().numpy(), p.B) <= 1e-12
        btc.btc_destroy(h)
    r.close()


def test_batch_shapes_of_many_instance_workload(btc):
    """A reduced draw of the many-instance workload (N in [32, 2048], n in
    {8, 16, 24, 32, 48}), FP32 factors with FP64 refinement, every instance
    to <= 1e-10 relative residual."""
    shapes = inputs.batch_shapes(48, seed=0)
    prs = [inputs.block_tridiag(N, n, seed=k, nrhs=1) for k, (N, n) in enumerate(shapes)]
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, btc.BTC_FP32_IR) for p in prs]
    Bs = [dev(p.B) for p in prs]
    Xs = [torch.empty_like(b) for b in Bs]
    Ds, Es = [dev(p.D) for p in prs], [dev(p.E) for p in prs]
    r.factor_batched(hs, Ds, Es)
    r.solve_batched(hs, Bs, Xs, 1)
    r.sync()
    for k, p in enumerate(prs):
        assert btc.btc_refine_info(hs[k])["converged"]
        assert oracle.relres(p.D, p.E, Xs[k].cpu().numpy(), p.B) <= 1e-10
        btc.btc_destroy(hs[k])
    r.close()


@pytest.mark.parametrize("precision,N,n,m", [(0, 300, 24, 2), (1, 300, 24, 2), (0, 1, 8, 1), (1, 37, 96, 1),
                                             (0, 4096, 16, 1), (1, 1000, 40, 3)])
def test_level_ranges_equal_single_levels(btc, precision, N, n, m):
    """A sweep run one level per step and the same sweep in the library's
    level ranges (one launch per range of elimination subtrees) do the same
    arithmetic per node: identical results, bit for bit."""
    pr = inputs.block_tridiag(N, n, seed=N + n + m, nrhs=m)
    D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
    f = btc.Factor(D, E, precision=precision)
    Xr = f.solve(B)                     # level ranges
    torch.cuda.synchronize()
    r = btc.Runner()
    X1 = torch.full_like(B, float("nan"))
    L = int(np.floor(np.log2(N))) + 1
    S = btc.step
    if precision == 0:
        plan = [[S(f.handle, btc.BTC_OP_FORWARD, l, B=B, X=X1, nrhs=m)] for l in range(L)]
        plan += [[S(f.handle, btc.BTC_OP_BACKWARD, l, B=B, X=X1, nrhs=m)] for l in reversed(range(L))]
    else:
        plan = [[S(f.handle, btc.BTC_OP_REFINE_INIT, 0, B=B, X=X1, nrhs=m)]]
        for rnd in range(1 + 4):
            plan += [[S(f.handle, btc.BTC_OP_FORWARD, l, B=B, X=X1, nrhs=m, first=rnd == 0)] for l in range(L)]
            plan += [[S(f.handle, btc.BTC_OP_BACKWARD, l, B=B, X=X1, nrhs=m, first=rnd == 0)]
                     for l in reversed(range(L))]
            plan += [[S(f.handle, btc.BTC_OP_RESIDUAL, 0, B=B, X=X1, nrhs=m),
                      S(f.handle, btc.BTC_OP_REFINE_TEST, 0, B=B, X=X1, nrhs=m)]]
    for call in plan:
        r.run(call)
    r.sync()
    assert np.array_equal(X1.cpu().numpy(), Xr.cpu().numpy())
    # and a whole refinement round in one call, stage by stage
    if precision == 1:
        b = btc.btc_sweep_ranges(N)
        X2 = torch.full_like(B, float("nan"))
        for rnd in range(1 + 4):
            call = [] if rnd else [S(f.handle, btc.BTC_OP_REFINE_INIT, 0, B=B, X=X2, nrhs=m, stage=0)]
            st = 1
            for q in range(len(b) - 1):
                call.append(S(f.handle, btc.BTC_OP_FORWARD, b[q], B=B, X=X2, nrhs=m, first=rnd == 0,
                              level_end=b[q + 1] if b[q + 1] > b[q] + 1 else 0, stage=st))
                st += 1
            for q in reversed(range(len(b) - 1)):
                call.append(S(f.handle, btc.BTC_OP_BACKWARD, b[q], B=B, X=X2, nrhs=m, first=rnd == 0,
                              level_end=b[q + 1] if b[q + 1] > b[q] + 1 else 0, stage=min(st, 7)))
                st += 1
            if st > 7:
                pytest.skip("more ranges than stages")
            call.append(S(f.handle, btc.BTC_OP_RESIDUAL, 0, B=B, X=X2, nrhs=m, stage=st))
            call.append(S(f.handle, btc.BTC_OP_REFINE_TEST, 0, B=B, X=X2, nrhs=m, stage=st))
            r.run(call)
        r.sync()
        assert np.array_equal(X2.cpu().numpy(), Xr.cpu().numpy())
    r.close()
    f.close()
