"""Large blocks (65 <= n <= 128: the tile-parallel factorization and the
two-rows-per-lane sweeps and residual) through the C ABI, against the FP64
CPU oracle.

FP64: factor blocks element by element within 1e-12 of the oracle's (relative
to the largest |L| entry), solution within 1e-12 of the oracle's, oracle FP64
relative residual <= 1e-12.  Mixed (BTC_FP32_IR): FP32 factor blocks within
1e-4, refined solution to <= 1e-10 relative residual.  Shapes span one and
several 16/32-row tiles, ragged tails (n not a multiple of 16), both padded
sizes (96 and 128), N = 1 and ragged N."""
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
    assert torch.cuda.is_available()
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# (700, 96) and (600, 81): more than 256 nodes at level 0, so the pivot kernel
# runs in both of its launch shapes (throughput shape at level 0, latency
# shape above)
SHAPES = [(1, 65), (2, 96), (3, 128), (7, 80), (16, 96), (21, 100), (33, 128), (40, 127), (64, 65), (100, 112),
          (700, 96), (600, 81)]


@pytest.mark.parametrize("N,n", SHAPES)
def test_fp64_large_blocks_match_oracle(btc, N, n):
    pr = inputs.block_tridiag(N, n, seed=3000 + 11 * N + n, nrhs=2)
    f = btc.Factor(dev(pr.D), dev(pr.E))
    X = f.solve(dev(pr.B)).cpu().numpy()
    assert f.info == 0
    blocks = f.export()
    f.close()
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    assert info == 0
    scale = max(np.abs(Ld).max(), 1.0)
    for name, g, o in zip("LRT", blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= 1e-12 * scale, name
    Xo = oracle.solve(pr.D, pr.E, pr.B)
    assert np.abs(X - Xo).max() <= 1e-12 * max(1.0, np.abs(Xo).max())
    assert oracle.relres(pr.D, pr.E, X, pr.B) <= 1e-12


@pytest.mark.parametrize("N,n", [(1, 70), (9, 96), (33, 128), (50, 90), (129, 120), (700, 96)])
def test_mixed_large_blocks_refine_to_target(btc, N, n):
    pr = inputs.block_tridiag(N, n, seed=4000 + N + n, nrhs=1)
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=btc.BTC_FP32_IR)
    X, info = f.solve(dev(pr.B), want_info=True)
    X = X.cpu().numpy()
    assert f.info == 0
    blocks = f.export()
    f.close()
    assert info["converged"], info
    rr = oracle.relres(pr.D, pr.E, X, pr.B)
    assert rr <= 1e-10
    assert abs(info["relres"] - rr) <= 0.5 * rr + 1e-15
    Ld, Rb, Tb, _ = oracle.factor_nd(pr.D, pr.E)
    scale = max(np.abs(Ld).max(), 1.0)
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= 1e-4 * scale


def test_upper_triangle_ignored_large(btc):
    pr = inputs.block_tridiag(13, 100, seed=8)
    D = pr.D.copy()
    D += np.triu(np.full((100, 100), 1e3), 1)[None]
    f = btc.Factor(dev(D), dev(pr.E))
    X = f.solve(dev(pr.B)).cpu().numpy()
    f.close()
    assert oracle.relres(pr.D, pr.E, X, pr.B) <= 1e-12


@pytest.mark.parametrize("case", ["leading", "trailing", "updated"])
def test_breakdown_large_blocks(btc, case):
    """The pivot factorization runs in two stages (leading 64 rows, then the
    trailing rows); a breakdown in either, or one that appears only after the
    Schur updates, reports the oracle's failing block."""
    N, n = 8, 96
    pr = inputs.block_tridiag(N, n, seed=4)
    D = pr.D.copy()
    if case == "leading":
        D[4] = -np.eye(n)
        expect = 5
    elif case == "trailing":
        d = np.ones(n)
        d[80:] = -1.0
        D[2] = np.diag(d)
        expect = 3
    else:
        D[3] = 1e-3 * np.eye(n)
        expect = 4
    *_, oinfo = oracle.factor_nd(D, pr.E)
    assert oinfo == expect
    for prec in (btc.BTC_FP64, btc.BTC_FP32_IR):
        f = btc.Factor(dev(D), dev(pr.E), precision=prec)
        assert f.info == expect
        f.close()


def test_large_fp64_sizes_residual(btc):
    """Padded-128 blocks at a size with many nodes per level: residual by the
    oracle's FP64 matvec, level-0 blocks checked one by one."""
    N, n = 1024, 128
    pr = inputs.block_tridiag(N, n, c=4.0, seed=inputs.sweep_seed(N, n), nrhs=1)
    f = btc.Factor(dev(pr.D), dev(pr.E))
    X = f.solve(dev(pr.B)).cpu().numpy()
    assert f.info == 0
    Ld, Rb, Tb = f.export()
    f.close()
    assert oracle.relres(pr.D, pr.E, X, pr.B) <= 1e-12
    rng = np.random.default_rng(1)
    for i in rng.choice(np.arange(3, N, 2), size=4, replace=False):
        L, linfo = oracle.dense_chol(np.tril(pr.D[i - 1]) + np.tril(pr.D[i - 1], -1).T)
        assert linfo == 0
        assert np.abs(Ld[i - 1] - L).max() <= 1e-12 * np.abs(L).max()
        R = np.linalg.solve(L, pr.E[i - 1].T).T
        T = np.linalg.solve(L, pr.E[i - 2])
        assert np.abs(Rb[i - 1] - R).max() <= 1e-12 * max(1.0, np.abs(R).max())
        assert np.abs(Tb[i - 1] - T).max() <= 1e-12 * max(1.0, np.abs(T).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_large_equals_single_bitwise(btc, precision):
    """Runner batches mixing small and large blocks and different levels in
    one launch: every instance equals its single-instance result bit for bit."""
    rng = np.random.default_rng(9 + precision)
    prs = []
    for k in range(10):
        N = int(rng.integers(1, 120))
        n = int(rng.choice([24, 64, 70, 96, 128]))
        prs.append(inputs.block_tridiag(N, n, seed=500 + k, nrhs=1))
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, precision) for p in prs]
    Ds, Es, Bs = [dev(p.D) for p in prs], [dev(p.E) for p in prs], [dev(p.B) for p in prs]
    Xs = [torch.empty_like(b) for b in Bs]
    r.factor_batched(hs, Ds, Es)
    r.solve_batched(hs, Bs, Xs, 1)
    r.sync()
    tol = 1e-12 if precision == 0 else 1e-10
    for k, p in enumerate(prs):
        assert btc.btc_status(hs[k]) == 0
        f = btc.Factor(Ds[k], Es[k], precision=precision)
        Xsng = f.solve(Bs[k]).cpu().numpy()
        bs = f.export()
        f.close()
        assert np.array_equal(Xs[k].cpu().numpy(), Xsng), (k, p.N, p.n)
        bb = btc.btc_export_factor(hs[k], p.N, p.n)
        assert all(np.array_equal(a, b) for a, b in zip(bb, bs))
        assert oracle.relres(p.D, p.E, Xsng, p.B) <= tol
    for h in hs:
        btc.btc_destroy(h)
    r.close()


@pytest.mark.parametrize("N,n", [(4096, 64), (1024, 128), (16384, 32)])
def test_full_size_device_residual(btc, N, n):
    """At the full benchmark sizes, the device's FP64 residual of the first,
    unrefined FP32 iterate (tolerance 1: no correction) matches the oracle's
    residual of the same iterate to 1e-6 relative."""
    pr = inputs.block_tridiag(N, n, c=4.0, seed=inputs.sweep_seed(N, n), nrhs=1)
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=btc.BTC_FP32_IR, tol=1.0)
    X, info = f.solve(dev(pr.B), want_info=True)
    f.close()
    assert info["converged"] and info["steps"] == 0, info
    rr = oracle.relres(pr.D, pr.E, X.cpu().numpy(), pr.B)
    assert rr > 1e-12
    assert abs(info["relres"] - rr) <= 1e-6 * rr, (info["relres"], rr)
