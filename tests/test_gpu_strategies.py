"""Elimination orders other than the multi-stage one (section "Parallel
Cholesky Factorization"): the k-stage orders (k = 0: sequential Algorithm 1,
1: single-stage, 2: two-stage) and the partition order (Algorithm 2 with
Proposition 1's chunk sizes) through the C ABI, against the oracle's
factorization in the same order (the factor of that permuted matrix is
unique) and its solution; the AUTO choice and its timing."""
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


SHAPES = [(1, 3), (2, 8), (3, 5), (5, 16), (16, 8), (20, 24), (33, 40), (100, 16), (64, 64), (7, 1), (257, 12)]


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("N,n", SHAPES)
def test_kstage_matches_oracle(btc, k, N, n):
    pr = inputs.block_tridiag(N, n, seed=900 + 7 * N + n + k, nrhs=2)
    D = pr.D + np.triu(np.full((n, n), 55.0), 1)[None]     # upper triangles are never read
    f = btc.Factor(dev(D), dev(pr.E), strategy=btc.BTC_STRATEGY_KSTAGE, stages=k)
    X = f.solve(dev(pr.B)).cpu().numpy()
    assert f.info == 0
    Ld, Rb, Tb = f.export()
    f.close()
    order = oracle.kstage_order(N, k)
    oL, oR, oT, rn, ln, info = oracle.factor_order(pr.D, pr.E, order)
    assert info == 0
    sc = max(1.0, np.abs(oL).max())
    assert np.abs(Ld - oL).max() <= 1e-12 * sc
    assert np.abs(Rb - oR).max() <= 1e-12 * max(1.0, np.abs(oR).max())
    assert np.abs(Tb - oT).max() <= 1e-12 * max(1.0, np.abs(oT).max())
    Xo = oracle.solve_order(order, oL, oR, oT, rn, ln, pr.B)
    assert np.abs(X - Xo).max() <= 1e-12 * max(1.0, np.abs(Xo).max())
    assert oracle.relres(pr.D, pr.E, X, pr.B) <= 1e-12


def test_kstage_breakdown_index(btc):
    """Breakdown in the chain: the status names the failing block."""
    N, n = 12, 4
    pr = inputs.block_tridiag(N, n, seed=3)
    D = pr.D.copy()
    D[7] = -np.eye(n)   # block 8: a chain block for k = 0, 1, 2, 3
    for k in (0, 2):
        *_, oinfo = oracle.factor_order(D, pr.E, oracle.kstage_order(N, k))
        f = btc.Factor(dev(D), dev(pr.E), strategy=btc.BTC_STRATEGY_KSTAGE, stages=k)
        assert f.info == oinfo == 8
        f.close()


def test_kstage_refuses_unsupported(btc):
    pr = inputs.block_tridiag(8, 70, seed=1)
    with pytest.raises(btc.BtcError) as ei:
        btc.Factor(dev(pr.D), dev(pr.E), strategy=btc.BTC_STRATEGY_KSTAGE, stages=0)
    assert ei.value.code == btc.BTC_ERR_UNSUPPORTED
    pr = inputs.block_tridiag(8, 8, seed=1)
    with pytest.raises(btc.BtcError):
        btc.Factor(dev(pr.D), dev(pr.E), precision=btc.BTC_FP32_IR, strategy=btc.BTC_STRATEGY_KSTAGE)
    # stages beyond the tree height: the multi-stage order itself
    f = btc.Factor(dev(pr.D), dev(pr.E), strategy=btc.BTC_STRATEGY_KSTAGE, stages=9)
    Ld, _, _ = f.export()
    f.close()
    assert np.allclose(Ld, oracle.factor_nd(pr.D, pr.E)[0], rtol=0, atol=1e-12)


def test_auto_strategy_takes_the_fastest(btc):
    """Autotuning the order for the smallest benchmark shape (N = 16, n = 8):
    the AUTO choice is the measured fastest, and its result is correct."""
    pr = inputs.block_tridiag(16, 8, seed=0, nrhs=1)
    D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
    X = torch.empty_like(B)
    ms = btc.btc_autotune_strategy(D, E, B, X, reps=20)
    cands = [(t, c) for c, t in enumerate(ms) if t > 0]
    assert len(cands) == 6
    best = min(cands)[1]
    s, k = btc.btc_select_strategy(16, 8)
    want = [(btc.BTC_STRATEGY_MULTISTAGE, 0), (btc.BTC_STRATEGY_KSTAGE, 0), (btc.BTC_STRATEGY_KSTAGE, 1),
            (btc.BTC_STRATEGY_KSTAGE, 2), (btc.BTC_STRATEGY_PARTITION, 2), (btc.BTC_STRATEGY_PARTITION, 4)][best]
    assert (s, k) == want
    f = btc.Factor(D, E, strategy=btc.BTC_STRATEGY_AUTO)
    Xa = f.solve(B).cpu().numpy()
    f.close()
    assert oracle.relres(pr.D, pr.E, Xa, pr.B) <= 1e-12
    print("strategy ms [multistage, k0, k1, k2, p2, p4]:", ms)


PART_SHAPES = [(3, 4, 2), (5, 8, 2), (16, 8, 2), (16, 8, 4), (40, 24, 3), (101, 16, 4), (64, 64, 2), (257, 12, 8),
               (9, 1, 4), (30, 40, 5)]


@pytest.mark.parametrize("N,n,p", PART_SHAPES)
def test_partition_matches_oracle(btc, N, n, p):
    pr = inputs.block_tridiag(N, n, seed=700 + 5 * N + n + p, nrhs=2)
    D = pr.D + np.triu(np.full((n, n), 33.0), 1)[None]     # upper triangles are never read
    f = btc.Factor(dev(D), dev(pr.E), strategy=btc.BTC_STRATEGY_PARTITION, stages=p)
    X = f.solve(dev(pr.B)).cpu().numpy()
    assert f.info == 0
    Ld, Rb, Tb = f.export()
    f.close()
    order, _ = oracle.partition_order(N, p)
    oL, oR, oT, rn, ln, info = oracle.factor_order(pr.D, pr.E, order)
    assert info == 0
    assert np.abs(Ld - oL).max() <= 1e-12 * max(1.0, np.abs(oL).max())
    assert np.abs(Rb - oR).max() <= 1e-12 * max(1.0, np.abs(oR).max())
    assert np.abs(Tb - oT).max() <= 1e-12 * max(1.0, np.abs(oT).max())
    Xo = oracle.solve_order(order, oL, oR, oT, rn, ln, pr.B)
    assert np.abs(X - Xo).max() <= 1e-12 * max(1.0, np.abs(Xo).max())
    assert oracle.relres(pr.D, pr.E, X, pr.B) <= 1e-12


def test_partition_breakdown_and_limits(btc):
    N, n, p = 21, 4, 3
    pr = inputs.block_tridiag(N, n, seed=4)
    order, _ = oracle.partition_order(N, p)
    for bad in (3, 12, 20):   # in the first chunk, the first separator, in the last chunk
        D = pr.D.copy()
        D[bad - 1] = -np.eye(n)
        *_, oinfo = oracle.factor_order(D, pr.E, order)
        f = btc.Factor(dev(D), dev(pr.E), strategy=btc.BTC_STRATEGY_PARTITION, stages=p)
        assert f.info == oinfo > 0
        f.close()
    # too few blocks for the chunks, mixed precision, blocks above 64: refused
    with pytest.raises(btc.BtcError) as ei:
        btc.Factor(dev(pr.D[:3]), dev(pr.E[:2]), strategy=btc.BTC_STRATEGY_PARTITION, stages=4)
    assert ei.value.code == btc.BTC_ERR_UNSUPPORTED
    with pytest.raises(btc.BtcError):
        btc.Factor(dev(pr.D), dev(pr.E), precision=btc.BTC_FP32_IR, strategy=btc.BTC_STRATEGY_PARTITION, stages=2)
