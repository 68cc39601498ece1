"""Pins of the oracle's other elimination orders (section "Parallel Cholesky
Factorization": sequential, single-stage, two-stage, partition), each the
Cholesky factorization of P Psi P^T for its own block permutation P: against
LAPACK's dense Cholesky of the explicitly permuted matrix (the factor is
unique), the structural zeros it predicts, the multi-stage oracle on the
multi-stage order, Proposition 1's chunk sizes (brute force over integer
sizes) and the operation counts of the partition method's cost table."""
import numpy as np
import pytest

import oracle
from paper_2601_03754_amd import inputs


def dense_permuted_factor(D, E, order):
    A = oracle.assemble_dense(D, E)
    N, n, _ = D.shape
    p = ((np.asarray(order) - 1)[:, None] * n + np.arange(n)[None, :]).reshape(-1)
    return np.linalg.cholesky(A[np.ix_(p, p)])


def orders(N):
    out = [("k0", oracle.kstage_order(N, 0), None), ("k1", oracle.kstage_order(N, 1), None),
           ("k2", oracle.kstage_order(N, 2), None), ("k3", oracle.kstage_order(N, 3), None)]
    for p in (2, 3, 4):
        try:
            o, ph = oracle.partition_order(N, p)
            out.append(("p%d" % p, o, ph))
        except ValueError:
            pass
    return out


@pytest.mark.parametrize("N,n", [(1, 3), (2, 2), (3, 4), (5, 3), (7, 2), (20, 3), (31, 2), (33, 3)])
def test_orders_match_dense_cholesky(N, n):
    pr = inputs.block_tridiag(N, n, seed=70 + N + n, nrhs=2)
    for name, order, _ in orders(N):
        assert sorted(order) == list(range(1, N + 1)), name
        Ld, Ro, To, rn, ln, info = oracle.factor_order(pr.D, pr.E, order)
        assert info == 0, name
        Lden = dense_permuted_factor(pr.D, pr.E, order)
        pos = {int(b): q for q, b in enumerate(order)}

        def blk(bi, bj):
            a, c = pos[bi], pos[bj]
            return Lden[a * n:(a + 1) * n, c * n:(c + 1) * n]

        for i in range(1, N + 1):
            assert np.allclose(Ld[i - 1], blk(i, i), rtol=0, atol=1e-13), (name, i)
            below = [j for j in range(1, N + 1) if pos[j] > pos[i]]
            for j in below:
                B = blk(j, i)
                if j == rn[i - 1]:
                    assert np.allclose(Ro[i - 1], B, rtol=0, atol=1e-13), (name, i, j)
                elif j == ln[i - 1]:
                    assert np.allclose(To[i - 1].T, B, rtol=0, atol=1e-13), (name, i, j)
                else:
                    assert np.all(B == 0.0), (name, i, j)   # exact structural zero
        X = oracle.solve_order(order, Ld, Ro, To, rn, ln, pr.B)
        A = oracle.assemble_dense(pr.D, pr.E)
        ref = np.linalg.solve(A, pr.B.reshape(N * n, -1))
        assert np.allclose(X.reshape(N * n, -1), ref, rtol=0, atol=1e-12), name


@pytest.mark.parametrize("N", [1, 2, 3, 16, 20, 33, 64])
def test_multistage_order_reproduces_nd_oracle(N):
    pr = inputs.block_tridiag(N, 3, seed=N)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    L2, Ro, To, rn, ln, info2 = oracle.factor_order(pr.D, pr.E, oracle.nd_order(N))
    assert info == info2 == 0
    assert np.allclose(Ld, L2, rtol=0, atol=1e-13)
    assert np.allclose(Rb, Ro, rtol=0, atol=1e-13)
    assert np.allclose(Tb, To, rtol=0, atol=1e-13)
    assert np.array_equal(oracle.kstage_order(N, oracle.num_levels(N)), oracle.nd_order(N))


@pytest.mark.parametrize("N", [20, 50, 100, 257, 1000])
@pytest.mark.parametrize("p", [2, 3, 4, 8])
def test_partition_sizes_proposition1(N, p):
    """N_1 + (p-1) N_k + (p-1) = N; N_k is N_k* rounded down or up, whichever
    gives the smaller larger phase cost, and no integer N_k does better."""
    try:
        s = oracle.partition_sizes(N, p)
    except ValueError:
        assert N < 2 * p - 1
        return
    assert s.sum() + (p - 1) == N and np.all(s >= 1)
    nk = (7 * N - 7 * p + 7) / (7 * p + 12)
    if p > 1:
        assert np.all(s[1:] == s[1]) and s[1] in (np.floor(nk), np.ceil(nk))
    cost = lambda n1, ck: max(7 / 3 * n1 - 1, 19 / 3 * ck - 1)
    best = min(cost(N - (p - 1) - (p - 1) * c, c) for c in range(1, N) if N - (p - 1) - (p - 1) * c >= 1)
    assert cost(s[0], s[1] if p > 1 else 0) <= best + 1e-9
    if p > 1 and N > 200:
        assert abs(s[0] / s[1] - 19 / 7) < 0.3   # the optimal ratio 19/7


@pytest.mark.parametrize("N,p", [(40, 3), (100, 4), (61, 2), (200, 5)])
def test_partition_cost_table(N, p):
    """Operation counts per chunk against the cost table of section
    "Partition Permutation" (potrf n^3/3, trsm and syrk n^3, gemm 2n^3).  The
    paper defers the product F_k F_k^T onto the next pivot to the sequential
    phase; the elimination here applies it with the chunk's last block, so
    that one syrk per chunk k < p moves between the columns.  The last chunk
    has no right pivot (no F, no H: 3 n^3 less than a middle chunk)."""
    order, phase = oracle.partition_order(N, p)
    sizes = oracle.partition_sizes(N, p)
    pr = inputs.block_tridiag(N, 2, seed=1)
    *_, info, cnt = oracle.factor_order(pr.D, pr.E, order, phase=phase, counts=True)
    assert info == 0
    flops = cnt @ np.array([1 / 3, 1.0, 1.0, 2.0])   # in units of n^3
    assert flops[0] - 1 == pytest.approx(7 / 3 * sizes[0] - 1)
    for k in range(1, p - 1):
        assert flops[k] - 1 == pytest.approx(19 / 3 * sizes[k] - 1)
    if p > 1:
        assert flops[p - 1] == pytest.approx(19 / 3 * sizes[p - 1] - 4)
    assert flops[p] + (p - 1) == pytest.approx(10 / 3 * p - 16 / 3)


@pytest.mark.parametrize("N", [2, 17, 64])
def test_sequential_order_is_algorithm1(N):
    """k = 0 is Algorithm 1: the same blocks as the natural-order oracle."""
    pr = inputs.block_tridiag(N, 3, seed=5)
    Dh, Eh, info = oracle.factor_seq(pr.D, pr.E)
    Ld, Ro, To, rn, ln, info2 = oracle.factor_order(pr.D, pr.E, oracle.kstage_order(N, 0))
    assert info == info2 == 0
    assert np.allclose(Ld, Dh, rtol=0, atol=1e-14)
    for i in range(1, N):
        assert rn[i - 1] == i + 1 and ln[i - 1] == 0
        assert np.allclose(Ro[i - 1], Eh[i - 1], rtol=0, atol=1e-14)
