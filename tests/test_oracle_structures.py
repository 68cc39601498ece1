"""Pins of the block-banded and arrow oracle (oracle/structures.py) against
LAPACK on the assembled dense matrices, LAPACK's banded solver, and the
special cases that reduce to the block-tridiagonal method.  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import structures as st
from paper_2601_03754_amd import inputs


def dense_band(A_band, b):
    """The block-banded matrix written out from its definition: block (i, j)
    = A_band[i, i-j] for 0 <= i-j <= b, its transpose above the diagonal."""
    N, _, n, _ = A_band.shape
    A = np.zeros((N * n, N * n))
    for i in range(N):
        for k in range(b + 1):
            j = i - k
            if j < 0:
                continue
            blk = A_band[i, k]
            if k == 0:
                blk = np.tril(blk) + np.tril(blk, -1).T
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] = blk
            A[j * n:(j + 1) * n, i * n:(i + 1) * n] = blk.T
    return A


@pytest.mark.parametrize("N,n,b", [(7, 3, 2), (9, 2, 3), (8, 3, 4), (5, 2, 1), (3, 2, 5)])
def test_super_blocks_hold_the_band(N, n, b):
    pr = inputs.block_banded(N, n, b, seed=N * 10 + b)
    D2, E2 = st.band_to_tridiag(pr.A_band, b)
    N2 = -(-N // b)
    assert D2.shape == (N2, b * n, b * n) and E2.shape == (max(N2 - 1, 0), b * n, b * n)
    A2 = oracle.assemble_dense(D2, E2)
    K = N * n
    np.testing.assert_array_equal(A2[:K, :K], dense_band(pr.A_band, b))
    # identity completion, decoupled from the band
    np.testing.assert_array_equal(A2[K:, K:], np.eye(A2.shape[0] - K))
    np.testing.assert_array_equal(A2[K:, :K], 0.0)


def test_band_of_width_one_is_the_tridiagonal_matrix():
    pr = inputs.block_banded(11, 4, 1, seed=3)
    D2, E2 = st.band_to_tridiag(pr.A_band, 1)
    D = pr.A_band[:, 0]
    np.testing.assert_array_equal(np.tril(D2), np.tril(D))
    np.testing.assert_array_equal(E2, pr.A_band[1:, 1])
    X = st.banded_solve(pr.A_band, 1, pr.B)
    np.testing.assert_array_equal(X, oracle.solve(D, pr.A_band[1:, 1], pr.B))


@pytest.mark.parametrize("N,n,b,m", [(7, 3, 2, 2), (10, 2, 3, 1), (6, 4, 4, 3), (13, 1, 5, 2)])
def test_banded_solve_matches_lapack(N, n, b, m):
    pr = inputs.block_banded(N, n, b, seed=100 + N, nrhs=m)
    A = dense_band(pr.A_band, b)
    want = sla.solve(A, pr.B.reshape(N * n, m), assume_a="pos")
    got = st.banded_solve(pr.A_band, b, pr.B).reshape(N * n, m)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_scalar_band_matches_lapack_banded_solver():
    # n = 1: a scalar SPD band matrix of bandwidth b (LAPACK dpbsv)
    N, b = 57, 6
    pr = inputs.block_banded(N, 1, b, seed=5, nrhs=2)
    ab = np.zeros((b + 1, N))
    for i in range(N):
        for k in range(b + 1):
            if i - k >= 0:
                ab[k, i - k] = pr.A_band[i, k, 0, 0]
    want = sla.solveh_banded(ab, pr.B.reshape(N, 2), lower=True)
    got = st.banded_solve(pr.A_band, b, pr.B).reshape(N, 2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_banded_factor_is_the_cholesky_factor_of_the_permuted_super_block_matrix():
    N, n, b = 11, 2, 3
    pr = inputs.block_banded(N, n, b, seed=9)
    D2, E2 = st.band_to_tridiag(pr.A_band, b)
    N2, n2 = D2.shape[0], D2.shape[1]
    perm = oracle.perm_indices(N2, n2)
    A2 = oracle.assemble_dense(D2, E2)
    L = np.linalg.cholesky(A2[np.ix_(perm, perm)])
    Ld, Rb, Tb = oracle.dense_factor_blocks(L, N2, n2)
    gL, gR, gT, info = st.banded_factor(pr.A_band, b)
    assert info == 0
    for got, want in ((gL, Ld), (gR, Rb), (gT, Tb)):
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_band_recipe_margin():
    # block Gershgorin shift: the smallest eigenvalue is at least c
    pr = inputs.block_banded(9, 3, 2, c=0.5, seed=1)
    w = np.linalg.eigvalsh(dense_band(pr.A_band, 2))
    assert w[0] >= 0.5 - 1e-12


@pytest.mark.parametrize("N,n,m,q", [(9, 3, 4, 2), (16, 2, 1, 1), (5, 4, 7, 3), (1, 3, 2, 1)])
def test_arrow_solve_matches_lapack(N, n, m, q):
    pr = inputs.arrow(N, n, m, seed=N + m, nrhs=q)
    A = st.assemble_arrow_dense(pr.D, pr.E, pr.F, pr.C)
    want = sla.solve(A, pr.B, assume_a="pos")
    fac = st.arrow_factor(pr.D, pr.E, pr.F, pr.C)
    assert fac["info_psi"] == 0 and fac["info_tip"] == 0
    got = st.arrow_solve(fac, pr.B)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_arrow_tip_is_the_trailing_block_of_the_permuted_cholesky():
    N, n, m = 13, 2, 5
    pr = inputs.arrow(N, n, m, seed=4)
    A = st.assemble_arrow_dense(pr.D, pr.E, pr.F, pr.C)
    perm = np.concatenate([oracle.perm_indices(N, n), N * n + np.arange(m)])
    L = np.linalg.cholesky(A[np.ix_(perm, perm)])
    fac = st.arrow_factor(pr.D, pr.E, pr.F, pr.C)
    np.testing.assert_allclose(fac["Ls"], L[-m:, -m:], rtol=0, atol=1e-12)
    # the border rows of the factor: F^T (P^T L^{-T}) in the permuted order
    W = L[-m:, :N * n]
    Fp = fac["F"][oracle.perm_indices(N, n)]
    np.testing.assert_allclose(W @ W.T, Fp.T @ np.linalg.solve(A[np.ix_(perm[:N * n], perm[:N * n])], Fp),
                               rtol=0, atol=1e-12)
    np.testing.assert_allclose(fac["S"], A[-m:, -m:] - W @ W.T, rtol=0, atol=1e-12)


def test_arrow_special_cases():
    N, n = 8, 3
    # no border: the block-tridiagonal solve
    pr = inputs.arrow(N, n, 0, seed=2, nrhs=2)
    fac = st.arrow_factor(pr.D, pr.E, pr.F, pr.C)
    got = st.arrow_solve(fac, pr.B)
    np.testing.assert_array_equal(got, oracle.solve(pr.D, pr.E, pr.B.reshape(N, n, 2)).reshape(N * n, 2))
    # zero coupling: the tip is C itself
    pr = inputs.arrow(N, n, 3, seed=2, nrhs=1)
    F0 = np.zeros_like(pr.F)
    fac = st.arrow_factor(pr.D, pr.E, F0, pr.C)
    np.testing.assert_allclose(fac["Ls"], np.linalg.cholesky(np.tril(pr.C) + np.tril(pr.C, -1).T), rtol=0,
                               atol=1e-13)
    x = st.arrow_solve(fac, pr.B)
    np.testing.assert_allclose(x[N * n:], np.linalg.solve(np.tril(pr.C) + np.tril(pr.C, -1).T, pr.B[N * n:]),
                               rtol=0, atol=1e-12)


def test_arrow_indefinite_tip_reports_the_lapack_column():
    N, n, m = 6, 2, 4
    pr = inputs.arrow(N, n, m, seed=8)
    C = pr.C.copy()
    C[2, 2] = -50.0  # the tip loses definiteness at its third column
    fac = st.arrow_factor(pr.D, pr.E, pr.F, C)
    assert fac["info_psi"] == 0
    S = np.tril(C) + np.tril(C, -1).T - fac["F"].T @ fac["Z"].reshape(N * n, m)
    _, info = sla.lapack.dpotrf(S, lower=1)
    assert fac["info_tip"] == info == 3


def test_triangular_substitution_matches_lapack():
    rng = np.random.default_rng(0)
    L = np.tril(rng.standard_normal((9, 9))) + 5 * np.eye(9)
    B = rng.standard_normal((9, 3))
    np.testing.assert_allclose(st.tri_solve_lower(L, B), sla.solve_triangular(L, B, lower=True), rtol=0,
                               atol=1e-13)
    np.testing.assert_allclose(st.tri_solve_lower(L, B, trans=True),
                               sla.solve_triangular(L, B, lower=True, trans="T"), rtol=0, atol=1e-13)
