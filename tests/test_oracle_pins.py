"""Pins of the FP64 CPU oracle against things other than itself: LAPACK's dense
Cholesky of the explicitly permuted matrix, a textbook dense Cholesky, closed
forms, special cases that reduce to library routines, the natural-order
Algorithm 1, the paper's printed N = 20 example, and the paper's sequential
cost formula.  None of these needs a GPU."""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2601_03754_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [(N, n) for N in (1, 2, 3, 4, 5, 7, 8, 16, 20, 31, 33) for n in (1, 3, 5)]


def permuted_dense(D, E):
    A = oracle.assemble_dense(D, E)
    N, n, _ = D.shape
    p = oracle.perm_indices(N, n)
    return A[np.ix_(p, p)]


@pytest.mark.parametrize("N,n", SHAPES)
def test_factor_matches_lapack_dense_cholesky(N, n):
    """Pin P1: the nested-dissection factor is the (unique) Cholesky factor of
    P Psi P^T, blockwise equal to LAPACK dpotrf of the dense permuted matrix."""
    pr = inputs.block_tridiag(N, n, seed=N * 100 + n)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    assert info == 0
    Ldense = np.linalg.cholesky(permuted_dense(pr.D, pr.E))
    L2, R2, T2 = oracle.dense_factor_blocks(Ldense, N, n)
    scale = np.abs(Ldense).max()
    assert np.abs(Ld - L2).max() <= 1e-13 * scale
    assert np.abs(Rb - R2).max() <= 1e-13 * scale
    assert np.abs(Tb - T2).max() <= 1e-13 * scale


@pytest.mark.parametrize("N,n", [(7, 3), (20, 2), (33, 4)])
def test_textbook_dense_cholesky_matches_lapack(N, n):
    """The oracle's own dense Cholesky (used as the brute-force definition)
    agrees with LAPACK on the permuted matrix, and reports failure on an
    indefinite one."""
    pr = inputs.block_tridiag(N, n, seed=5)
    A = permuted_dense(pr.D, pr.E)
    L, info = oracle.dense_chol(A)
    assert info == 0
    assert np.abs(L - np.linalg.cholesky(A)).max() <= 1e-13 * np.abs(L).max()
    A2 = A.copy()
    A2[3, 3] = -1.0
    _, info2 = oracle.dense_chol(A2)
    assert info2 == 4


@pytest.mark.parametrize("N,n", [(5, 3), (16, 4), (20, 3), (33, 2)])
def test_reconstruction(N, n):
    """Pin P2: L L^T reproduces P Psi P^T."""
    pr = inputs.block_tridiag(N, n, seed=11)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    assert info == 0
    # assemble the dense factor from the blocks
    order = oracle.nd_order(N)
    pos = {int(b): p for p, b in enumerate(order)}
    L = np.zeros((N * n, N * n))
    for i in range(1, N + 1):
        s = 1 << oracle.level_of(i)
        pi = pos[i]
        L[pi * n:(pi + 1) * n, pi * n:(pi + 1) * n] = Ld[i - 1]
        if i + s <= N:
            pr_ = pos[i + s]
            L[pr_ * n:(pr_ + 1) * n, pi * n:(pi + 1) * n] = Rb[i - 1]
        if i > s:
            pl = pos[i - s]
            L[pl * n:(pl + 1) * n, pi * n:(pi + 1) * n] = Tb[i - 1].T
    A = permuted_dense(pr.D, pr.E)
    assert np.linalg.norm(L @ L.T - A) <= 1e-14 * np.linalg.norm(A)
    assert np.allclose(np.triu(L, 1), 0.0)


@pytest.mark.parametrize("N", [7, 16, 20, 33])
def test_structural_zeros(N):
    """Pin P3: wherever nested dissection predicts no factor block, LAPACK's
    dense factor of P Psi P^T is exactly zero; the predicted blocks are the
    diagonal and, for node i at stride s, rows i+s and i-s."""
    n = 3
    pr = inputs.block_tridiag(N, n, seed=3)
    Ldense = np.linalg.cholesky(permuted_dense(pr.D, pr.E))
    order = oracle.nd_order(N)
    pos = {int(b): p for p, b in enumerate(order)}
    allowed = np.zeros((N, N), dtype=bool)
    for i in range(1, N + 1):
        s = 1 << oracle.level_of(i)
        allowed[pos[i], pos[i]] = True
        if i + s <= N:
            allowed[pos[i + s], pos[i]] = True
        if i > s:
            allowed[pos[i - s], pos[i]] = True
    for a in range(N):
        for b in range(a + 1):
            blk = Ldense[a * n:(a + 1) * n, b * n:(b + 1) * n]
            if not allowed[a, b]:
                assert np.all(blk == 0.0), (a, b)
    # number of off-diagonal factor blocks and of fill-in gemms
    n_off = int(allowed.sum()) - N
    _, _, _, info, cnt = oracle.factor_nd(pr.D, pr.E, counts=True)
    assert info == 0
    assert cnt["trsm"] == n_off and cnt["syrk"] == n_off
    assert cnt["potrf"] == N


def test_paper_n20_display():
    """The N = 20 example the paper prints: level groups of Phi_inf start with
    the blocks its display shows, and L_inf has nonzero blocks where its
    display shows Ehat entries."""
    groups, nz = {}, []
    with open(os.path.join(GOLDEN, "nd_n20_display.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line.startswith("group"):
                k, v = line[len("group"):].split(":")
                groups[int(k)] = [int(x) for x in v.split()]
            elif line.startswith("nz:"):
                a, b = line[3:].split()
                nz.append((int(a), int(b)))
    N, n = 20, 2
    order = list(oracle.nd_order(N))
    lvl = [oracle.level_of(i) for i in order]
    for g, shown in groups.items():
        members = [b for b, l in zip(order, lvl) if l == g]
        assert members[:len(shown)] == shown
    # groups are contiguous and in increasing level order
    assert lvl == sorted(lvl)
    pr = inputs.block_tridiag(N, n, seed=1)
    Ldense = np.linalg.cholesky(permuted_dense(pr.D, pr.E))
    pos = {int(b): p for p, b in enumerate(order)}
    for a, b in nz:
        blk = Ldense[pos[a] * n:(pos[a] + 1) * n, pos[b] * n:(pos[b] + 1) * n]
        assert np.abs(blk).max() > 0.0
    assert oracle.num_levels(N) == 5


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_closed_form_laplacian_factor(k):
    """Pin P4: for D_i = 2I, E_i = -I and N = 2^k - 1 every separator keeps two
    neighbours at every level, so by induction S = 2^{1-l} I at level l:
    L_ii = 2^{(1-l)/2} I and R_i = T_i = -2^{-(l+1)/2} I."""
    N, n = 2 ** k - 1, 3
    pr = inputs.laplacian(N, n)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    assert info == 0
    eye = np.eye(n)
    for i in range(1, N + 1):
        lv = oracle.level_of(i)
        s = 1 << lv
        assert np.allclose(Ld[i - 1], 2.0 ** ((1 - lv) / 2) * eye, rtol=0, atol=2e-15)
        if i + s <= N:
            assert np.allclose(Rb[i - 1], -(2.0 ** (-(lv + 1) / 2)) * eye, rtol=0, atol=2e-15)
        if i > s:
            assert np.allclose(Tb[i - 1], -(2.0 ** (-(lv + 1) / 2)) * eye, rtol=0, atol=2e-15)


@pytest.mark.parametrize("N", [1, 2, 5, 7, 16, 31])
def test_closed_form_laplacian_solve(N):
    """Pin P5: (T_N^{-1})_{ij} = min(i,j) (N+1-max(i,j)) / (N+1) for
    T_N = tridiag(-1, 2, -1), so x = (T_N^{-1} (x) I_n) b."""
    n, m = 2, 3
    pr = inputs.laplacian(N, n, nrhs=m, seed=N)
    X = oracle.solve(pr.D, pr.E, pr.B)
    i = np.arange(1, N + 1)
    Tinv = np.minimum.outer(i, i) * (N + 1 - np.maximum.outer(i, i)) / (N + 1)
    Xref = np.einsum("ij,jrq->irq", Tinv, pr.B)
    assert np.abs(X - Xref).max() <= 1e-13 * max(1.0, np.abs(Xref).max()) * N


@pytest.mark.parametrize("N,n", [(1, 4), (6, 3), (17, 5)])
def test_decoupled_blocks_reduce_to_potrf(N, n):
    """Pin P6: with E = 0 the factor is chol(D_i) per block (LAPACK) and the
    couplings vanish; N = 1 is a single potrf/potrs."""
    pr = inputs.block_tridiag(N, n, seed=9)
    E = np.zeros_like(pr.E)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, E)
    assert info == 0
    for i in range(N):
        assert np.allclose(Ld[i], np.linalg.cholesky(pr.D[i]), rtol=0, atol=1e-14 * np.abs(pr.D[i]).max())
    assert np.all(Rb == 0) and np.all(Tb == 0)
    X = oracle.solve_nd(Ld, Rb, Tb, pr.B)
    for i in range(N):
        ref = scipy.linalg.cho_solve((np.linalg.cholesky(pr.D[i]), True), pr.B[i])
        assert np.allclose(X[i], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("N", [2, 3, 9, 64, 100])
def test_scalar_case_matches_banded_solver(N):
    """Pin P7: n = 1 is a scalar SPD tridiagonal system (LAPACK pbsv via
    scipy.linalg.solveh_banded)."""
    pr = inputs.block_tridiag(N, 1, seed=N, nrhs=2)
    X = oracle.solve(pr.D, pr.E, pr.B)
    ab = np.zeros((2, N))
    ab[0] = pr.D[:, 0, 0]
    if N > 1:
        ab[1, :-1] = pr.E[:, 0, 0]
    ref = scipy.linalg.solveh_banded(ab, pr.B.reshape(N, 2), lower=True)
    assert np.allclose(X.reshape(N, 2), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("N,n,m", [(1, 3, 1), (2, 4, 2), (13, 5, 3), (64, 6, 1), (100, 3, 4)])
def test_nd_solve_matches_natural_order(N, n, m):
    """Pin P8: Algorithm 1 (natural order, bidiagonal factor, a different
    factor) gives the same solution; both match a dense LAPACK solve."""
    pr = inputs.block_tridiag(N, n, seed=7, nrhs=m)
    Xnd = oracle.solve(pr.D, pr.E, pr.B)
    Dh, Eh, info = oracle.factor_seq(pr.D, pr.E)
    assert info == 0
    Xseq = oracle.solve_seq(Dh, Eh, pr.B)
    A = oracle.assemble_dense(pr.D, pr.E)
    Xd = np.linalg.solve(A, pr.B.reshape(N * n, m)).reshape(N, n, m)
    tol = 1e-12 * np.abs(Xd).max()
    assert np.abs(Xnd - Xd).max() <= tol
    assert np.abs(Xseq - Xd).max() <= tol
    # the natural-order factor is LAPACK's Cholesky of the unpermuted matrix
    Ldense = np.linalg.cholesky(A)
    for i in range(N):
        assert np.allclose(Dh[i], Ldense[i * n:(i + 1) * n, i * n:(i + 1) * n], rtol=0, atol=1e-13)


@pytest.mark.parametrize("N,n,m", [(1, 2, 1), (5, 3, 2), (12, 4, 3)])
def test_residual_matches_dense_product(N, n, m):
    """The FP64 residual b - Psi x against a dense product; the lower triangle
    of D alone defines the matrix."""
    pr = inputs.block_tridiag(N, n, seed=2, nrhs=m)
    X = np.random.default_rng(0).standard_normal((N, n, m))
    D = pr.D.copy()
    D += np.triu(np.ones((n, n)), 1)[None] * 123.0  # garbage in the upper triangle
    R = oracle.residual(D, pr.E, X, pr.B)
    A = oracle.assemble_dense(pr.D, pr.E)
    ref = pr.B.reshape(N * n, m) - A @ X.reshape(N * n, m)
    assert np.allclose(R.reshape(N * n, m), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N,n,k", [(9, 3, 13), (16, 2, 9), (31, 1, 15)])
def test_relres_closed_form(N, n, k):
    """The relative residual is the maximum over right-hand-side columns of
    ||b_j - Psi x_j||_2 / ||b_j||_2.  Closed form: for the block Laplacian
    tridiag(-I, 2I, -I) and an iterate that is a multiple d_j of the unit
    vector e_k (k an interior scalar row, 0-based), column k of Psi holds
    2, -1, -1 at rows k, k-n, k+n, so Psi x_j = d_j (2 e_k - e_{k-n} -
    e_{k+n}).  With b_j supported on rows far from k, ||b_j - Psi x_j||^2 =
    ||b_j||^2 + 6 d_j^2.  Three columns with different ratios pin the
    reduction: a norm over rows, a Frobenius norm over all columns, a mean
    or a minimum over columns would each give another number."""
    D = np.tile(2.0 * np.eye(n), (N, 1, 1))
    E = np.tile(-np.eye(n), (N - 1, 1, 1))
    dim = N * n
    d = np.array([0.5, 3.0, 1e-3])
    bnorm = np.array([2.0, 1.5, 4.0])
    B = np.zeros((dim, 3))
    X = np.zeros((dim, 3))
    far = [r for r in range(dim) if abs(r - k) > n]
    for j in range(3):
        B[far[j], j] = bnorm[j]          # one entry, so ||b_j|| = bnorm[j]
        X[k, j] = d[j]
    expect = np.sqrt(1.0 + 6.0 * d ** 2 / bnorm ** 2)
    got = oracle.relres(D, E, X.reshape(N, n, 3), B.reshape(N, n, 3))
    assert got == pytest.approx(expect.max(), rel=1e-15)
    assert np.argmax(expect) == 1                      # the largest ratio is not the first column
    assert abs(got - expect.min()) > 0.1 and abs(got - expect.mean()) > 0.1
    fro = np.sqrt((bnorm ** 2 + 6 * d ** 2).sum() / (bnorm ** 2).sum())
    assert abs(got - fro) > 0.1
    # an exact solution has zero residual; x = 0 has relative residual 1
    assert oracle.relres(D, E, np.zeros((N, n, 3)), B.reshape(N, n, 3)) == pytest.approx(1.0, rel=1e-15)


@pytest.mark.parametrize("N", [1, 2, 7, 16, 33, 100])
def test_sequential_cost_formula(N):
    """Section "Computational Complexity": Algorithm 1 costs
    (7N/3 - 2) n^3 flops with potrf n^3/3, trsm n^3, syrk n^3."""
    n = 2
    pr = inputs.block_tridiag(N, n, seed=1)
    *_, info, cnt = oracle.factor_seq(pr.D, pr.E, counts=True)
    assert info == 0
    flops = cnt["potrf"] / 3 + cnt["trsm"] + cnt["syrk"] + 2 * cnt["gemm"]
    assert abs(flops - (7 * N / 3 - 2)) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 15, 16, 20, 1000, 4096, 16384])
def test_levels_and_order(N):
    """Section "Multi-Stage Permutation": floor(log2 N)+1 levels; level l holds
    the odd multiples of 2^l; the order is a permutation."""
    order = oracle.nd_order(N)
    assert sorted(order.tolist()) == list(range(1, N + 1))
    L = oracle.num_levels(N)
    assert L == int(np.floor(np.log2(N))) + 1
    lv = np.array([oracle.level_of(int(i)) for i in order]) if N <= 1000 else None
    if lv is not None:
        assert lv.max() == L - 1
        for l in range(L):
            s = 1 << l
            assert int((lv == l).sum()) == (N + s) // (2 * s)


def test_breakdown_reports_first_failing_block():
    """Indefinite input: a negative leaf block fails at level 0; a separator
    that becomes indefinite after the Schur updates fails at its level."""
    N, n = 8, 3
    pr = inputs.block_tridiag(N, n, seed=4)
    D = pr.D.copy()
    D[4] = -np.eye(n)  # block 5 (odd, level 0)
    *_, info = oracle.factor_nd(D, pr.E)
    assert info == 5
    D = pr.D.copy()
    D[3] = 1e-3 * np.eye(n)  # block 4 (level 2): positive, but not after updates
    *_, info = oracle.factor_nd(D, pr.E)
    assert info == 4
    # the literal generator at c = 0.1 is indefinite
    pr2 = inputs.block_tridiag(64, 8, c=0.1, seed=0)
    *_, info = oracle.factor_nd(pr2.D, pr2.E)
    assert info > 0


def test_margin_generator_sets_smallest_eigenvalue():
    """The spectral-margin reading of the diagonal shift: lambda_min == c."""
    for c in (4.0, 0.1, 0.001):
        pr = inputs.block_tridiag(12, 4, c=c, seed=3, margin=True)
        w = np.linalg.eigvalsh(oracle.assemble_dense(pr.D, pr.E))
        assert abs(w[0] - c) <= 1e-10 * max(1.0, abs(w[-1]))


def test_generator_is_reproducible():
    a = inputs.block_tridiag(9, 5, seed=42, nrhs=2)
    b = inputs.block_tridiag(9, 5, seed=42, nrhs=2)
    assert a.D.tobytes() == b.D.tobytes() and a.E.tobytes() == b.E.tobytes()
    assert a.B.tobytes() == b.B.tobytes()
    assert np.allclose(a.D, a.D.transpose(0, 2, 1))
