"""FP64 CPU oracle for the block-banded and arrow extensions.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the library path never does.
It shares no code with the GPU library and imports nothing from it.

The paper names both structures as extensions of the method without giving
an algorithm for either (section "Multi-Stage Permutation", remark after the
cyclic-reduction equivalence: arrow structures; section "Conclusion": block
banded matrices with a larger bandwidth).  The readings implemented here:

Block-banded, block bandwidth b (block (i, j) is zero for |i - j| > b):
    grouping b consecutive block rows and columns into one super-block of
    order b*n makes the matrix block tridiagonal with ceil(N/b) super-blocks
    (the block (i, j) with |i - j| <= b lands in the same or a neighbouring
    super-block).  The multi-stage method then applies unchanged.  When b
    does not divide N the last super-block is completed with identity rows
    and columns, decoupled from the rest (zero right-hand side, zero
    solution).

Arrow (a block-tridiagonal Psi bordered by m dense rows and columns):
        A = [[Psi, F], [F^T, C]],  F of size (N*n) x m,  C of size m x m.
    Psi is eliminated first, in the multi-stage order, then the tip:
        Z = Psi^{-1} F,    S = C - F^T Z    (Schur complement),    L_S = chol(S)
    and a solve of A [x1; x2] = [b1; b2] is
        y = Psi^{-1} b1,   x2 = S^{-1} (b2 - F^T y),   x1 = y - Z x2.
    The block Cholesky factor of A in that order is [[L, 0], [F^T L^{-T}, L_S]]
    with L the multi-stage factor of Psi, so L_S is the trailing block of the
    Cholesky factor of the permuted A.

Storage: a block-banded matrix is A_band of shape (N, b+1, n, n) with
A_band[i, k] the block at (i, i-k) (0-based block rows; k = 0 the diagonal
block, only its lower triangle read; entries with i - k < 0 unused).
"""
from __future__ import annotations

import numpy as np

from . import dense_chol, factor_nd, solve_nd


def band_to_tridiag(A_band, b: int):
    """Super-blocks of b block rows: (D2, E2) of the block-tridiagonal
    matrix of order ceil(N/b) * b*n (identity completion)."""
    A_band = np.asarray(A_band, dtype=np.float64)
    N, bb, n, _ = A_band.shape
    assert bb == b + 1 and b >= 1
    N2 = -(-N // b)
    n2 = b * n
    D2 = np.zeros((N2, n2, n2))
    E2 = np.zeros((max(N2 - 1, 0), n2, n2))
    for I in range(N2):
        for r in range(b):
            i = b * I + r
            if i >= N:
                # completion: identity on the missing block rows
                D2[I, r * n:(r + 1) * n, r * n:(r + 1) * n] = np.eye(n)
                continue
            for c in range(r + 1):
                blk = A_band[i, r - c]
                if c == r:
                    blk = np.tril(blk) + np.tril(blk, -1).T
                D2[I, r * n:(r + 1) * n, c * n:(c + 1) * n] = blk
                if c < r:
                    D2[I, c * n:(c + 1) * n, r * n:(r + 1) * n] = blk.T
            if I >= 1:
                # block (i, j) of the previous super-block: j = b(I-1) + c,
                # distance i - j = b + r - c <= b exactly when c >= r
                for c in range(r, b):
                    E2[I - 1, r * n:(r + 1) * n, c * n:(c + 1) * n] = A_band[i, b + r - c]
    return D2, E2


def _pad_rhs(B, N: int, n: int, b: int):
    B = np.asarray(B, dtype=np.float64).reshape(N * n, -1)
    N2 = -(-N // b)
    P = np.zeros((N2 * b * n, B.shape[1]))
    P[:N * n] = B
    return P.reshape(N2, b * n, -1)


def banded_factor(A_band, b: int):
    """Multi-stage factor (Ld, Rb, Tb, info) of the super-block matrix."""
    D2, E2 = band_to_tridiag(A_band, b)
    return factor_nd(D2, E2)


def banded_solve(A_band, b: int, B) -> np.ndarray:
    """x = A^{-1} B for the block-banded A; B and x of shape (N, n, m)."""
    A_band = np.asarray(A_band, dtype=np.float64)
    N, _, n, _ = A_band.shape
    Ld, Rb, Tb, info = banded_factor(A_band, b)
    if info != 0:
        raise np.linalg.LinAlgError("super-block %d is not positive definite" % info)
    X2 = solve_nd(Ld, Rb, Tb, _pad_rhs(B, N, n, b))
    return X2.reshape(-1, X2.shape[2])[:N * n].reshape(N, n, -1)


def tri_solve_lower(L, B, trans: bool = False) -> np.ndarray:
    """L^{-1} B (or L^{-T} B) for a lower-triangular L by substitution."""
    L = np.asarray(L, dtype=np.float64)
    X = np.array(B, dtype=np.float64, copy=True).reshape(L.shape[0], -1)
    m = L.shape[0]
    if not trans:
        for j in range(m):
            X[j] /= L[j, j]
            X[j + 1:] -= np.outer(L[j + 1:, j], X[j])
    else:
        for j in range(m - 1, -1, -1):
            X[j] /= L[j, j]
            X[:j] -= np.outer(L[j, :j], X[j])
    return X


def arrow_factor(D, E, F, C):
    """Factor of the arrow [[Psi, F], [F^T, C]]: a dict with the multi-stage
    factor of Psi (Ld, Rb, Tb), Z = Psi^{-1} F (shape (N, n, m)), the Schur
    complement S, its Cholesky factor Ls, and info_psi / info_tip (0, or the
    1-based failing block of Psi / column of S)."""
    D = np.asarray(D, dtype=np.float64)
    N, n, _ = D.shape
    F = np.asarray(F, dtype=np.float64).reshape(N * n, -1)
    m = F.shape[1]
    C = np.asarray(C, dtype=np.float64).reshape(m, m)
    Ld, Rb, Tb, info = factor_nd(D, E)
    out = {"Ld": Ld, "Rb": Rb, "Tb": Tb, "F": F, "info_psi": info, "info_tip": 0, "m": m}
    if info != 0:
        return out
    Z = solve_nd(Ld, Rb, Tb, F.reshape(N, n, m))
    Cl = np.tril(C) + np.tril(C, -1).T
    S = Cl - F.T @ Z.reshape(N * n, m)
    Ls, info_tip = dense_chol(S)
    out.update(Z=Z, S=S, Ls=np.tril(Ls), info_tip=info_tip)
    return out


def arrow_solve(fac, B) -> np.ndarray:
    """Solve with an arrow factor; B of shape (N*n + m, nrhs) (the rows of
    Psi first, then the m rows of the tip); returns x of the same shape."""
    Ld = fac["Ld"]
    N, n, _ = Ld.shape
    m = fac["m"]
    B = np.asarray(B, dtype=np.float64).reshape(N * n + m, -1)
    q = B.shape[1]
    y = solve_nd(Ld, fac["Rb"], fac["Tb"], B[:N * n].reshape(N, n, q)).reshape(N * n, q)
    if m == 0:
        return y
    Z = fac["Z"].reshape(N * n, m)
    F = fac["F"]
    r2 = B[N * n:] - F.T @ y
    x2 = tri_solve_lower(fac["Ls"], tri_solve_lower(fac["Ls"], r2), trans=True)
    x1 = y - Z @ x2
    return np.vstack([x1, x2])


def assemble_arrow_dense(D, E, F, C) -> np.ndarray:
    """The full symmetric arrow matrix of order N*n + m."""
    from . import assemble_dense
    P = assemble_dense(D, E)
    K = P.shape[0]
    F = np.asarray(F, dtype=np.float64).reshape(K, -1)
    m = F.shape[1]
    C = np.asarray(C, dtype=np.float64).reshape(m, m)
    A = np.zeros((K + m, K + m))
    A[:K, :K] = P
    A[:K, K:] = F
    A[K:, :K] = F.T
    A[K:, K:] = np.tril(C) + np.tril(C, -1).T
    return A
