"""FP64 CPU oracle for the nested-dissection block-tridiagonal Cholesky.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library path never does.
It shares no code with the GPU library (``paper_2601_03754_amd``) and imports
nothing from it.

The arithmetic lives in ``btc_oracle.c`` (plain C, FP64, plain loops), which
is compiled with gcc into ``liboracle.so`` next to this file and called
through ctypes.  This module only marshals numpy arrays and adds the dense
assembly helpers the brute-force pins need.

Conventions (paper, section "Sequential Cholesky Factorization"): D has
shape (N, n, n) with only the lower triangle of each block read; E has shape
(N-1, n, n) with E[i-1] the block at (i+1, i); right-hand sides are (N, n, m).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "btc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile btc_oracle.c into liboracle.so with gcc (no -march tuning, no
    FMA contraction, so results do not depend on the host CPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.orc_level_of.restype = i64
        lib.orc_level_of.argtypes = [i64]
        lib.orc_num_levels.restype = i64
        lib.orc_num_levels.argtypes = [i64]
        lib.orc_nd_order.restype = None
        lib.orc_nd_order.argtypes = [i64, ip]
        lib.orc_dense_chol.restype = i64
        lib.orc_dense_chol.argtypes = [i64, dp]
        lib.orc_factor_nd.restype = i64
        lib.orc_factor_nd.argtypes = [i64, i64, dp, dp, dp, dp, dp, ip]
        lib.orc_solve_nd.restype = None
        lib.orc_solve_nd.argtypes = [i64, i64, i64, dp, dp, dp, dp, dp]
        lib.orc_factor_seq.restype = i64
        lib.orc_factor_seq.argtypes = [i64, i64, dp, dp, dp, dp, ip]
        lib.orc_solve_seq.restype = None
        lib.orc_solve_seq.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.orc_residual.restype = None
        lib.orc_residual.argtypes = [i64, i64, i64, dp, dp, dp, dp, dp]
        lib.orc_factor_order.restype = i64
        lib.orc_factor_order.argtypes = [i64, i64, ip, dp, dp, dp, dp, dp, ip, ip, ip, ip]
        lib.orc_solve_order.restype = None
        lib.orc_solve_order.argtypes = [i64, i64, i64, ip, dp, dp, dp, ip, ip, dp, dp]
        lib.orc_kstage_order.restype = None
        lib.orc_kstage_order.argtypes = [i64, i64, ip]
        lib.orc_partition_sizes.restype = i64
        lib.orc_partition_sizes.argtypes = [i64, i64, ip]
        lib.orc_partition_order.restype = None
        lib.orc_partition_order.argtypes = [i64, i64, ip, ip, ip]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(D, E):
    D = _f64(D)
    N, n, n2 = D.shape
    assert n == n2 and N >= 1 and n >= 1
    E = _f64(E) if N > 1 else np.zeros((1, n, n))
    if N > 1:
        assert E.shape == (N - 1, n, n)
    return D, E, N, n


def level_of(i: int) -> int:
    return int(_load().orc_level_of(i))


def num_levels(N: int) -> int:
    return int(_load().orc_num_levels(N))


def nd_order(N: int) -> np.ndarray:
    """1-based original block indices in the multi-stage permuted order."""
    out = np.zeros(N, dtype=np.int64)
    _load().orc_nd_order(N, _ip(out))
    return out


def dense_chol(A) -> tuple[np.ndarray, int]:
    """Textbook dense Cholesky (lower), returns (L, info)."""
    L = _f64(A).copy()
    info = int(_load().orc_dense_chol(L.shape[0], _dp(L)))
    return L, info


def factor_nd(D, E, counts: bool = False):
    """Nested-dissection factor (Ld, Rb, Tb) indexed by original block
    (slot i-1 holds block i), plus info (0 or failing 1-based block)."""
    D, E, N, n = _shape(D, E)
    Ld = np.zeros((N, n, n))
    Rb = np.zeros((N, n, n))
    Tb = np.zeros((N, n, n))
    cnt = np.zeros(4, dtype=np.int64)
    info = int(_load().orc_factor_nd(N, n, _dp(D), _dp(E), _dp(Ld), _dp(Rb), _dp(Tb), _ip(cnt)))
    if counts:
        return Ld, Rb, Tb, info, {"potrf": int(cnt[0]), "trsm": int(cnt[1]),
                                  "syrk": int(cnt[2]), "gemm": int(cnt[3])}
    return Ld, Rb, Tb, info


def solve_nd(Ld, Rb, Tb, B) -> np.ndarray:
    Ld = _f64(Ld)
    Rb = _f64(Rb)
    Tb = _f64(Tb)
    N, n, _ = Ld.shape
    B = _f64(B).reshape(N, n, -1)
    m = B.shape[2]
    X = np.empty_like(B)
    _load().orc_solve_nd(N, n, m, _dp(Ld), _dp(Rb), _dp(Tb), _dp(B), _dp(X))
    return X


def factor_seq(D, E, counts: bool = False):
    """Natural-order factor of Algorithm 1: (Dh, Eh, info)."""
    D, E, N, n = _shape(D, E)
    Dh = np.zeros((N, n, n))
    Eh = np.zeros((max(N - 1, 1), n, n))
    cnt = np.zeros(4, dtype=np.int64)
    info = int(_load().orc_factor_seq(N, n, _dp(D), _dp(E), _dp(Dh), _dp(Eh), _ip(cnt)))
    if counts:
        return Dh, Eh, info, {"potrf": int(cnt[0]), "trsm": int(cnt[1]),
                              "syrk": int(cnt[2]), "gemm": int(cnt[3])}
    return Dh, Eh, info


def solve_seq(Dh, Eh, B) -> np.ndarray:
    Dh = _f64(Dh)
    Eh = _f64(Eh)
    N, n, _ = Dh.shape
    B = _f64(B).reshape(N, n, -1)
    m = B.shape[2]
    X = np.empty_like(B)
    _load().orc_solve_seq(N, n, m, _dp(Dh), _dp(Eh), _dp(B), _dp(X))
    return X


def residual(D, E, X, B) -> np.ndarray:
    """B - Psi X in FP64."""
    D, E, N, n = _shape(D, E)
    X = _f64(X).reshape(N, n, -1)
    B = _f64(B).reshape(N, n, -1)
    m = X.shape[2]
    R = np.empty_like(B)
    _load().orc_residual(N, n, m, _dp(D), _dp(E), _dp(X), _dp(B), _dp(R))
    return R


def relres(D, E, X, B) -> float:
    """max over right-hand-side columns of ||b_j - Psi x_j||_2 / ||b_j||_2."""
    R = residual(D, E, X, B)
    N, n, m = R.shape
    r = np.linalg.norm(R.reshape(N * n, m), axis=0)
    b = np.linalg.norm(_f64(B).reshape(N * n, m), axis=0)
    b[b == 0] = 1.0
    return float(np.max(r / b))


def solve(D, E, B) -> np.ndarray:
    """x = Psi^{-1} b via the nested-dissection factor (raises if not SPD)."""
    Ld, Rb, Tb, info = factor_nd(D, E)
    if info != 0:
        raise np.linalg.LinAlgError("block %d is not positive definite" % info)
    return solve_nd(Ld, Rb, Tb, B)


# --------------------------------------------------------------------------
# Other elimination orders (section "Parallel Cholesky Factorization").

def kstage_order(N: int, k: int) -> np.ndarray:
    """First k multi-stage levels, then the remaining blocks in natural order
    (k = 0: Algorithm 1; 1: single-stage; 2: two-stage)."""
    out = np.zeros(N, dtype=np.int64)
    _load().orc_kstage_order(N, k, _ip(out))
    return out


def partition_sizes(N: int, p: int) -> np.ndarray:
    """Chunk sizes N_1..N_p of Proposition 1 (rounded as the paper states)."""
    out = np.zeros(p, dtype=np.int64)
    rc = int(_load().orc_partition_sizes(N, p, _ip(out)))
    if rc != 0:
        raise ValueError("no partition of %d blocks into %d chunks" % (N, p))
    return out


def partition_order(N: int, p: int, sizes=None):
    """(order, phase) of the partition permutation of Algorithm 2."""
    sizes = partition_sizes(N, p) if sizes is None else np.ascontiguousarray(sizes, dtype=np.int64)
    order = np.zeros(N, dtype=np.int64)
    phase = np.zeros(N, dtype=np.int64)
    _load().orc_partition_order(N, p, _ip(sizes), _ip(order), _ip(phase))
    return order, phase


def factor_order(D, E, order, phase=None, counts: bool = False):
    """Block Cholesky of P Psi P^T for the elimination order `order`: (Ld,
    Ro, To, rn, ln, info), indexed by original block; with counts, also the
    potrf/trsm/syrk/gemm counts (per phase when phase is given)."""
    D, E, N, n = _shape(D, E)
    order = np.ascontiguousarray(order, dtype=np.int64)
    Ld, Ro, To = (np.zeros((N, n, n)) for _ in range(3))
    rn = np.zeros(N, dtype=np.int64)
    ln = np.zeros(N, dtype=np.int64)
    nph = 1 if phase is None else int(np.max(phase)) + 1
    cnt = np.zeros(4 * nph, dtype=np.int64)
    ph = None if phase is None else np.ascontiguousarray(phase, dtype=np.int64)
    info = int(_load().orc_factor_order(N, n, _ip(order), _dp(D), _dp(E), _dp(Ld), _dp(Ro), _dp(To),
                                        _ip(rn), _ip(ln), _ip(ph) if ph is not None else None, _ip(cnt)))
    out = (Ld, Ro, To, rn, ln, info)
    if counts:
        return out + (cnt.reshape(nph, 4),)
    return out


def solve_order(order, Ld, Ro, To, rn, ln, B) -> np.ndarray:
    Ld, Ro, To = _f64(Ld), _f64(Ro), _f64(To)
    N, n, _ = Ld.shape
    B = _f64(B).reshape(N, n, -1)
    m = B.shape[2]
    X = np.empty_like(B)
    _load().orc_solve_order(N, n, m, _ip(np.ascontiguousarray(order, dtype=np.int64)), _dp(Ld), _dp(Ro),
                            _dp(To), _ip(np.ascontiguousarray(rn, dtype=np.int64)),
                            _ip(np.ascontiguousarray(ln, dtype=np.int64)), _dp(B), _dp(X))
    return X


# --------------------------------------------------------------------------
# Dense assembly (brute-force pins only).

def assemble_dense(D, E) -> np.ndarray:
    """The full symmetric matrix Psi of order N*n (lower triangles of D)."""
    D, E, N, n = _shape(D, E)
    A = np.zeros((N * n, N * n))
    for i in range(N):
        Di = np.tril(D[i]) + np.tril(D[i], -1).T
        A[i * n:(i + 1) * n, i * n:(i + 1) * n] = Di
        if i + 1 < N:
            A[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = E[i]
            A[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = E[i].T
    return A


def perm_indices(N: int, n: int) -> np.ndarray:
    """Scalar row permutation of P_inf: row p of P Psi P^T is row perm[p]."""
    order = nd_order(N) - 1
    return (order[:, None] * n + np.arange(n)[None, :]).reshape(-1)


def dense_factor_blocks(Ldense: np.ndarray, N: int, n: int):
    """Extract (Ld, Rb, Tb) in the oracle's convention from a dense lower
    factor of P Psi P^T."""
    order = nd_order(N)
    pos = {int(b): p for p, b in enumerate(order)}
    Ld = np.zeros((N, n, n))
    Rb = np.zeros((N, n, n))
    Tb = np.zeros((N, n, n))

    def blk(bi, bj):
        pi, pj = pos[bi], pos[bj]
        return Ldense[pi * n:(pi + 1) * n, pj * n:(pj + 1) * n]

    for i in range(1, N + 1):
        s = 1 << level_of(i)
        Ld[i - 1] = blk(i, i)
        if i + s <= N:
            Rb[i - 1] = blk(i + s, i)
        if i > s:
            Tb[i - 1] = blk(i - s, i).T
    return Ld, Rb, Tb
