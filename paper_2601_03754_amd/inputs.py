"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input recipes only: it draws random blocks and assembles
no part of the factorization or solve.  Both the GPU library's tests and
benchmark and the CPU oracle's tests draw their inputs from here, so the two
sides see identical bytes for a given seed.

Recipe (the block-tridiagonal matrix of the section "Sequential Cholesky
Factorization"; the paper never states how its own test matrices were drawn):
    rng = numpy.random.default_rng(seed)          # PCG64
    G   = rng.standard_normal((N, n, n))
    D_i = G_i G_i^T / n + c I                      # symmetric positive definite
    E   = rng.standard_normal((N-1, n, n)) / sqrt(n)
    B   = rng.standard_normal((N, n, nrhs))
With c = 4 the whole matrix is positive definite with a margin of about 1.3-1.7
(smallest eigenvalue) for every shape used here.  For the conditioning sweep
the shift is read as a spectral margin (``margin=True``): the identity shift is
chosen so that the smallest eigenvalue of the assembled matrix equals c
exactly, found with LAPACK's banded symmetric eigensolver.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Problem:
    D: np.ndarray  # (N, n, n) float64, symmetric blocks
    E: np.ndarray  # (N-1, n, n) float64, E[i-1] = block (i+1, i)
    B: np.ndarray  # (N, n, nrhs) float64
    c: float       # identity shift actually applied to the diagonal blocks

    @property
    def N(self) -> int:
        return self.D.shape[0]

    @property
    def n(self) -> int:
        return self.D.shape[1]

    @property
    def nrhs(self) -> int:
        return self.B.shape[2]


def sweep_seed(N: int, n: int) -> int:
    """Seed used for the (N, n) sweep: 1000*log2(N) + n."""
    return int(1000 * round(math.log2(N)) + n)


def _draw(N: int, n: int, nrhs: int, seed: int):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, n, n))
    GG = np.matmul(G, G.transpose(0, 2, 1)) / n
    del G
    E = rng.standard_normal((max(N - 1, 0), n, n)) / math.sqrt(n)
    B = rng.standard_normal((N, n, nrhs))
    return GG, E, B


def band_lower(D: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Lower banded storage (LAPACK 'L', bandwidth 2n-1) of the assembled
    block-tridiagonal matrix: band[d, j] = A[j+d, j]."""
    N, n, _ = D.shape
    dim = N * n
    band = np.zeros((2 * n, dim))
    j = np.arange(dim)
    bj, cj = j // n, j % n
    for d in range(2 * n):
        i = j + d
        ok = i < dim
        bi, ri = i[ok] // n, i[ok] % n
        same = bi == bj[ok]
        vals = np.zeros(ok.sum())
        vals[same] = D[bj[ok][same], ri[same], cj[ok][same]]
        nxt = bi == bj[ok] + 1
        vals[nxt] = E[bj[ok][nxt], ri[nxt], cj[ok][nxt]]
        band[d, ok] = vals
    return band


def lambda_min(D: np.ndarray, E: np.ndarray) -> float:
    """Smallest eigenvalue of the assembled matrix (LAPACK dsbevx)."""
    from scipy.linalg import eigvals_banded
    w = eigvals_banded(band_lower(D, E), lower=True, select="i", select_range=(0, 0))
    return float(w[0])


def block_tridiag(N: int, n: int, c: float = 4.0, seed: int = 0, nrhs: int = 1,
                  margin: bool = False, lam0: float | None = None) -> Problem:
    """One instance.  ``margin=False``: D_i = G G^T/n + c I (literal shift).
    ``margin=True``: the shift is chosen so that lambda_min(Psi) == c, with
    lambda_min of the unshifted matrix from LAPACK's banded eigensolver, or
    ``lam0`` when the caller has it (large instances: the banded eigensolver
    is too slow there)."""
    if N < 1 or n < 1:
        raise ValueError("N and n must be positive")
    GG, E, B = _draw(N, n, nrhs, seed)
    eye = np.eye(n)
    if margin:
        if lam0 is None:
            lam0 = lambda_min(GG, E)
        shift = c - lam0
    else:
        shift = c
    D = GG + shift * eye[None, :, :]
    return Problem(D=D, E=E, B=B, c=float(shift))


def unshifted(N: int, n: int, seed: int = 0, nrhs: int = 1):
    """(G G^T / n, E, B) of the recipe before any identity shift."""
    return _draw(N, n, nrhs, seed)


def laplacian(N: int, n: int, nrhs: int = 1, seed: int = 0) -> Problem:
    """Block Laplacian D_i = 2I, E_i = -I: Psi = T_N (x) I_n with
    T_N = tridiag(-1, 2, -1), whose inverse and factors have closed forms."""
    rng = np.random.default_rng(seed)
    D = np.broadcast_to(2.0 * np.eye(n), (N, n, n)).copy()
    E = np.broadcast_to(-np.eye(n), (max(N - 1, 0), n, n)).copy()
    B = rng.standard_normal((N, n, nrhs))
    return Problem(D=D, E=E, B=B, c=0.0)


def batch_shapes(count: int = 512, seed: int = 0, N_range=(32, 2048),
                 n_choices=(8, 16, 24, 32, 48)):
    """(N, n) of the many-instance batch: N ~ U{N_lo..N_hi}, n ~ U(choices)."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b)) for a, b in zip(Ns, ns)]


def served_clients(count: int = 256, seed: int = 0, N_range=(64, 4096), n_range=(12, 96)):
    """(N, n) of the clients of the served workload: N = round(exp(U[ln N_lo,
    ln N_hi])) (log-uniform), n ~ U{n_lo..n_hi}."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(N_range[0]), math.log(N_range[1])
    Ns = np.rint(np.exp(rng.uniform(lo, hi, size=count))).astype(np.int64)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(Ns, ns)]


def block_tridiag_device(N: int, n: int, c: float = 4.0, seed: int = 0, nrhs: int = 1, device="cuda:0"):
    """The same recipe drawn with torch's device generator (seeded; for
    benchmark inputs too large to draw on the host): returns (D, E, B) FP64
    tensors on `device`, D exactly symmetric (its lower triangle mirrored)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    G = torch.randn((N, n, n), generator=g, device=device, dtype=torch.float64)
    D = torch.bmm(G, G.transpose(1, 2).contiguous()) / n
    del G
    low = torch.tril(D)
    D = low + torch.tril(D, -1).transpose(1, 2) + c * torch.eye(n, device=device, dtype=torch.float64)
    D = D.contiguous()
    E = torch.randn((max(N - 1, 0), n, n), generator=g, device=device, dtype=torch.float64) / math.sqrt(n)
    B = torch.randn((N, n, max(nrhs, 1)), generator=g, device=device, dtype=torch.float64)
    return D, E, B


# ---------------------------------------------------------------------------
# Block-banded and arrow structures (the method's extensions).

@dataclass
class BandedProblem:
    A_band: np.ndarray  # (N, b+1, n, n): A_band[i, k] = block (i, i-k), k = 0 symmetric
    B: np.ndarray       # (N, n, nrhs)
    c: float            # lower bound of the smallest eigenvalue

    @property
    def b(self) -> int:
        return self.A_band.shape[1] - 1


def block_banded(N: int, n: int, b: int, c: float = 1.0, seed: int = 0, nrhs: int = 1) -> BandedProblem:
    """Block-banded SPD matrix of block bandwidth b.  Recipe:
        rng = default_rng(seed); G = rng.standard_normal((N, n, n))
        O = rng.standard_normal((N, b, n, n)) / sqrt(n)   # A_band[i, k] = O[i, k-1], k >= 1
        (blocks with i - k < 0 set to zero)
        D_i = G_i G_i^T / n + (c + rho_i) I,  rho_i = sum of the spectral norms
              of the off-diagonal blocks of block row i (both sides)
        B = rng.standard_normal((N, n, nrhs))
    By the block Gershgorin theorem every eigenvalue is at least c."""
    if N < 1 or n < 1 or b < 1:
        raise ValueError("N, n and b must be positive")
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, n, n))
    O = rng.standard_normal((N, b, n, n)) / math.sqrt(n)
    B = rng.standard_normal((N, n, nrhs))
    for k in range(1, b + 1):
        O[:min(k, N), k - 1] = 0.0
    norms = np.linalg.norm(O, ord=2, axis=(2, 3))  # (N, b): ||block (i, i-k)||
    rho = norms.sum(axis=1)
    for k in range(1, min(b, N - 1) + 1):
        # block (i, i-k) also sits in block row i-k (transposed)
        rho[:N - k] += norms[k:, k - 1]
    A = np.empty((N, b + 1, n, n))
    A[:, 0] = np.matmul(G, G.transpose(0, 2, 1)) / n + (c + rho)[:, None, None] * np.eye(n)[None]
    A[:, 1:] = O
    return BandedProblem(A_band=A, B=B, c=float(c))


@dataclass
class ArrowProblem:
    D: np.ndarray  # (N, n, n) diagonal blocks of Psi
    E: np.ndarray  # (N-1, n, n) sub-diagonal blocks of Psi
    F: np.ndarray  # (N*n, m) border: the rows of Psi, the columns of the tip
    C: np.ndarray  # (m, m) tip, symmetric
    B: np.ndarray  # (N*n + m, nrhs)
    c: float       # lower bound of the smallest eigenvalue of the tip's Schur complement


def arrow(N: int, n: int, m: int, c: float = 1.0, seed: int = 0, nrhs: int = 1) -> ArrowProblem:
    """Arrow matrix [[Psi, F], [F^T, C]].  Recipe: Psi is block_banded(N, n,
    1, c, seed) (smallest eigenvalue >= c); then with
    rng = default_rng(seed + 1):
        F = rng.standard_normal((N*n, m)) / sqrt(N*n)
        H = rng.standard_normal((m, m));  C = H H^T / m + (c + ||F||_2^2 / c) I
        B = rng.standard_normal((N*n + m, nrhs))
    so that C - F^T Psi^{-1} F >= c I."""
    t = block_banded(N, n, 1, c=c, seed=seed)
    rng = np.random.default_rng(seed + 1)
    K = N * n
    F = rng.standard_normal((K, m)) / math.sqrt(K)
    H = rng.standard_normal((m, m))
    fn = float(np.linalg.norm(F, 2)) if m else 0.0
    C = H @ H.T / max(m, 1) + (c + fn * fn / c) * np.eye(m)
    B = rng.standard_normal((K + m, nrhs))
    return ArrowProblem(D=t.A_band[:, 0].copy(), E=t.A_band[1:, 1].copy(), F=F, C=C, B=B, c=float(c))
