"""Spectral margin of the conditioning sweep: the smallest eigenvalue of the
unshifted block-tridiagonal matrix, by bisection on whether the oracle's
block Cholesky of the shifted matrix succeeds.  Test infrastructure (calls
the oracle only)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


# Smallest eigenvalue of the unshifted matrix, by bisection on the success of
# the oracle's natural-order block Cholesky (section "Sequential Cholesky
# Factorization") of Psi_0 - sigma I: it succeeds exactly when sigma is below
# lambda_min.  Each round factors at several shifts at once (the oracle
# releases the interpreter lock, so threads run in parallel).

def _spd_at(GG, E, sigma):
    D = GG - sigma * np.eye(GG.shape[1])[None]
    *_, info = oracle.factor_seq(D, E)
    return info == 0


def lambda0_bisect(GG, E, tol=1e-7):
    n = GG.shape[1]
    lam_d = np.linalg.eigvalsh(GG).min(axis=1)                  # lambda_min(D_i)
    enorm = np.linalg.norm(E, ord=2, axis=(1, 2)) if len(E) else np.zeros(0)
    left = np.concatenate([[0.0], enorm])                        # ||E_{i-1}||
    right = np.concatenate([enorm, [0.0]])                       # ||E_i||
    lo = float((lam_d - left - right).min()) - 1e-9             # block Gershgorin: SPD below
    hi = float(lam_d.min())                                      # Rayleigh quotient on one block
    assert _spd_at(GG, E, lo)
    workers = max(2, min(16, os.cpu_count() or 2))
    with ThreadPoolExecutor(workers) as ex:
        while hi - lo > tol:
            sig = np.linspace(lo, hi, workers + 2)[1:-1]
            ok = list(ex.map(lambda s: _spd_at(GG, E, s), sig))
            for s, good in zip(sig, ok):
                if good:
                    lo = max(lo, s)
                else:
                    hi = min(hi, s)
    return lo  # the shifted matrix keeps lambda_min in [c, c + tol]


