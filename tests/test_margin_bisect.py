"""The identity shift of the full-size conditioning sweep (lambda_min of the
assembled matrix equal to the margin c) uses lambda_min of the unshifted
matrix found by bisection on the success of the oracle's block Cholesky
(Sylvester's law of inertia).  Pinned here against LAPACK's banded symmetric
eigensolver at sizes where that one is quick.  CPU only."""
import pytest

from paper_2601_03754_amd import inputs
from margin import lambda0_bisect


@pytest.mark.parametrize("N,n,seed", [(64, 8, 1), (200, 12, 2), (33, 20, 3)])
def test_bisection_matches_lapack(N, n, seed):
    GG, E, _ = inputs.unshifted(N, n, seed=seed)
    lam = inputs.lambda_min(GG, E)
    got = lambda0_bisect(GG, E)
    assert lam - 2e-7 <= got <= lam + 1e-12
