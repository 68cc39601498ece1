"""The window construction of tests/blockwin.py reproduces the oracle's whole
factor (CPU)."""
import numpy as np
import pytest

import oracle
from blockwin import window_blocks
from paper_2601_03754_amd import inputs


@pytest.mark.parametrize("N", [45, 64, 33])
def test_window_blocks_match_whole_factor(N):
    """The window construction reproduces the oracle's whole factor (small
    instance, every node of levels 0..3)."""
    pr = inputs.block_tridiag(N, 5, seed=3)
    Ld, Rb, Tb, info = oracle.factor_nd(pr.D, pr.E)
    assert info == 0
    for i in range(1, N + 1):
        l = oracle.level_of(i)
        if l > 3:
            continue
        s = 1 << l
        L, R, T = window_blocks(pr.D, pr.E, i, s)
        assert np.abs(L - Ld[i - 1]).max() <= 1e-12
        if R is not None:
            assert np.abs(R - Rb[i - 1]).max() <= 1e-12
        if T is not None:
            assert np.abs(T - Tb[i - 1]).max() <= 1e-12
