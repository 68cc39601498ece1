"""Oracle factor blocks of one node of a long chain, from the short windows of
the chain that determine them (test helper)."""
import numpy as np

import oracle


# Factor blocks of node i (level l, stride s = 2^l) depend only on the blocks
# strictly between i-s and i+s and on the couplings to i-s and i+s.  On the
# window of 2s blocks (i-s, i+s], renumbered from 1 (a shift by a multiple of
# 2s, so every level below l keeps its nodes), node i is node s of level l
# with right neighbour 2s: its L_ii and R_i are the window's.  T_i comes from
# the mirrored window [i-s, i+s): reversing the chain turns the coupling to
# i-s into node s's right coupling, so T_i is the transpose of that R.

def window_blocks(D, E, i, s):
    N = D.shape[0]
    lo, hi = i - s, min(i + s, N)  # right window: blocks lo+1 .. hi (1-based)
    Dr = D[lo:hi]
    Er = E[lo:hi - 1]
    Lw, Rw, _, info = oracle.factor_nd(Dr, Er)
    assert info == 0
    L, R = Lw[s - 1], (Rw[s - 1] if i + s <= N else None)
    T = None
    if i > s:
        # blocks i+s-1 down to i-s, renumbered 1 .. 2s
        top = min(i + s - 1, N)
        idx = np.arange(top, i - s - 1, -1)            # 1-based original indices, descending
        Dm = D[idx - 1]
        Em = np.stack([E[j - 2].T for j in idx[:-1]])  # block (j-1, j) of the chain is E_{j-1}^T
        off = (i + s) - top - 1                        # keep node i at local index s
        if off:
            # the window is cut by the end of the chain: pad on the far side
            # with decoupled identity blocks so that node i stays at local s
            n = D.shape[1]
            Dm = np.concatenate([np.tile(np.eye(n), (off, 1, 1)), Dm])
            Em = np.concatenate([np.zeros((off, n, n)), Em])
        Lm, Rm, _, info = oracle.factor_nd(Dm, Em)
        assert info == 0
        T = Rm[s - 1].T
        assert np.abs(Lm[s - 1] - L).max() <= 1e-12 * np.abs(L).max()
    return L, R, T
