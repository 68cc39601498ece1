"""Autotuned kernel variants through the C ABI: every variant of every
tunable family meets the oracle's accuracy, the column-grouping variants of
the sweeps and residual give bit-identical results, batched runs follow the
table exactly as single-instance runs do, and btc_autotune picks variants
that keep all of this true."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    b.lib()
    yield b
    for op in (0, 1, 2, 3):
        for n in (16, 32, 64):
            for lvl in (0, 1):
                for prec in (0, 1, 2):
                    try:
                        b.btc_tune_set(op, prec, n, lvl, 1 if (op == 0 and n == 64) else 0)
                    except b.BtcError:
                        pass


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run(btc, p, precision=0):
    f = btc.Factor(dev(p.D), dev(p.E), precision=precision)
    X = f.solve(dev(p.B)).cpu().numpy()
    blocks = f.export()
    f.close()
    return X, blocks


@pytest.mark.parametrize("n,variant", [(12, 0), (12, 1), (24, 0), (24, 1), (24, 2), (32, 0), (32, 1), (32, 2)])
def test_factor_variants_match_oracle(btc, n, variant):
    p = inputs.block_tridiag(77, n, seed=400 + n, nrhs=2)
    btc.btc_tune_set(0, 0, n, 0, variant)
    btc.btc_tune_set(0, 0, n, 1, variant)
    X, blocks = run(btc, p)
    btc.btc_tune_set(0, 0, n, 0, 0)
    btc.btc_tune_set(0, 0, n, 1, 0)
    Ld, Rb, Tb, info = oracle.factor_nd(p.D, p.E)
    scale = max(np.abs(Ld).max(), 1.0)
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= 1e-12 * scale
    assert oracle.relres(p.D, p.E, X, p.B) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("n", [40, 64])
@pytest.mark.parametrize("variant", [0, 1])
def test_factor_variants_at_64(btc, precision, n, variant):
    """Padded size 64 through the one-workgroup-per-node kernel (variant 0)
    or the tile-parallel level step (variant 1, the default) at every level:
    oracle accuracy for FP64, refinement target for mixed."""
    p = inputs.block_tridiag(150, n, seed=600 + n, nrhs=2)
    btc.btc_tune_set(0, precision, n, 0, variant)
    btc.btc_tune_set(0, precision, n, 1, variant)
    f = btc.Factor(dev(p.D), dev(p.E), precision=precision)
    X, info = f.solve(dev(p.B), want_info=True)
    X = X.cpu().numpy()
    blocks = f.export()
    f.close()
    btc.btc_tune_set(0, precision, n, 0, 1)
    btc.btc_tune_set(0, precision, n, 1, 1)
    Ld, Rb, Tb, _ = oracle.factor_nd(p.D, p.E)
    scale = max(np.abs(Ld).max(), 1.0)
    ftol = {0: 1e-12, 1: 1e-4, 2: 3e-2}[precision]
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= ftol * scale
    assert oracle.relres(p.D, p.E, X, p.B) <= (1e-12 if precision == 0 else 1e-10)
    assert info["converged"]


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("v0,v1", [(1, 0), (0, 1)])
def test_factor_families_mixed_across_levels(btc, precision, v0, v1):
    """Padded size 64 with the tile-parallel step at level 0 only, or above
    level 0 only: the separator updates deferred or applied eagerly follow
    the kernel family of each level (no update lost or applied twice)."""
    n = 56
    p = inputs.block_tridiag(200, n, seed=700 + v0, nrhs=2)
    btc.btc_tune_set(0, precision, n, 0, v0)
    btc.btc_tune_set(0, precision, n, 1, v1)
    try:
        f = btc.Factor(dev(p.D), dev(p.E), precision=precision)
        X, info = f.solve(dev(p.B), want_info=True)
        X = X.cpu().numpy()
        blocks = f.export()
        f.close()
    finally:
        btc.btc_tune_set(0, precision, n, 0, 1)
        btc.btc_tune_set(0, precision, n, 1, 1)
    Ld, Rb, Tb, _ = oracle.factor_nd(p.D, p.E)
    scale = max(np.abs(Ld).max(), 1.0)
    ftol = {0: 1e-12, 1: 1e-4, 2: 3e-2}[precision]
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= ftol * scale
    assert oracle.relres(p.D, p.E, X, p.B) <= (1e-12 if precision == 0 else 1e-10)
    assert info["converged"]


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("v0,v1", [(1, 1), (1, 0), (0, 1)])
def test_tiled_step_at_32(btc, precision, v0, v1):
    """Padded size 32 through the tile-parallel level step at every level, at
    level 0 only, or above level 0 only (FP64 variant 2, mixed variant 1;
    the one-workgroup kernels elsewhere): oracle accuracy for FP64,
    refinement target for mixed, no separator update lost or applied twice."""
    n = 28
    tiled = 2 if precision == 0 else 1
    p = inputs.block_tridiag(300, n, seed=900 + 3 * v0 + v1, nrhs=2)
    before = [btc.btc_tune_get(0, precision, n, lv) for lv in (0, 1)]
    btc.btc_tune_set(0, precision, n, 0, tiled if v0 else 0)
    btc.btc_tune_set(0, precision, n, 1, tiled if v1 else 0)
    try:
        f = btc.Factor(dev(p.D), dev(p.E), precision=precision)
        X, info = f.solve(dev(p.B), want_info=True)
        X = X.cpu().numpy()
        blocks = f.export()
        f.close()
    finally:
        btc.btc_tune_set(0, precision, n, 0, before[0])
        btc.btc_tune_set(0, precision, n, 1, before[1])
    Ld, Rb, Tb, _ = oracle.factor_nd(p.D, p.E)
    scale = max(np.abs(Ld).max(), 1.0)
    ftol = {0: 1e-12, 1: 1e-4, 2: 3e-2}[precision]
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= ftol * scale
    assert oracle.relres(p.D, p.E, X, p.B) <= (1e-12 if precision == 0 else 1e-10)
    assert info["converged"]


@pytest.mark.parametrize("precision", [0, 1])
def test_column_grouping_is_bitwise_neutral(btc, precision):
    p = inputs.block_tridiag(65, 40, seed=5, nrhs=3)
    outs = []
    for v in (0, 1):
        for op in (1, 2, 3):
            btc.btc_tune_set(op, precision, 40, 0, v)
        outs.append(run(btc, p, precision)[0])
    for op in (1, 2, 3):
        btc.btc_tune_set(op, precision, 40, 0, 0)
    assert np.array_equal(outs[0], outs[1])
    assert oracle.relres(p.D, p.E, outs[0], p.B) <= (1e-12 if precision == 0 else 1e-10)


def test_batched_follows_table_like_single(btc):
    btc.btc_tune_set(0, 0, 30, 1, 1)  # VALU kernel above level 0 for padded 32
    prs = [inputs.block_tridiag(N, 30, seed=N, nrhs=1) for N in (9, 40, 100)]
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, 0) for p in prs]
    Xs = [torch.empty_like(dev(p.B)) for p in prs]
    r.factor_batched(hs, [dev(p.D) for p in prs], [dev(p.E) for p in prs])
    r.solve_batched(hs, [dev(p.B) for p in prs], Xs, 1)
    r.sync()
    for k, p in enumerate(prs):
        Xsng, _ = run(btc, p)
        assert np.array_equal(Xs[k].cpu().numpy(), Xsng)
        btc.btc_destroy(hs[k])
    r.close()
    btc.btc_tune_set(0, 0, 30, 1, 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_keeps_results_correct(btc, precision):
    p = inputs.block_tridiag(300, 28, seed=8, nrhs=4)
    D, E, B = dev(p.D), dev(p.E), dev(p.B)
    X = torch.empty_like(B)
    h = btc.btc_create(p.N, p.n, precision)
    btc.btc_autotune(h, D, E, B, X, reps=2)
    torch.cuda.synchronize()
    for op, lvl in ((0, 0), (0, 1), (1, 0), (2, 0), (3, 0)):
        assert btc.btc_tune_get(op, precision, 28, lvl) in (0, 1)
    btc.btc_destroy(h)
    X2, _ = run(btc, p, precision)
    assert oracle.relres(p.D, p.E, X2, p.B) <= (1e-12 if precision == 0 else 1e-10)


@pytest.mark.parametrize("precision,N,n", [(0, 4096, 24), (1, 1500, 40), (1, 300, 96), (0, 77, 128)])
def test_sweep_shapes_identical(btc, precision, N, n):
    """The sweep launch shapes (level ranges with 4- or 8-wavefront
    workgroups, one launch per level) do the same arithmetic per node:
    identical solutions, single handle and batched."""
    from paper_2601_03754_amd import inputs
    pr = inputs.block_tridiag(N, n, seed=N + n, nrhs=2)
    D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
    S = 6  # BTC_TUNE_SWEEP_SHAPE
    old = btc.btc_tune_get(S, precision, n, 0)
    outs = []
    try:
        for v in (0, 1, 2):
            btc.btc_tune_set(S, precision, n, 0, v)
            f = btc.Factor(D, E, precision=precision)
            outs.append(f.solve(B).cpu().numpy())
            r = btc.Runner()
            h = btc.btc_create(N, n, precision)
            X = torch.empty_like(B)
            r.factor_batched([h], [D], [E])
            r.solve_batched([h], [B], [X])
            r.sync()
            outs.append(X.cpu().numpy())
            btc.btc_destroy(h)
            r.close()
            f.close()
    finally:
        btc.btc_tune_set(S, precision, n, 0, old)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    tol = 1e-12 if precision == 0 else 1e-10
    assert oracle.relres(pr.D, pr.E, outs[0], pr.B) <= tol


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_batched_keeps_results_correct(btc, precision):
    """btc_autotune_batched on a small mixed batch: the instances come back
    factored and solved within the path's accuracy, and every key holds a
    valid variant (the previous table is restored afterwards)."""
    shapes = [(37, 7), (120, 16), (64, 28), (200, 40), (9, 60), (301, 12)]
    keys = [(op, n, lvl) for op in (0, 1, 2, 3, 6) for n in (7, 16, 28, 40, 60, 12) for lvl in (0, 1)]
    saved = {k: btc.btc_tune_get(k[0], precision, k[1], k[2]) for k in keys}
    prs = [inputs.block_tridiag(N, n, seed=5 + k, nrhs=2) for k, (N, n) in enumerate(shapes)]
    r = btc.Runner()
    hs = [btc.btc_create(N, n, precision) for N, n in shapes]
    Ds, Es, Bs = [dev(p.D) for p in prs], [dev(p.E) for p in prs], [dev(p.B) for p in prs]
    Xs = [torch.empty_like(b) for b in Bs]
    try:
        r.autotune(hs, Ds, Es, Bs, Xs, reps=1)
        torch.cuda.synchronize()
        for (op, n, lvl) in keys:
            assert btc.btc_tune_get(op, precision, n, lvl) in (0, 1, 2)
        for p, X in zip(prs, Xs):
            assert oracle.relres(p.D, p.E, X.cpu().numpy(), p.B) <= (1e-12 if precision == 0 else 1e-10)
    finally:
        for k, v in saved.items():
            btc.btc_tune_set(k[0], precision, k[1], k[2], v)
        for h in hs:
            btc.btc_destroy(h)
        r.close()
