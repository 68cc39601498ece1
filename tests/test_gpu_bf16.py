"""BF16 Schur / fill products with FP64 refinement (BTC_BF16_IR) through the
C ABI, against the FP64 oracle.

Every result is refined to a max-column relative residual <= 1e-10 measured
by the oracle's FP64 matvec; the device-reported residual agrees with it; the
factor blocks agree with the oracle's to BF16-product accuracy; batched runs
equal single runs bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    b.lib()
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def solve_bf16(btc, p, max_refine=0):
    f = btc.Factor(dev(p.D), dev(p.E), precision=btc.BTC_BF16_IR, max_refine=max_refine)
    X, info = f.solve(dev(p.B), want_info=True)
    st = f.info
    blocks = f.export()
    X = X.cpu().numpy()
    f.close()
    return st, info, blocks, X


@pytest.mark.parametrize("N,n", [(1, 5), (7, 12), (33, 16), (64, 24), (100, 32), (65, 48), (40, 64), (17, 80),
                                 (33, 96), (20, 128)])
def test_bf16_refines_to_target(btc, N, n):
    p = inputs.block_tridiag(N, n, seed=900 + N + n, nrhs=2)
    st, info, blocks, X = solve_bf16(btc, p)
    assert st == 0
    assert info["converged"], info
    rr = oracle.relres(p.D, p.E, X, p.B)
    assert rr <= TOL
    assert abs(info["relres"] - rr) <= 0.5 * rr + 1e-15
    Ld, Rb, Tb, _ = oracle.factor_nd(p.D, p.E)
    scale = max(np.abs(Ld).max(), 1.0)
    for g, o in zip(blocks, (Ld, Rb, Tb)):
        assert np.abs(g - o).max() <= 3e-2 * scale


@pytest.mark.parametrize("c", [4.0, 0.1, 0.001])
def test_bf16_conditioning_sweep_margin_reading(btc, c):
    """lambda_min(Psi) = c (margin reading): condition numbers ~3 to ~1e4.
    The refinement converges, or stops as stalled with its residual
    reported; the well-conditioned cases must converge."""
    p = inputs.block_tridiag(128, 32, c=c, seed=11, nrhs=2, margin=True)
    st, info, _, X = solve_bf16(btc, p, max_refine=30)
    assert st == 0
    rr = oracle.relres(p.D, p.E, X, p.B)
    assert np.isfinite(rr)
    assert abs(info["relres"] - rr) <= 0.5 * rr + 1e-15
    if c >= 0.1:
        assert info["converged"] and rr <= TOL, info
    else:
        assert (info["converged"] and rr <= TOL) or info["steps"] > 1, info


def test_bf16_batched_equals_single(btc):
    rng = np.random.default_rng(4)
    prs = [inputs.block_tridiag(int(rng.integers(2, 150)), int(rng.choice([8, 30, 64, 90])), seed=k, nrhs=1)
           for k in range(8)]
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, btc.BTC_BF16_IR) for p in prs]
    Bs = [dev(p.B) for p in prs]
    Xs = [torch.empty_like(b) for b in Bs]
    r.factor_batched(hs, [dev(p.D) for p in prs], [dev(p.E) for p in prs])
    r.solve_batched(hs, Bs, Xs, 1)
    r.sync()
    for k, p in enumerate(prs):
        _, info, _, Xs1 = solve_bf16(btc, p)
        assert np.array_equal(Xs[k].cpu().numpy(), Xs1)
        assert btc.btc_refine_info(hs[k])["converged"]
        assert oracle.relres(p.D, p.E, Xs1, p.B) <= TOL
        btc.btc_destroy(hs[k])
    r.close()


@pytest.mark.parametrize("c", [4.0, 0.001])
@pytest.mark.parametrize("m", [1, 3])
def test_gmres_refinement_small(btc, c, m):
    """GMRES-based refinement on a small ill-conditioned instance: target met
    in a few corrections; each right-hand side is its own problem (the same
    result column by column as solved alone)."""
    p = inputs.block_tridiag(128, 32, c=c, seed=11, nrhs=m, margin=True)
    f = btc.Factor(dev(p.D), dev(p.E), precision=btc.BTC_BF16_IR, refine=btc.BTC_REFINE_GMRES)
    X, info = f.solve(dev(p.B), want_info=True)
    X = X.cpu().numpy()
    assert info["converged"] and info["steps"] <= 3 and info["inner"] >= 1, info
    assert oracle.relres(p.D, p.E, X, p.B) <= TOL
    if m > 1:
        X0, _ = f.solve(dev(np.ascontiguousarray(p.B[:, :, :1])), want_info=True)
        assert oracle.relres(p.D, p.E, X0.cpu().numpy(), p.B[:, :, :1]) <= TOL
    f.close()
