"""Block-banded and arrow extensions on the GPU against the oracle
(oracle/structures.py): the super-block factor element by element, the tip's
Cholesky factor and Psi^{-1} F, the solutions, the breakdown reports, and the
edge cases (a bandwidth that does not divide N, N smaller than the bandwidth,
one block row, an empty tip, the largest super-block and tip)."""
import numpy as np
import pytest

import oracle
from oracle import structures as st
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu

PREC = {"fp64": 0, "fp32_ir": 1, "bf16_ir": 2}


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    b.lib()
    return b


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def band_relres(A_band, b, X, B):
    """max-column relative residual of the banded system, through the
    super-block matrix (the completion rows carry zeros)."""
    N, _, n, _ = A_band.shape
    D2, E2 = st.band_to_tridiag(A_band, b)
    N2, n2 = D2.shape[0], D2.shape[1]
    q = B.shape[-1]
    pad = lambda V: np.vstack([V.reshape(N * n, q), np.zeros((N2 * n2 - N * n, q))]).reshape(N2, n2, q)
    return oracle.relres(D2, E2, pad(X), pad(B))


@pytest.mark.parametrize("N,n,b,prec", [
    (1000, 16, 4, "fp64"), (1000, 16, 4, "fp32_ir"),
    (777, 8, 3, "fp64"),          # b does not divide N: identity completion
    (50, 1, 64, "fp64"),          # scalar band of bandwidth 64
    (300, 32, 4, "fp64"),         # super-blocks of the largest order, 128
    (300, 32, 4, "bf16_ir"),
    (5, 4, 7, "fp64"),            # N < b: one super-block
    (1, 3, 2, "fp64"),            # one block row
])
def test_banded_matches_oracle(btc, N, n, b, prec):
    import torch
    pr = inputs.block_banded(N, n, b, seed=31 * N + b, nrhs=2)
    f = btc.Banded(dev(pr.A_band), precision=PREC[prec])
    X, inf = f.solve(dev(pr.B), want_info=True)
    torch.cuda.synchronize()
    assert f.info == 0
    Xg = X.cpu().numpy()
    want = st.banded_solve(pr.A_band, b, pr.B)
    rr = band_relres(pr.A_band, b, Xg, pr.B)
    print("banded N=%d n=%d b=%d %s: relres %.2e, steps %d" % (N, n, b, prec, rr, inf["steps"]))
    assert rr <= 1e-10
    assert inf["converged"]
    if prec == "fp64":
        np.testing.assert_allclose(Xg, want, rtol=0, atol=1e-11 * np.abs(want).max())
        Ld, Rb, Tb, info = st.banded_factor(pr.A_band, b)
        assert info == 0
        for got, ref in zip(f.export(), (Ld, Rb, Tb)):
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    else:
        np.testing.assert_allclose(Xg, want, rtol=0, atol=1e-8 * np.abs(want).max())
    f.close()


def test_banded_refactor_and_breakdown(btc):
    import torch
    N, n, b = 64, 6, 3
    p1 = inputs.block_banded(N, n, b, seed=1, nrhs=1)
    p2 = inputs.block_banded(N, n, b, seed=2, nrhs=1)
    f = btc.Banded(dev(p1.A_band))
    f.refactor(dev(p2.A_band))
    X = f.solve(dev(p2.B)).cpu().numpy()
    g = btc.Banded(dev(p2.A_band))
    np.testing.assert_array_equal(X, g.solve(dev(p2.B)).cpu().numpy())
    # an indefinite diagonal block: the failing super-block as the oracle finds it
    bad = p2.A_band.copy()
    bad[40, 0] -= 60.0 * np.eye(n)
    f.refactor(dev(bad))
    torch.cuda.synchronize()
    _, _, _, info = st.banded_factor(bad, b)
    assert info > 0 and f.info == info
    f.close()
    g.close()


def arrow_relres(pr, X):
    N, n, _ = pr.D.shape
    K = N * n
    x1, x2 = X[:K], X[K:]
    q = X.shape[1]
    r1 = oracle.residual(pr.D, pr.E, x1.reshape(N, n, q), pr.B[:K].reshape(N, n, q)).reshape(K, q) - pr.F @ x2
    C = np.tril(pr.C) + np.tril(pr.C, -1).T
    r2 = pr.B[K:] - pr.F.T @ x1 - C @ x2
    r = np.sqrt((r1 ** 2).sum(0) + (r2 ** 2).sum(0))
    return float((r / np.linalg.norm(pr.B, axis=0)).max())


@pytest.mark.parametrize("N,n,m,prec", [
    (500, 16, 32, "fp64"), (500, 16, 32, "fp32_ir"),
    (64, 8, 1, "fp64"),
    (300, 32, 128, "fp64"),       # the largest tip
    (200, 24, 40, "bf16_ir"),
    (3, 4, 5, "fp64"),
    (1, 3, 2, "fp64"),            # one block row
    (100, 8, 0, "fp64"),          # no border
])
def test_arrow_matches_oracle(btc, N, n, m, prec):
    import torch
    pr = inputs.arrow(N, n, m, seed=7 * N + m, nrhs=3)
    a = btc.Arrow(dev(pr.D), dev(pr.E), dev(pr.F), dev(pr.C), precision=PREC[prec])
    X, inf = a.solve(dev(pr.B), want_info=True)
    torch.cuda.synchronize()
    assert a.info == (0, 0)
    Xg = X.cpu().numpy()
    fac = st.arrow_factor(pr.D, pr.E, pr.F, pr.C)
    want = st.arrow_solve(fac, pr.B)
    rr = arrow_relres(pr, Xg)
    print("arrow N=%d n=%d m=%d %s: relres %.2e, steps %d" % (N, n, m, prec, rr, inf["steps"]))
    Ls, Z = a.export()
    if prec == "fp64":
        assert rr <= 1e-12
        np.testing.assert_allclose(Xg, want, rtol=0, atol=1e-11 * np.abs(want).max())
        if m:
            np.testing.assert_allclose(Ls, fac["Ls"], rtol=0, atol=1e-12 * np.abs(fac["Ls"]).max())
            np.testing.assert_allclose(Z, fac["Z"].reshape(N * n, m), rtol=0,
                                       atol=1e-12 * np.abs(fac["Z"]).max())
    else:
        assert rr <= 5e-10
        np.testing.assert_allclose(Xg, want, rtol=0, atol=1e-7 * np.abs(want).max())
        if m:
            np.testing.assert_allclose(Ls, fac["Ls"], rtol=0, atol=1e-7 * np.abs(fac["Ls"]).max())
    a.close()


def test_arrow_refactor_repeated_solves_and_breakdowns(btc):
    import torch
    N, n, m = 90, 12, 9
    p1 = inputs.arrow(N, n, m, seed=1, nrhs=2)
    p2 = inputs.arrow(N, n, m, seed=2, nrhs=5)
    a = btc.Arrow(dev(p1.D), dev(p1.E), dev(p1.F), dev(p1.C))
    a.refactor(dev(p2.D), dev(p2.E), dev(p2.F), dev(p2.C))
    g = btc.Arrow(dev(p2.D), dev(p2.E), dev(p2.F), dev(p2.C))
    B5 = dev(p2.B)
    np.testing.assert_array_equal(a.solve(B5).cpu().numpy(), g.solve(B5).cpu().numpy())
    # a second solve of another width on the same object
    B1 = dev(p2.B[:, :1].copy())
    x5 = g.solve(B5).cpu().numpy()[:, :1]
    np.testing.assert_allclose(a.solve(B1).cpu().numpy(), x5, rtol=0, atol=1e-13 * np.abs(x5).max())
    # an indefinite tip: the failing column as the oracle finds it
    C = p2.C.copy()
    C[4, 4] = -80.0
    a.refactor(dev(p2.D), dev(p2.E), dev(p2.F), dev(C))
    torch.cuda.synchronize()
    fac = st.arrow_factor(p2.D, p2.E, p2.F, C)
    assert fac["info_tip"] > 0 and a.info == (0, fac["info_tip"])
    # an indefinite Psi: reported for Psi
    D = p2.D.copy()
    D[17] -= 90.0 * np.eye(n)
    a.refactor(dev(D), dev(p2.E), dev(p2.F), dev(p2.C))
    torch.cuda.synchronize()
    _, _, _, info = oracle.factor_nd(D, p2.E)
    assert info > 0 and a.info[0] == info
    a.close()
    g.close()
