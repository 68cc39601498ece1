"""The benchmark configurations at their own sizes, through the C ABI, against
the FP64 CPU oracle.

* Conditioning sweep: N = 4096, n = 64, four right-hand sides, FP32 and BF16
  products with FP64 refinement, diagonal shift read as the spectral margin
  c in {4, 0.1, 0.001} (lambda_min(Psi) = c).  The oracle's FP64 matvec
  measures the relative residual of every result, the oracle's FP64 solution
  the forward error, and the refinement steps are recorded.
* The many-instance batch: all 512 instances (N ~ U{32..2048}, n in {8, 16,
  24, 32, 48}), FP32 factors with FP64 refinement, batched equal to single bit
  for bit and every result within 1e-10.
* The largest FP64 sweep point, N = 16384, n = 128: residual, and factor
  blocks of levels 0 to 5 checked one by one against the oracle on the
  windows of the chain that determine them.

Set BTC_TEST_RECORD to a file path to append the measured outcomes (JSON
lines)."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from blockwin import window_blocks
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


def record(**kw):
    path = os.environ.get("BTC_TEST_RECORD")
    line = json.dumps(kw, sort_keys=True)
    print(line, flush=True)
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")


# ---------------------------------------------------------------------------
from margin import lambda0_bisect  # noqa: E402


@pytest.fixture(scope="module")
def sweep_problems():
    N, n, m, seed = 4096, 64, 4, 11
    GG, E, _ = inputs.unshifted(N, n, seed=seed, nrhs=m)
    lam0 = lambda0_bisect(GG, E)
    del GG, E
    cs = (4.0, 0.1, 0.001)
    prs = [inputs.block_tridiag(N, n, c=c, seed=seed, nrhs=m, margin=True, lam0=lam0) for c in cs]
    with ThreadPoolExecutor(len(cs)) as ex:
        Xos = list(ex.map(lambda pr: oracle.solve(pr.D, pr.E, pr.B), prs))
    return lam0, {c: (pr, Xo) for c, pr, Xo in zip(cs, prs, Xos)}


def lambda_max_bound(pr):
    """Block Gershgorin: lambda_max(Psi) <= max_i lambda_max(D_i) + ||E_{i-1}||
    + ||E_i|| (spectral norms)."""
    Dsym = np.tril(pr.D) + np.tril(pr.D, -1).transpose(0, 2, 1)
    lam = np.linalg.eigvalsh(Dsym).max(axis=1)
    en = np.linalg.norm(pr.E, ord=2, axis=(1, 2))
    return float((lam + np.concatenate([[0.0], en]) + np.concatenate([en, [0.0]])).max())


def colwise_rel(X, Xo):
    d = (X - Xo).reshape(-1, X.shape[-1])
    o = Xo.reshape(-1, X.shape[-1])
    return float((np.linalg.norm(d, axis=0) / np.linalg.norm(o, axis=0)).max())


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("c", [4.0, 0.1, 0.001])
def test_conditioning_sweep_full_size(btc, sweep_problems, c, prec):
    lam0, probs = sweep_problems
    pr, Xo = probs[c]
    precision = btc.BTC_FP32_IR if prec == "fp32" else btc.BTC_BF16_IR
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=precision)
    X, info = f.solve(dev(pr.B), want_info=True)
    st = f.info
    f.close()
    X = X.cpu().numpy()
    assert st == 0
    rr = oracle.relres(pr.D, pr.E, X, pr.B)
    fwd = colwise_rel(X, Xo)
    kappa = lambda_max_bound(pr) / c  # lambda_min(Psi) = c (margin reading)
    record(test="conditioning_sweep", N=pr.N, n=pr.n, nrhs=pr.nrhs, c=c, lam0=lam0, precision=prec,
           steps=info["steps"], converged=info["converged"], relres_device=info["relres"], relres_oracle=rr,
           forward_error=fwd, kappa_bound=kappa)
    # the device's own residual is the oracle's (the reported outcome is true)
    assert abs(info["relres"] - rr) <= 1e-3 * rr + 1e-16
    if prec == "fp32" or c >= 0.1:
        assert info["converged"], info
        assert rr <= TOL
        # ||x - x*|| / ||x*|| <= kappa ||r|| / ||b|| per column, the oracle's
        # own solution carrying an error of order kappa * 1e-16
        assert fwd <= 2.0 * kappa * (rr + 1e-15)
    else:
        # BF16 products at kappa ~ 1e4: either the target is reached, or
        # refinement stops and says so
        assert info["converged"] == (rr <= TOL)


# ---------------------------------------------------------------------------
def test_many_instance_batch_full(btc):
    """All 512 instances of the batch workload: batched factor + refined solve
    equal the single-instance results bit for bit, each within 1e-10."""
    shapes = inputs.batch_shapes(512, seed=0)
    r = btc.Runner()
    hs, Ds, Es, Bs, prs = [], [], [], [], []
    for k, (N, n) in enumerate(shapes):
        pr = inputs.block_tridiag(N, n, seed=k, nrhs=1)
        prs.append(pr)
        Ds.append(dev(pr.D))
        Es.append(dev(pr.E))
        Bs.append(dev(pr.B))
        hs.append(btc.btc_create(N, n, btc.BTC_FP32_IR))
    Xs = [torch.empty_like(b) for b in Bs]
    fi = r.factor_batched(hs, Ds, Es, want_info=True)
    si = r.solve_batched(hs, Bs, Xs, want_info=True)
    assert all(v == 0 for v in fi)
    steps = []
    for k, pr in enumerate(prs):
        Xb = Xs[k].cpu().numpy()
        assert si[k]["converged"], (k, si[k])
        assert oracle.relres(pr.D, pr.E, Xb, pr.B) <= TOL, k
        f = btc.Factor(Ds[k], Es[k], precision=btc.BTC_FP32_IR)
        Xa = f.solve(Bs[k]).cpu().numpy()
        f.close()
        assert np.array_equal(Xb, Xa), k
        steps.append(si[k]["steps"])
        btc.btc_destroy(hs[k])
    r.close()
    record(test="many_instance_batch", instances=len(prs), steps_max=int(max(steps)),
           steps_hist={str(s): int(sum(1 for x in steps if x == s)) for s in sorted(set(steps))})


def test_fp64_largest_sweep_point(btc):
    N, n = 16384, 128
    pr = inputs.block_tridiag(N, n, c=4.0, seed=inputs.sweep_seed(N, n), nrhs=1)
    f = btc.Factor(dev(pr.D), dev(pr.E))
    X = f.solve(dev(pr.B)).cpu().numpy()
    assert f.info == 0
    Ld, Rb, Tb = f.export()
    f.close()
    rr = oracle.relres(pr.D, pr.E, X, pr.B)
    record(test="fp64_16384_128", relres=rr)
    assert rr <= 1e-12
    rng = np.random.default_rng(1)
    for l in range(6):
        s = 1 << l
        nodes = np.arange(s, N + 1, 2 * s)
        for i in rng.choice(nodes, size=min(3, len(nodes)), replace=False):
            L, R, T = window_blocks(pr.D, pr.E, int(i), s)
            sc = max(1.0, np.abs(L).max())
            assert np.abs(Ld[i - 1] - L).max() <= 1e-12 * sc, (l, i)
            if R is not None:
                assert np.abs(Rb[i - 1] - R).max() <= 1e-12 * max(1.0, np.abs(R).max()), (l, i)
            if T is not None:
                assert np.abs(Tb[i - 1] - T).max() <= 1e-12 * max(1.0, np.abs(T).max()), (l, i)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("c", [4.0, 0.001])
def test_conditioning_sweep_gmres_refinement(btc, sweep_problems, c, prec):
    """GMRES-based refinement (the low-precision factor as preconditioner of
    FP64 GMRES on the correction equation) at the full size: converges to
    the target at every margin, also with BF16 products at kappa ~ 1e4, in
    few corrections."""
    lam0, probs = sweep_problems
    pr, Xo = probs[c]
    precision = btc.BTC_FP32_IR if prec == "fp32" else btc.BTC_BF16_IR
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=precision, refine=btc.BTC_REFINE_GMRES)
    X, info = f.solve(dev(pr.B), want_info=True)
    f.close()
    X = X.cpu().numpy()
    rr = oracle.relres(pr.D, pr.E, X, pr.B)
    fwd = colwise_rel(X, Xo)
    kappa = lambda_max_bound(pr) / c
    record(test="conditioning_sweep_gmres", N=pr.N, n=pr.n, nrhs=pr.nrhs, c=c, precision=prec,
           steps=info["steps"], inner=info["inner"], converged=info["converged"], relres_device=info["relres"],
           relres_oracle=rr, forward_error=fwd, kappa_bound=kappa)
    assert info["converged"], info
    assert rr <= TOL
    assert abs(info["relres"] - rr) <= 1e-3 * rr + 1e-16
    assert fwd <= 2.0 * kappa * (rr + 1e-15)
    assert info["steps"] <= 3
