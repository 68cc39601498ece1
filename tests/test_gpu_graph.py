"""Level schedules captured as HIP graphs (btc_graph_*), through the C ABI.

A graph records the runner calls of a batched factorization and solve and
replays them with no host work per level.  Every replay must equal the eager
run of the same calls bit for bit (same kernels, same descriptors), also with
other eager work and synchronisations between replays, and a replay after new
values are written into the recorded input buffers must equal an eager
factor+solve of the new matrices (the repeated re-solve of an MPC loop); the
eager results themselves are checked against the FP64 oracle."""
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
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def shapes(seed, count):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(1, 200)), int(rng.choice([5, 16, 24, 40, 64, 80, 128]))) for _ in range(count)]


def eager(btc, prs, precision):
    out = []
    for p in prs:
        f = btc.Factor(dev(p.D), dev(p.E), precision=precision)
        out.append(f.solve(dev(p.B)).cpu().numpy())
        f.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager_and_follow_new_values(btc, precision):
    shp = shapes(3 + precision, 8)
    prs = [inputs.block_tridiag(N, n, seed=70 + k, nrhs=1) for k, (N, n) in enumerate(shp)]
    prs2 = [inputs.block_tridiag(N, n, seed=170 + k, nrhs=1) for k, (N, n) in enumerate(shp)]
    Ds = [dev(p.D) for p in prs]
    Es = [dev(p.E) for p in prs]
    Bs = [dev(p.B) for p in prs]
    Xs = [torch.full_like(b, float("nan")) for b in Bs]
    r = btc.Runner()
    hs = [btc.btc_create(p.N, p.n, precision) for p in prs]
    r.graph_begin()
    r.factor_batched(hs, Ds, Es)
    r.solve_batched(hs, Bs, Xs, 1)
    g = r.graph_end()
    ref = eager(btc, prs, precision)
    tol = 1e-12 if precision == 0 else 1e-10
    for k, p in enumerate(prs):
        assert oracle.relres(p.D, p.E, ref[k], p.B) <= tol
    side = inputs.block_tridiag(50, 12, seed=9)
    for rep in range(3):
        for x in Xs:
            x.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        for k in range(len(prs)):
            assert np.array_equal(Xs[k].cpu().numpy(), ref[k]), (rep, k)
            assert btc.btc_status(hs[k]) == 0
        eager(btc, [side], precision)  # unrelated eager work between replays
        torch.cuda.synchronize()
    # new matrix values and right-hand sides in the recorded buffers
    for k, p in enumerate(prs2):
        Ds[k].copy_(dev(p.D))
        Es[k].copy_(dev(p.E))
        Bs[k].copy_(dev(p.B))
    g.launch()
    torch.cuda.synchronize()
    ref2 = eager(btc, prs2, precision)
    for k, p in enumerate(prs2):
        assert np.array_equal(Xs[k].cpu().numpy(), ref2[k]), k
        assert oracle.relres(p.D, p.E, ref2[k], p.B) <= tol
    g.close()
    for h in hs:
        btc.btc_destroy(h)
    r.close()


def test_graph_refuses_growing_a_recorded_workspace(btc):
    p = inputs.block_tridiag(20, 8, seed=1, nrhs=4)
    h = btc.btc_create(p.N, p.n, 0)
    D, E = dev(p.D), dev(p.E)
    B1, X1 = dev(p.B[:, :, :1]), torch.empty((p.N, p.n, 1), dtype=torch.float64, device="cuda:0")
    B4, X4 = dev(p.B), torch.empty_like(dev(p.B))
    r = btc.Runner()
    r.graph_begin()
    r.factor_batched([h], [D], [E])
    r.solve_batched([h], [B1], [X1], 1)
    with pytest.raises(btc.BtcError) as ei:
        r.solve_batched([h], [B4], [X4], 4)
    assert ei.value.code == btc.BTC_ERR_UNSUPPORTED
    g = r.graph_end()
    g.launch()
    torch.cuda.synchronize()
    assert oracle.relres(p.D, p.E, X1.cpu().numpy(), p.B[:, :, :1]) <= 1e-12
    g.close()
    btc.btc_destroy(h)
    r.close()
