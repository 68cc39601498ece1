"""No result may depend on what the library's device memory held before:
every allocation the library makes is filled with NaN by the allocator hook
(btc_set_allocator), and every path (one instance per precision and kernel
family, many instances per launch, the server) must give the same results,
bit for bit, as with memory from torch's caching allocator, and meet the
oracle's tolerance."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu


class PoisonAllocator:
    """Device memory as NaN-filled torch tensors kept alive until freed (the
    tests run on the default stream and synchronise before tensors go)."""

    def __init__(self, btc):
        self.btc = btc
        self.live = {}
        self._a = btc._ALLOC_FN(self._alloc)
        self._f = btc._FREE_FN(self._free)

    def _alloc(self, size, stream, ctx):
        try:
            t = torch.full(((int(size) + 7) // 8 + 32,), float("nan"), dtype=torch.float64, device="cuda:0")
            torch.cuda.synchronize()
            p = (t.data_ptr() + 255) & ~255
            self.live[p] = t
            return p
        except Exception:
            return 0

    def _free(self, ptr, stream, ctx):
        torch.cuda.synchronize()
        self.live.pop(int(ptr), None)

    def __enter__(self):
        assert self.btc.lib().btc_set_allocator(self._a, self._f, None) == 0
        return self

    def __exit__(self, *exc):
        torch.cuda.synchronize()
        self.btc.btc_set_allocator(True)


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    b.lib()
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def one(btc, pr, precision):
    f = btc.Factor(dev(pr.D), dev(pr.E), precision=precision)
    X = f.solve(dev(pr.B))
    torch.cuda.synchronize()
    out = (X.cpu().numpy(), f.export(), f.info)
    f.close()
    return out


SHAPES = [(1, 5), (3, 8), (20, 12), (33, 16), (45, 30), (17, 40), (12, 64), (9, 90), (6, 128), (100, 24)]


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_single_instance_poisoned_memory(btc, precision):
    prs = [inputs.block_tridiag(N, n, seed=600 + N + n, nrhs=2) for N, n in SHAPES]
    ref = [one(btc, p, precision) for p in prs]
    with PoisonAllocator(btc):
        got = [one(btc, p, precision) for p in prs]
    tol = 1e-12 if precision == 0 else 1e-10
    for p, (Xr, br, ir), (Xg, bg, ig) in zip(prs, ref, got):
        assert ig == ir == 0, (p.N, p.n)
        assert np.array_equal(Xg, Xr), (p.N, p.n)
        for a, b in zip(bg, br):
            assert np.array_equal(a, b), (p.N, p.n)
        assert oracle.relres(p.D, p.E, Xg, p.B) <= tol


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batched_poisoned_memory(btc, precision):
    rng = np.random.default_rng(40 + precision)
    prs = [inputs.block_tridiag(int(rng.integers(2, 150)), int(rng.choice([8, 30, 64, 90, 128])), seed=k, nrhs=1)
           for k in range(10)]

    def run():
        r = btc.Runner()
        hs = [btc.btc_create(p.N, p.n, precision) for p in prs]
        Bs = [dev(p.B) for p in prs]
        Xs = [torch.full_like(b, float("nan")) for b in Bs]
        fi = r.factor_batched(hs, [dev(p.D) for p in prs], [dev(p.E) for p in prs], want_info=True)
        si = r.solve_batched(hs, Bs, Xs, want_info=True)
        out = [X.cpu().numpy() for X in Xs]
        for h in hs:
            btc.btc_destroy(h)
        r.close()
        return fi, si, out

    fr, sr, Xr = run()
    with PoisonAllocator(btc):
        fg, sg, Xg = run()
    tol = 1e-12 if precision == 0 else 1e-10
    assert fr == fg == [0] * len(prs)
    for k, p in enumerate(prs):
        assert sg[k]["converged"], (k, sg[k])
        assert np.array_equal(Xg[k], Xr[k]), (k, p.N, p.n)
        assert oracle.relres(p.D, p.E, Xg[k], p.B) <= tol
