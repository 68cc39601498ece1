"""btc_solve_noalloc through the C ABI: the same results as btc_solve, bit for
bit, on two calls in a row (the second with a smaller system, so the shared
scratch array holds the first call's contents), with no device allocation by
the library during the calls, and a refusal of workspaces beyond the limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def btc():
    from paper_2601_03754_amd import btc as b
    L = b.lib()
    L.btc_solve_noalloc.restype = ctypes.c_int
    L.btc_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.POINTER(b.btc_solve_info)]
    return b


class CountingAllocator:
    """torch's caching allocator behind the library's hook, counting calls."""

    def __init__(self, btc):
        self.btc = btc
        self.allocs = 0
        self.frees = 0
        self._a = btc._ALLOC_FN(self._alloc)
        self._f = btc._FREE_FN(self._free)

    def _alloc(self, size, stream, ctx):
        self.allocs += 1
        return self.btc._torch_alloc(size, stream, ctx)

    def _free(self, ptr, stream, ctx):
        self.frees += 1
        self.btc._torch_free(ptr, stream, ctx)

    def __enter__(self):
        assert self.btc.lib().btc_set_allocator(self._a, self._f, None) == 0
        return self

    def __exit__(self, *exc):
        self.btc.btc_set_allocator(True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def noalloc(btc, h, B, X, want_info=False):
    info = btc.btc_solve_info()
    nrhs = B.shape[-1]
    rc = btc.lib().btc_solve_noalloc(h, B.data_ptr(), X.data_ptr(), nrhs,
                                     torch.cuda.current_stream().cuda_stream,
                                     ctypes.byref(info) if want_info else None)
    return rc, info


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_noalloc_equals_solve_twice(btc, precision):
    shapes = [(300, 40, 3), (37, 24, 1)]  # the second call is smaller
    with CountingAllocator(btc) as ca:
        for k, (N, n, m) in enumerate(shapes):
            pr = inputs.block_tridiag(N, n, seed=70 + 10 * precision + k, nrhs=m)
            D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
            f = btc.Factor(D, E, precision=precision)
            Xref, iref = f.solve(B, want_info=True)
            Xn = torch.full_like(B, np.nan)
            torch.cuda.synchronize()
            before = (ca.allocs, ca.frees)
            rc, info = noalloc(btc, f.handle, B, Xn, want_info=True)
            torch.cuda.synchronize()
            assert rc == 0
            assert (ca.allocs, ca.frees) == before  # nothing allocated or freed
            assert np.array_equal(Xn.cpu().numpy(), Xref.cpu().numpy()), (N, n, m)
            assert info.steps == iref["steps"] and bool(info.converged) == iref["converged"]
            tol = 1e-12 if precision == 0 else 1e-10
            assert oracle.relres(pr.D, pr.E, Xn.cpu().numpy(), pr.B) <= tol
            f.close()


def test_noalloc_without_info_and_limits(btc):
    pr = inputs.block_tridiag(64, 16, seed=5, nrhs=2)
    D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
    f = btc.Factor(D, E, precision=btc.BTC_FP32_IR)
    Xref = f.solve(B)
    Xn = torch.empty_like(B)
    rc, _ = noalloc(btc, f.handle, B, Xn)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(Xn.cpu().numpy(), Xref.cpu().numpy())
    # aliasing and argument errors as btc_solve
    rc, _ = noalloc(btc, f.handle, B, B)
    assert rc == -3
    f.close()
    # a workspace beyond the fixed array is refused before any device work
    N, n = 4096, 128
    big = btc.btc_create(N, n, btc.BTC_FP64)
    try:
        # a handle never factored is an argument error; factor a cheap stand-in
        # of the same shape (identity blocks) to reach the size check
        Di = torch.eye(n, dtype=torch.float64, device="cuda:0").expand(N, n, n).contiguous()
        Ei = torch.zeros((N - 1, n, n), dtype=torch.float64, device="cuda:0")
        btc.btc_refactor(big, Di, Ei)
        Bb = torch.ones((N, n, 4), dtype=torch.float64, device="cuda:0")  # 84 MB of workspace
        Xb = torch.empty_like(Bb)
        rc, _ = noalloc(btc, big, Bb, Xb)
        assert rc == btc.BTC_ERR_UNSUPPORTED
    finally:
        torch.cuda.synchronize()
        btc.btc_destroy(big)
