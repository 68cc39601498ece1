"""Every device allocation of the library goes through the allocator hook:
with torch's caching allocator installed (the binding's default), the device
memory the library's objects take is exactly what torch's allocator reserves
for them, so no allocation bypasses the hook (a direct hipMalloc would lower
the device's free memory without raising torch's reserved bytes)."""
import numpy as np
import pytest

from paper_2601_03754_amd import inputs

pytestmark = pytest.mark.gpu


def test_library_memory_comes_from_the_hook():
    import torch
    from paper_2601_03754_amd import btc
    btc.lib()

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")

    def run(N, n, prec):
        pr = inputs.block_tridiag(N, n, seed=N + n, nrhs=2)
        D, E, B = dev(pr.D), dev(pr.E), dev(pr.B)
        f = btc.Factor(D, E, precision=prec)
        X = f.solve(B)
        r = btc.Runner()
        h = btc.btc_create(N, n, prec)
        r.factor_batched([h], [D], [E])
        r.solve_batched([h], [B], [torch.empty_like(B)])
        r.sync()
        srv = btc.Server(precision=prec)
        c = srv.add_client(N, n)
        Xs = torch.empty_like(B)
        srv.submit(c, B, Xs, A=(D, E))
        while srv.step() > 0:
            pass
        torch.cuda.synchronize()
        return [f, X, r, h, srv, Xs, D, E, B]

    # module loads and runtime set-up first
    keep = run(64, 16, btc.BTC_FP64)
    for o in keep:
        if hasattr(o, "close"):
            o.close()
    del keep
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    res0 = torch.cuda.memory_reserved()
    keep = run(2048, 64, btc.BTC_FP32_IR) + run(1500, 96, btc.BTC_FP64)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    res1 = torch.cuda.memory_reserved()
    taken, reserved = free0 - free1, res1 - res0
    print("device memory taken %.1f MB, reserved by torch's allocator %.1f MB" % (taken / 1e6, reserved / 1e6))
    assert reserved > 200e6  # the factors and workspaces of the objects above
    # anything the runtime itself maps (descriptor pools, kernel arguments) is small
    assert abs(taken - reserved) < 16e6
    for o in keep:
        if hasattr(o, "close"):
            o.close()
