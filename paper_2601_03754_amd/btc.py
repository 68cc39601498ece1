"""Thin Python binding of libbtc (include/btc.h): ctypes marshalling of torch
device tensors and streams into the C ABI.  Every computation runs in the HIP
library; there is no CPU fallback, and every entry point raises when
libbtc.so is missing.

The functions carry the C names (btc_factor, btc_solve, ...).  ``Factor`` is a
small convenience owner of a handle that also keeps the input tensors alive
for as long as the device may read them.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbtc.so")
_lib = None

BTC_FP64 = 0
BTC_FP32_IR = 1
BTC_BF16_IR = 2
BTC_OK = 0
BTC_ERR_HIP = -100
BTC_ERR_OOM = -101
BTC_ERR_NOT_SPD = -102
BTC_ERR_UNSUPPORTED = -103
BTC_MAX_BLOCK = 128

i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


BTC_REFINE_CLASSIC = 0
BTC_REFINE_GMRES = 1


BTC_STRATEGY_MULTISTAGE = 0
BTC_STRATEGY_KSTAGE = 1
BTC_STRATEGY_AUTO = 2
BTC_STRATEGY_PARTITION = 3


class btc_options(ctypes.Structure):
    _fields_ = [("precision", i32), ("max_refine", i32), ("tol", dbl), ("refine", i32), ("gmres_m", i32),
                ("strategy", i32), ("stages", i32)]


class btc_solve_info(ctypes.Structure):
    _fields_ = [("steps", i32), ("converged", i32), ("relres", dbl), ("inner", i32), ("pad", i32)]


BTC_OP_FACTOR, BTC_OP_FORWARD, BTC_OP_BACKWARD = 0, 1, 2
BTC_OP_RESIDUAL, BTC_OP_REFINE_INIT, BTC_OP_REFINE_TEST = 3, 4, 5


class btc_step(ctypes.Structure):
    _fields_ = [("h", vp), ("op", i32), ("level", i32), ("A_diag", vp), ("A_off", vp), ("B", vp), ("X", vp),
                ("nrhs", i64), ("first", i32), ("level_end", i32), ("stage", i32), ("pad", i32)]


class btc_server_options(ctypes.Structure):
    _fields_ = [("precision", i32), ("max_refine", i32), ("tol", dbl), ("hbm_budget", ctypes.c_size_t),
                ("max_active", i32), ("sweep_ranges", i32), ("lanes", i32)]


class btc_kernel_stat(ctypes.Structure):
    _fields_ = [("op", i32), ("kind", i32), ("np", i32), ("part", i32), ("launches", i64), ("items", i64),
                ("ms", dbl), ("bytes", dbl), ("flops", dbl)]


class btc_server_completion(ctypes.Structure):
    _fields_ = [("ticket", i64), ("client", i64), ("t_submit", dbl), ("t_admit", dbl), ("t_done", dbl),
                ("refactored", i32), ("converged", i32), ("info", i64), ("steps", i32), ("pad", i32),
                ("relres", dbl)]


_ALLOC_FN = ctypes.CFUNCTYPE(vp, ctypes.c_size_t, vp, vp)
_FREE_FN = ctypes.CFUNCTYPE(None, vp, vp, vp)


def _torch_alloc(size, stream, ctx):
    # memory of the current device from torch's caching allocator, bound to
    # the library's stream (stream-ordered reuse); 0 reports out of memory
    try:
        return torch.cuda.caching_allocator_alloc(int(size), torch.cuda.current_device(), int(stream or 0))
    except Exception:
        return 0


def _torch_free(ptr, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_alloc_cb = _ALLOC_FN(_torch_alloc)
_free_cb = _FREE_FN(_torch_free)


class BtcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %d (%s)" % (what, code, btc_error_string(code)))
        self.code = code


def lib():
    """The loaded libbtc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libbtc.so is not built (run: python -m paper_2601_03754_amd.build); "
                               "there is no CPU fallback")
        L = ctypes.CDLL(_LIB_PATH)
        L.btc_factor.restype = ctypes.c_int
        L.btc_factor.argtypes = [vp, vp, i64, i64, ctypes.POINTER(btc_options), vp, ctypes.POINTER(vp)]
        L.btc_refactor.restype = ctypes.c_int
        L.btc_refactor.argtypes = [vp, vp, vp, vp]
        L.btc_solve.restype = ctypes.c_int
        L.btc_solve.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(btc_solve_info)]
        L.btc_status.restype = ctypes.c_int
        L.btc_status.argtypes = [vp, ctypes.POINTER(i64)]
        L.btc_destroy.restype = None
        L.btc_destroy.argtypes = [vp]
        L.btc_footprint_bytes.restype = ctypes.c_size_t
        L.btc_footprint_bytes.argtypes = [i64, i64, i32, i64]
        L.btc_export_factor.restype = ctypes.c_int
        L.btc_export_factor.argtypes = [vp, vp, vp, vp]
        L.btc_permutation.restype = ctypes.c_int
        L.btc_permutation.argtypes = [i64, vp]
        L.btc_error_string.restype = ctypes.c_char_p
        L.btc_error_string.argtypes = [ctypes.c_int]
        L.btc_profile.restype = ctypes.c_int
        L.btc_profile.argtypes = [vp, ctypes.c_int]
        L.btc_profile_read.restype = ctypes.c_int
        L.btc_profile_read.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int]
        L.btc_create.restype = ctypes.c_int
        L.btc_create.argtypes = [i64, i64, ctypes.POINTER(btc_options), ctypes.POINTER(vp)]
        L.btc_runner_create.restype = ctypes.c_int
        L.btc_runner_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.btc_runner_run.restype = ctypes.c_int
        L.btc_runner_run.argtypes = [vp, i32, ctypes.POINTER(btc_step)]
        L.btc_runner_query.restype = ctypes.c_int
        L.btc_runner_query.argtypes = [vp]
        L.btc_runner_sync.restype = ctypes.c_int
        L.btc_runner_sync.argtypes = [vp]
        L.btc_runner_destroy.restype = None
        L.btc_runner_destroy.argtypes = [vp]
        L.btc_factor_batched.restype = ctypes.c_int
        L.btc_factor_batched.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(i64)]
        L.btc_solve_batched.restype = ctypes.c_int
        L.btc_solve_batched.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(i64), ctypes.POINTER(btc_solve_info)]
        L.btc_refine_info.restype = ctypes.c_int
        L.btc_refine_info.argtypes = [vp, ctypes.POINTER(btc_solve_info)]
        L.btc_server_create.restype = ctypes.c_int
        L.btc_server_create.argtypes = [ctypes.POINTER(btc_server_options), vp, ctypes.POINTER(vp)]
        L.btc_server_add_client.restype = ctypes.c_int
        L.btc_server_add_client.argtypes = [vp, i64, i64, ctypes.POINTER(i64)]
        L.btc_server_submit.restype = ctypes.c_int
        L.btc_server_submit.argtypes = [vp, i64, vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.btc_server_step.restype = ctypes.c_int
        L.btc_server_step.argtypes = [vp]
        L.btc_server_poll.restype = ctypes.c_int
        L.btc_server_poll.argtypes = [vp, ctypes.POINTER(btc_server_completion), i32, ctypes.POINTER(i32),
                                      ctypes.c_int]
        L.btc_server_stats.restype = ctypes.c_int
        L.btc_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)]
        L.btc_server_client_handle.restype = vp
        L.btc_server_client_handle.argtypes = [vp, i64]
        L.btc_server_destroy.restype = None
        L.btc_server_destroy.argtypes = [vp]
        L.btc_runner_profile.restype = ctypes.c_int
        L.btc_runner_profile.argtypes = [vp, i32, i32]
        L.btc_runner_profile_read.restype = ctypes.c_int
        L.btc_runner_profile_read.argtypes = [vp, ctypes.POINTER(btc_kernel_stat), i32, ctypes.POINTER(i32)]
        L.btc_level_work.restype = ctypes.c_int
        L.btc_level_work.argtypes = [i32, i32, i64, i64, i64, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.btc_graph_begin.restype = ctypes.c_int
        L.btc_graph_begin.argtypes = [vp]
        L.btc_graph_end.restype = ctypes.c_int
        L.btc_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
        L.btc_graph_launch.restype = ctypes.c_int
        L.btc_graph_launch.argtypes = [vp, vp]
        L.btc_graph_destroy.restype = None
        L.btc_graph_destroy.argtypes = [vp]
        L.btc_tune_get.restype = ctypes.c_int
        L.btc_tune_get.argtypes = [i32, i32, i64, i32, ctypes.POINTER(i32)]
        L.btc_tune_set.restype = ctypes.c_int
        L.btc_tune_set.argtypes = [i32, i32, i64, i32, i32]
        L.btc_autotune.restype = ctypes.c_int
        L.btc_autotune.argtypes = [vp, vp, vp, vp, vp, i64, i32, vp]
        L.btc_server_runner.restype = vp
        L.btc_server_runner.argtypes = [vp]
        L.btc_server_lane_runner.restype = vp
        L.btc_server_lane_runner.argtypes = [vp, i32]
        L.btc_server_host_stats.restype = ctypes.c_int
        L.btc_server_host_stats.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.c_int]
        L.btc_version.restype = ctypes.c_int
        L.btc_version.argtypes = []
        L.btc_autotune_strategy.restype = ctypes.c_int
        L.btc_autotune_strategy.argtypes = [i64, i64, i32, vp, vp, vp, vp, i64, i32, vp, ctypes.POINTER(dbl)]
        L.btc_select_strategy.restype = ctypes.c_int
        L.btc_select_strategy.argtypes = [i64, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.btc_sweep_ranges.restype = ctypes.c_int
        L.btc_sweep_ranges.argtypes = [i64, ctypes.POINTER(i32), i32]
        L.btc_set_allocator.restype = ctypes.c_int
        L.btc_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
        L.btc_runner_host_stats.restype = ctypes.c_int
        L.btc_runner_host_stats.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                            ctypes.c_int]
        L.btc_autotune_batched.restype = ctypes.c_int
        L.btc_autotune_batched.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64), i32]
        L.btc_banded_create.restype = ctypes.c_int
        L.btc_banded_create.argtypes = [ctypes.POINTER(btc_options), i64, i64, i64, vp, vp, ctypes.POINTER(vp)]
        L.btc_banded_refactor.restype = ctypes.c_int
        L.btc_banded_refactor.argtypes = [vp, vp, vp]
        L.btc_banded_solve.restype = ctypes.c_int
        L.btc_banded_solve.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(btc_solve_info)]
        L.btc_banded_status.restype = ctypes.c_int
        L.btc_banded_status.argtypes = [vp, ctypes.POINTER(i64)]
        L.btc_banded_inner.restype = vp
        L.btc_banded_inner.argtypes = [vp]
        L.btc_banded_destroy.restype = None
        L.btc_banded_destroy.argtypes = [vp]
        L.btc_arrow_create.restype = ctypes.c_int
        L.btc_arrow_create.argtypes = [ctypes.POINTER(btc_options), i64, i64, i64, vp, vp, vp, vp, vp,
                                       ctypes.POINTER(vp)]
        L.btc_arrow_refactor.restype = ctypes.c_int
        L.btc_arrow_refactor.argtypes = [vp, vp, vp, vp, vp, vp]
        L.btc_arrow_solve.restype = ctypes.c_int
        L.btc_arrow_solve.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(btc_solve_info)]
        L.btc_arrow_status.restype = ctypes.c_int
        L.btc_arrow_status.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.btc_arrow_export.restype = ctypes.c_int
        L.btc_arrow_export.argtypes = [vp, vp, vp]
        L.btc_arrow_inner.restype = vp
        L.btc_arrow_inner.argtypes = [vp]
        L.btc_arrow_destroy.restype = None
        L.btc_arrow_destroy.argtypes = [vp]
        _lib = L
        # device memory of the library comes from torch's caching allocator
        _check(L.btc_set_allocator(_alloc_cb, _free_cb, None), "btc_set_allocator")
    return _lib


def btc_set_allocator(use_torch: bool = True) -> None:
    """Route the library's device allocations through torch's caching
    allocator (the default once the library is loaded), or back to HIP's own
    allocator (use_torch=False)."""
    L = lib()
    if use_torch:
        _check(L.btc_set_allocator(_alloc_cb, _free_cb, None), "btc_set_allocator")
    else:
        _check(L.btc_set_allocator(ctypes.cast(None, _ALLOC_FN), ctypes.cast(None, _FREE_FN), None),
               "btc_set_allocator")


def btc_error_string(code: int) -> str:
    return lib().btc_error_string(int(code)).decode()


def _check(rc: int, what: str):
    if rc != BTC_OK:
        raise BtcError(rc, what)


def _dev(t: torch.Tensor, name: str, dtype=torch.float64) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def btc_factor(A_diag: torch.Tensor, A_off: torch.Tensor, precision: int = BTC_FP64,
               stream=None, max_refine: int = 0, tol: float = 0.0, refine: int = BTC_REFINE_CLASSIC,
               gmres_m: int = 0, strategy: int = BTC_STRATEGY_MULTISTAGE, stages: int = 0) -> int:
    """Factor; returns the raw handle (int)."""
    N, n, n2 = A_diag.shape
    if n != n2:
        raise ValueError("A_diag must be (N, n, n)")
    pa = _dev(A_diag, "A_diag")
    po = _dev(A_off, "A_off") if N > 1 else 0
    if N > 1 and tuple(A_off.shape) != (N - 1, n, n):
        raise ValueError("A_off must be (N-1, n, n)")
    opt = btc_options(precision, max_refine, tol, refine, gmres_m, strategy, stages)
    h = vp()
    with torch.cuda.device(A_diag.device):
        _check(lib().btc_factor(pa, po, N, n, ctypes.byref(opt), _stream(stream), ctypes.byref(h)),
               "btc_factor")
    return h.value


def btc_refactor(h: int, A_diag: torch.Tensor, A_off: torch.Tensor, stream=None) -> None:
    N = A_diag.shape[0]
    po = _dev(A_off, "A_off") if N > 1 else 0
    with torch.cuda.device(A_diag.device):
        _check(lib().btc_refactor(h, _dev(A_diag, "A_diag"), po, _stream(stream)), "btc_refactor")


def btc_solve(h: int, B: torch.Tensor, X: Optional[torch.Tensor] = None, stream=None,
              want_info: bool = False):
    """Solve into X (allocated like B when None); returns X, or (X, info)."""
    if X is None:
        X = torch.empty_like(B)
    nrhs = B.shape[-1] if B.dim() == 3 else 1
    info = btc_solve_info() if want_info else None
    with torch.cuda.device(B.device):
        rc = lib().btc_solve(h, _dev(B, "B"), _dev(X, "X"), nrhs, _stream(stream),
                             ctypes.byref(info) if info is not None else None)
    _check(rc, "btc_solve")
    if want_info:
        return X, {"steps": info.steps, "converged": bool(info.converged), "relres": info.relres,
                   "inner": info.inner}
    return X


def btc_status(h: int) -> int:
    v = i64(0)
    _check(lib().btc_status(h, ctypes.byref(v)), "btc_status")
    return int(v.value)


def btc_destroy(h: int) -> None:
    if h:
        lib().btc_destroy(h)


def btc_footprint_bytes(N: int, n: int, precision: int = BTC_FP64, nrhs: int = 1) -> int:
    return int(lib().btc_footprint_bytes(N, n, precision, nrhs))


def btc_export_factor(h: int, N: int, n: int):
    """(Ld, Rb, Tb) as host float64 arrays indexed by original block."""
    out = [np.zeros((N, n, n)) for _ in range(3)]
    _check(lib().btc_export_factor(h, *[a.ctypes.data for a in out]), "btc_export_factor")
    return tuple(out)


def btc_permutation(N: int) -> np.ndarray:
    out = np.zeros(N, dtype=np.int64)
    _check(lib().btc_permutation(N, out.ctypes.data), "btc_permutation")
    return out


def btc_profile(h: int, enable: bool) -> None:
    _check(lib().btc_profile(h, 1 if enable else 0), "btc_profile")


def btc_profile_read(h: int, phase: int):
    """(ms per level, launches per level) accumulated since btc_profile(h, True)."""
    ms = np.zeros(64)
    cnt = np.zeros(64, dtype=np.int64)
    L = lib().btc_profile_read(h, phase, ms.ctypes.data, cnt.ctypes.data, 64)
    if L < 0:
        _check(L, "btc_profile_read")
    return ms[:L].copy(), cnt[:L].copy()


def btc_create(N: int, n: int, precision: int = BTC_FP64, max_refine: int = 0, tol: float = 0.0) -> int:
    """Allocate a handle (no factorization) on the current device."""
    h = vp()
    opt = btc_options(precision, max_refine, tol, 0, 0, 0, 0)
    _check(lib().btc_create(N, n, ctypes.byref(opt), ctypes.byref(h)), "btc_create")
    return h.value


def btc_refine_info(h: int) -> dict:
    info = btc_solve_info()
    _check(lib().btc_refine_info(h, ctypes.byref(info)), "btc_refine_info")
    return {"steps": info.steps, "converged": bool(info.converged), "relres": info.relres}


def _ptr_array(vals):
    arr = (vp * max(1, len(vals)))()
    for k, v in enumerate(vals):
        arr[k] = v
    return arr


class Runner:
    """A libbtc step runner bound to one stream (default: torch's current
    stream of the current device)."""

    def __init__(self, stream=None):
        self.stream = _stream(stream)
        r = vp()
        _check(lib().btc_runner_create(self.stream, ctypes.byref(r)), "btc_runner_create")
        self.handle = r.value
        # matrices of the handles factored through this runner: the mixed
        # precision paths read them again for the FP64 residual, so they stay
        # referenced until the handle is factored again or the runner closes
        self._mats = {}

    def run(self, steps) -> None:
        """Enqueue raw steps (the caller keeps every tensor they point to
        alive while the device may read it)."""
        arr = (btc_step * max(1, len(steps)))(*steps)
        _check(lib().btc_runner_run(self.handle, len(steps), arr), "btc_runner_run")

    def query(self) -> bool:
        rc = lib().btc_runner_query(self.handle)
        if rc < 0:
            _check(rc, "btc_runner_query")
        return rc == 1

    def sync(self) -> None:
        _check(lib().btc_runner_sync(self.handle), "btc_runner_sync")

    def factor_batched(self, handles, A_diags, A_offs, want_info: bool = False):
        """Factor the instances together; with want_info, synchronise and
        return each instance's status (0 or the failing block)."""
        n = len(handles)
        info = (i64 * max(1, n))() if want_info else None
        for h, a, o in zip(handles, A_diags, A_offs):
            self._mats[h] = (a, o)
        _check(lib().btc_factor_batched(self.handle, n, _ptr_array(handles),
                                        _ptr_array([_dev(a, "A_diag") for a in A_diags]),
                                        _ptr_array([_dev(a, "A_off") if a.numel() else 0 for a in A_offs]),
                                        info),
               "btc_factor_batched")
        return [int(info[k]) for k in range(n)] if want_info else None

    def solve_batched(self, handles, Bs, Xs, nrhs=None, want_info: bool = False):
        """Solve the instances together; nrhs per instance (default: the
        last dimension of each B).  With want_info, synchronise and return
        each instance's outcome (steps, converged, relres)."""
        n = len(handles)
        if nrhs is None:
            nrhs = [b.shape[-1] if b.dim() == 3 else 1 for b in Bs]
        elif isinstance(nrhs, int):
            nrhs = [nrhs] * n
        m = (i64 * max(1, n))(*[int(v) for v in nrhs])
        info = (btc_solve_info * max(1, n))() if want_info else None
        _check(lib().btc_solve_batched(self.handle, n, _ptr_array(handles),
                                       _ptr_array([_dev(b, "B") for b in Bs]),
                                       _ptr_array([_dev(x, "X") for x in Xs]), m, info),
               "btc_solve_batched")
        if not want_info:
            return None
        return [{"steps": info[k].steps, "converged": bool(info[k].converged), "relres": info[k].relres}
                for k in range(n)]

    def autotune(self, handles, A_diags, A_offs, Bs, Xs, nrhs=None, reps: int = 3) -> None:
        """Tune the variant table on this batch as the batched calls run it
        (btc_autotune_batched); leaves the instances factored and solved."""
        n = len(handles)
        if nrhs is None:
            nrhs = [b.shape[-1] if b.dim() == 3 else 1 for b in Bs]
        elif isinstance(nrhs, int):
            nrhs = [nrhs] * n
        for h, a, o in zip(handles, A_diags, A_offs):
            self._mats[h] = (a, o)
        m = (i64 * max(1, n))(*[int(v) for v in nrhs])
        _check(lib().btc_autotune_batched(self.handle, n, _ptr_array(handles),
                                          _ptr_array([_dev(a, "A_diag") for a in A_diags]),
                                          _ptr_array([_dev(a, "A_off") if a.numel() else 0 for a in A_offs]),
                                          _ptr_array([_dev(b, "B") for b in Bs]),
                                          _ptr_array([_dev(x, "X") for x in Xs]), m, reps),
               "btc_autotune_batched")

    def graph_begin(self) -> None:
        """Record the following runner calls instead of running them."""
        _check(lib().btc_graph_begin(self.handle), "btc_graph_begin")

    def graph_end(self) -> "Graph":
        """Capture the recorded calls into a replayable HIP graph."""
        g = vp()
        _check(lib().btc_graph_end(self.handle, ctypes.byref(g)), "btc_graph_end")
        return Graph(g.value)

    def profile(self, op: int = -1, kind: int = -1) -> None:
        """Switch the launch profiler on for (op, kind) (-1: any; op -2: off)."""
        runner_profile(self.handle, op, kind)

    def profile_read(self):
        return runner_profile_read(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lib().btc_runner_destroy(self.handle)
            self.handle = None
            self._mats.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An instantiated level schedule (btc_graph_*)."""

    def __init__(self, handle: int):
        self.handle = handle

    def launch(self, stream=None) -> None:
        _check(lib().btc_graph_launch(self.handle, _stream(stream)), "btc_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            lib().btc_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def runner_host_stats(r: int, reset: bool = False) -> dict:
    """Host seconds in btc_runner_run (total, and blocked waiting for the
    device) and the number of calls, since creation or the last reset."""
    a, b, c = dbl(), dbl(), i64()
    _check(lib().btc_runner_host_stats(r, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 1 if reset else 0),
           "btc_runner_host_stats")
    return {"run_s": a.value, "wait_s": b.value, "calls": c.value}


def runner_profile(r: int, op: int = -1, kind: int = -1) -> None:
    _check(lib().btc_runner_profile(r, op, kind), "btc_runner_profile")


def runner_profile_read(r: int):
    """Totals per (op, kind, np) since the profiler was switched on, largest
    time first: dicts with launches, items, ms, bytes, flops."""
    buf = (btc_kernel_stat * 256)()
    cnt = i32()
    _check(lib().btc_runner_profile_read(r, buf, 256, ctypes.byref(cnt)), "btc_runner_profile_read")
    return [{"op": b.op, "kind": b.kind, "np": b.np, "part": b.part, "launches": b.launches, "items": b.items,
             "ms": b.ms,
             "bytes": b.bytes, "flops": b.flops} for b in buf[:cnt.value]]


def btc_tune_get(op: int, precision: int, n: int, level: int) -> int:
    v = i32()
    _check(lib().btc_tune_get(op, precision, n, level, ctypes.byref(v)), "btc_tune_get")
    return v.value


def btc_tune_set(op: int, precision: int, n: int, level: int, variant: int) -> None:
    _check(lib().btc_tune_set(op, precision, n, level, variant), "btc_tune_set")


def btc_autotune(h: int, A_diag: torch.Tensor, A_off: torch.Tensor, B: torch.Tensor, X: torch.Tensor,
                 reps: int = 3, stream=None) -> None:
    """Time the kernel variants on this instance and keep the fastest."""
    nrhs = B.shape[-1] if B.dim() == 3 else 1
    po = _dev(A_off, "A_off") if A_off.numel() else 0
    _check(lib().btc_autotune(h, _dev(A_diag, "A_diag"), po, _dev(B, "B"), _dev(X, "X"), nrhs, reps,
                              _stream(stream)), "btc_autotune")


def btc_level_work(op: int, precision: int, N: int, n: int, nrhs: int, level: int):
    """(bytes, flops) of one step as the library counts them (host only)."""
    b, f = dbl(), dbl()
    _check(lib().btc_level_work(op, precision, N, n, nrhs, level, ctypes.byref(b), ctypes.byref(f)),
           "btc_level_work")
    return b.value, f.value


def step(h: int, op: int, level: int = 0, A_diag=None, A_off=None, B=None, X=None, nrhs: int = 0,
         first: bool = False, level_end: int = 0, stage: int = 0) -> btc_step:
    """One step for Runner.run (tensor arguments are device tensors);
    level_end > level + 1 makes a sweep step cover the levels
    level .. level_end-1; stage orders dependent steps of one call."""
    ptr = lambda t: (t.data_ptr() if (t is not None and t.numel()) else 0)
    return btc_step(h, op, level, ptr(A_diag), ptr(A_off), ptr(B), ptr(X), nrhs, 1 if first else 0, level_end,
                    stage, 0)


def btc_sweep_ranges(N: int):
    """Level ranges the library runs a sweep in (bounds, 0 .. levels)."""
    b = (i32 * 70)()
    r = lib().btc_sweep_ranges(N, b, 70)
    if r < 0:
        _check(r, "btc_sweep_ranges")
    return [int(b[k]) for k in range(r + 1)]


class Server:
    """Continuous-batching request server (btc_server_*).  Keeps the tensors of
    every request referenced until the request has completed."""

    def __init__(self, precision: int = BTC_FP64, hbm_budget: int = 1 << 40, max_refine: int = 0,
                 tol: float = 0.0, max_active: int = 0, stream=None, sweep_ranges: bool = False, lanes: int = 0):
        # lanes: 0 the library's choice (three), 1 one tick over all clients, 2..4 lanes by block size
        self.stream = _stream(stream)
        opt = btc_server_options(precision, max_refine, tol, hbm_budget, max_active, 1 if sweep_ranges else 0,
                                 lanes)
        h = vp()
        _check(lib().btc_server_create(ctypes.byref(opt), self.stream, ctypes.byref(h)), "btc_server_create")
        self.handle = h.value
        self._live = {}
        self._mats = {}
        self._buf = (btc_server_completion * 4096)()

    def add_client(self, N: int, n: int) -> int:
        c = i64()
        _check(lib().btc_server_add_client(self.handle, N, n, ctypes.byref(c)), "btc_server_add_client")
        return c.value

    def submit(self, client: int, B: torch.Tensor, X: torch.Tensor, A=None) -> int:
        t = i64()
        nrhs = B.shape[-1] if B.dim() == 3 else 1
        pa = _dev(A[0], "A_diag") if A is not None else 0
        po = (_dev(A[1], "A_off") if A[1].numel() else 0) if A is not None else 0
        _check(lib().btc_server_submit(self.handle, client, pa, po, _dev(B, "B"), _dev(X, "X"), nrhs,
                                       ctypes.byref(t)), "btc_server_submit")
        self._live[t.value] = (client, B, X, A)
        if A is not None:
            self._mats.setdefault(client, []).append((t.value, A))
        return t.value

    def _release(self, ticket: int) -> None:
        # drop the request's tensors; once a refactorization has completed,
        # the client's older matrices are no longer referenced by the server
        # (a later eviction refactors with this one)
        ent = self._live.pop(ticket, None)
        if ent is None:
            return
        client, _, _, A = ent
        if A is not None:
            self._mats[client] = [(t, a) for (t, a) in self._mats.get(client, []) if t >= ticket]

    def step(self) -> int:
        rc = lib().btc_server_step(self.handle)
        if rc < 0:
            _check(rc, "btc_server_step")
        return rc

    def poll(self, wait: bool = False):
        out = []
        while True:
            cnt = i32()
            _check(lib().btc_server_poll(self.handle, self._buf, len(self._buf), ctypes.byref(cnt),
                                         1 if wait else 0), "btc_server_poll")
            for k in range(cnt.value):
                d = self._buf[k]
                out.append({"ticket": d.ticket, "client": d.client, "t_submit": d.t_submit,
                            "t_admit": d.t_admit, "t_done": d.t_done, "refactored": bool(d.refactored),
                            "converged": bool(d.converged), "info": d.info, "steps": d.steps,
                            "relres": d.relres})
                self._release(d.ticket)
            if cnt.value < len(self._buf):
                return out
            wait = False

    def stats(self):
        q, a, b = i64(), i64(), ctypes.c_size_t()
        _check(lib().btc_server_stats(self.handle, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b)),
               "btc_server_stats")
        return {"queued": q.value, "in_flight": a.value, "resident_bytes": b.value}

    def client_handle(self, client: int) -> int:
        return lib().btc_server_client_handle(self.handle, client) or 0

    def runner_handle(self) -> int:
        """The server's step runner (for runner_profile / runner_profile_read)."""
        return lib().btc_server_runner(self.handle) or 0

    def host_stats(self, reset: bool = False) -> dict:
        """Host seconds btc_server_step blocked on the oldest tick, and the
        ticks enqueued over all lanes (since creation or the last reset)."""
        a, t = dbl(), i64()
        _check(lib().btc_server_host_stats(self.handle, ctypes.byref(a), ctypes.byref(t), 1 if reset else 0),
               "btc_server_host_stats")
        return {"wait_s": a.value, "ticks": t.value}

    def runner_handles(self) -> list:
        """The step runners of every lane."""
        out = []
        while True:
            r = lib().btc_server_lane_runner(self.handle, len(out))
            if not r:
                return out
            out.append(r)

    def close(self):
        if getattr(self, "handle", None):
            lib().btc_server_destroy(self.handle)
            self.handle = None
            self._live.clear()
            self._mats.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def btc_autotune_strategy(A_diag: torch.Tensor, A_off: torch.Tensor, B: torch.Tensor, X: torch.Tensor,
                          precision: int = BTC_FP64, reps: int = 5, stream=None):
    """Time the elimination orders on this matrix, keep the fastest for
    BTC_STRATEGY_AUTO; returns ms per refactor+solve of [multi-stage, k=0,
    k=1, k=2, partition p=2, partition p=4] (-1: not a candidate)."""
    N, n, _ = A_diag.shape
    nrhs = B.shape[-1] if B.dim() == 3 else 1
    ms = (dbl * 6)()
    po = _dev(A_off, "A_off") if A_off.numel() else 0
    _check(lib().btc_autotune_strategy(N, n, precision, _dev(A_diag, "A_diag"), po, _dev(B, "B"), _dev(X, "X"),
                                       nrhs, reps, _stream(stream), ms), "btc_autotune_strategy")
    return [ms[k] for k in range(6)]


def btc_select_strategy(N: int, n: int, precision: int = BTC_FP64):
    """(strategy, stages) that BTC_STRATEGY_AUTO takes for (N, n)."""
    s, k = i32(), i32()
    _check(lib().btc_select_strategy(N, n, precision, ctypes.byref(s), ctypes.byref(k)), "btc_select_strategy")
    return s.value, k.value


def btc_version() -> int:
    return int(lib().btc_version())


class Factor:
    """Owner of a libbtc handle.  Keeps the input tensors referenced while the
    device may still read them."""

    def __init__(self, A_diag: torch.Tensor, A_off: torch.Tensor, precision: int = BTC_FP64,
                 stream=None, max_refine: int = 0, tol: float = 0.0, refine: int = BTC_REFINE_CLASSIC,
                 gmres_m: int = 0, strategy: int = BTC_STRATEGY_MULTISTAGE, stages: int = 0):
        if A_off is None or A_off.numel() == 0:
            A_off = torch.zeros((0, A_diag.shape[1], A_diag.shape[1]), dtype=A_diag.dtype,
                                device=A_diag.device)
        self.N, self.n = int(A_diag.shape[0]), int(A_diag.shape[1])
        self.precision = precision
        self._A = (A_diag, A_off)
        self.handle = btc_factor(A_diag, A_off, precision, stream, max_refine, tol, refine, gmres_m, strategy,
                                 stages)

    def refactor(self, A_diag: torch.Tensor, A_off: torch.Tensor, stream=None) -> "Factor":
        btc_refactor(self.handle, A_diag, A_off, stream)
        self._A = (A_diag, A_off)
        return self

    def solve(self, B: torch.Tensor, X: Optional[torch.Tensor] = None, stream=None,
              want_info: bool = False):
        return btc_solve(self.handle, B, X, stream, want_info)

    @property
    def info(self) -> int:
        return btc_status(self.handle)

    def export(self):
        return btc_export_factor(self.handle, self.N, self.n)

    def close(self):
        if getattr(self, "handle", None):
            btc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor(A_diag: torch.Tensor, A_off: torch.Tensor, precision: int = BTC_FP64, stream=None,
           max_refine: int = 0, tol: float = 0.0, refine: int = BTC_REFINE_CLASSIC, gmres_m: int = 0) -> Factor:
    return Factor(A_diag, A_off, precision, stream, max_refine, tol, refine, gmres_m)


# ---------------------------------------------------------------------------
# Block-banded and arrow extensions

def _options(precision, max_refine, tol, refine=BTC_REFINE_CLASSIC, gmres_m=0, strategy=BTC_STRATEGY_MULTISTAGE,
             stages=0):
    return btc_options(precision, max_refine, tol, refine, gmres_m, strategy, stages)


def _info_dict(inf: btc_solve_info) -> dict:
    return {"steps": inf.steps, "converged": bool(inf.converged), "relres": inf.relres, "inner": inf.inner}


class Banded:
    """Owner of a btc_banded object: a block-banded SPD matrix A_band of shape
    (N, b+1, n, n) (A_band[i, k] = block (i, i-k)), factored as ceil(N/b)
    super-blocks of order b*n."""

    def __init__(self, A_band: torch.Tensor, precision: int = BTC_FP64, stream=None, max_refine: int = 0,
                 tol: float = 0.0):
        N, b1, n, n2 = A_band.shape
        if n != n2 or b1 < 2:
            raise ValueError("A_band must have shape (N, b+1, n, n) with b >= 1")
        self.N, self.n, self.b = int(N), int(n), int(b1) - 1
        opt = _options(precision, max_refine, tol)
        h = vp()
        _check(lib().btc_banded_create(ctypes.byref(opt), self.N, self.n, self.b, _dev(A_band, "A_band"),
                                       _stream(stream), ctypes.byref(h)), "btc_banded_create")
        self.handle = h.value

    def refactor(self, A_band: torch.Tensor, stream=None) -> "Banded":
        _check(lib().btc_banded_refactor(self.handle, _dev(A_band, "A_band"), _stream(stream)),
               "btc_banded_refactor")
        return self

    def solve(self, B: torch.Tensor, X: Optional[torch.Tensor] = None, stream=None, want_info: bool = False):
        if X is None:
            X = torch.empty_like(B)
        nrhs = B.numel() // (self.N * self.n)
        inf = btc_solve_info()
        _check(lib().btc_banded_solve(self.handle, _dev(B, "B"), _dev(X, "X"), nrhs, _stream(stream),
                                      ctypes.byref(inf) if want_info else None), "btc_banded_solve")
        return (X, _info_dict(inf)) if want_info else X

    @property
    def info(self) -> int:
        v = i64()
        _check(lib().btc_banded_status(self.handle, ctypes.byref(v)), "btc_banded_status")
        return v.value

    def export(self):
        """(Ld, Rb, Tb) of the super-block factor (btc_export_factor)."""
        N2 = -(-self.N // self.b)
        return btc_export_factor(lib().btc_banded_inner(self.handle), N2, self.b * self.n)

    def close(self):
        if getattr(self, "handle", None):
            lib().btc_banded_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Arrow:
    """Owner of a btc_arrow object: [[Psi, F], [F^T, C]] with Psi the block
    tridiagonal (A_diag, A_off), F of shape (N*n, m), C of shape (m, m).
    Keeps A_diag / A_off referenced (the mixed modes read them in solves)."""

    def __init__(self, A_diag: torch.Tensor, A_off: torch.Tensor, F: torch.Tensor, C: torch.Tensor,
                 precision: int = BTC_FP64, stream=None, max_refine: int = 0, tol: float = 0.0):
        self.N, self.n = int(A_diag.shape[0]), int(A_diag.shape[1])
        self.m = int(F.shape[1]) if F.dim() == 2 else 0
        if A_off is None or A_off.numel() == 0:
            A_off = torch.zeros((0, self.n, self.n), dtype=A_diag.dtype, device=A_diag.device)
        opt = _options(precision, max_refine, tol)
        h = vp()
        self._A = (A_diag, A_off)
        _check(lib().btc_arrow_create(ctypes.byref(opt), self.N, self.n, self.m, _dev(A_diag, "A_diag"),
                                      _dev(A_off, "A_off") if A_off.numel() else None,
                                      _dev(F, "F") if self.m else None, _dev(C, "C") if self.m else None,
                                      _stream(stream), ctypes.byref(h)), "btc_arrow_create")
        self.handle = h.value

    def refactor(self, A_diag, A_off, F, C, stream=None) -> "Arrow":
        if A_off is None or A_off.numel() == 0:
            A_off = torch.zeros((0, self.n, self.n), dtype=A_diag.dtype, device=A_diag.device)
        _check(lib().btc_arrow_refactor(self.handle, _dev(A_diag, "A_diag"),
                                        _dev(A_off, "A_off") if A_off.numel() else None,
                                        _dev(F, "F") if self.m else None, _dev(C, "C") if self.m else None,
                                        _stream(stream)), "btc_arrow_refactor")
        self._A = (A_diag, A_off)
        return self

    def solve(self, B: torch.Tensor, X: Optional[torch.Tensor] = None, stream=None, want_info: bool = False):
        if X is None:
            X = torch.empty_like(B)
        nrhs = B.numel() // (self.N * self.n + self.m)
        inf = btc_solve_info()
        _check(lib().btc_arrow_solve(self.handle, _dev(B, "B"), _dev(X, "X"), nrhs, _stream(stream),
                                     ctypes.byref(inf) if want_info else None), "btc_arrow_solve")
        return (X, _info_dict(inf)) if want_info else X

    @property
    def info(self):
        """(info of Psi, info of the tip)."""
        a, t = i64(), i64()
        _check(lib().btc_arrow_status(self.handle, ctypes.byref(a), ctypes.byref(t)), "btc_arrow_status")
        return a.value, t.value

    def export(self):
        """(L_S, Z) on the host: the tip's Cholesky factor (m x m) and Psi^{-1} F."""
        Ls = np.zeros((self.m, self.m))
        Z = np.zeros((self.N * self.n, self.m))
        _check(lib().btc_arrow_export(self.handle, Ls.ctypes.data if self.m else None,
                                      Z.ctypes.data if self.m else None), "btc_arrow_export")
        return Ls, Z

    def close(self):
        if getattr(self, "handle", None):
            lib().btc_arrow_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
