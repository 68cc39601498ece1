"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/btc.h declares, and its host-only helpers (permutation,
footprint, error strings, argument checks that fail before any device call)
behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_03754_amd", "libbtc.so")


def declared_symbols():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            src = open(os.path.join(ROOT, "include", hdr)).read()
            names += re.findall(r"^BTC_API\s+[\w\s\*]+?\b(btc_\w+)\s*\(", src, re.M)
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2601_03754_amd import build
        build.build()
    from paper_2601_03754_amd import btc
    return btc


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("btc_factor", "btc_solve", "btc_refactor", "btc_status", "btc_destroy",
                 "btc_footprint_bytes", "btc_export_factor", "btc_permutation", "btc_create",
                 "btc_runner_create", "btc_runner_run", "btc_factor_batched", "btc_solve_batched"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    L = lib.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_only_declared_symbols_are_exported(lib):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(btc_\w+)", out))
    assert exported == set(declared_symbols())


@pytest.mark.parametrize("N", [1, 2, 3, 20, 1000, 4097])
def test_permutation_matches_oracle(lib, N):
    assert np.array_equal(lib.btc_permutation(N), oracle.nd_order(N))


def test_footprint(lib):
    fp64 = lib.btc_footprint_bytes(16, 8, lib.BTC_FP64, 0)
    assert fp64 == 3 * 16 * 64 * 8 + 8  # three n x n FP64 blocks per node + info word
    mixed = lib.btc_footprint_bytes(16, 8, lib.BTC_FP32_IR, 0)
    assert mixed == 16 * 64 * (8 + 3 * 4) + 8  # FP64 Schur complements + FP32 factor
    assert lib.btc_footprint_bytes(16, 8, lib.BTC_FP64, 4) > lib.btc_footprint_bytes(16, 8, lib.BTC_FP64, 1) > fp64
    assert lib.btc_footprint_bytes(0, 8, 0, 1) == 0
    assert lib.btc_footprint_bytes(16, 129, 0, 1) == 0
    assert lib.btc_footprint_bytes(16, 8, 7, 1) == 0


def test_argument_errors_before_device_work(lib):
    L = lib.lib()
    h = ctypes.c_void_p()
    # null A_diag -> -1, N < 1 -> -3, n < 1 -> -4, n too large -> unsupported, null out -> -7
    assert L.btc_factor(None, None, 4, 4, None, None, ctypes.byref(h)) == -1
    assert L.btc_factor(8, 8, 0, 4, None, None, ctypes.byref(h)) == -3
    assert L.btc_factor(8, 8, 4, 0, None, None, ctypes.byref(h)) == -4
    assert L.btc_factor(8, 8, 4, 129, None, None, ctypes.byref(h)) == lib.BTC_ERR_UNSUPPORTED
    assert L.btc_factor(8, 8, 4, 4, None, None, None) == -7
    assert L.btc_solve(None, 8, 8, 1, None, None) == -1
    assert L.btc_status(None, None) == -1
    L.btc_destroy(None)
    assert L.btc_create(0, 4, None, ctypes.byref(h)) == -1
    assert L.btc_create(4, 129, None, ctypes.byref(h)) == lib.BTC_ERR_UNSUPPORTED
    assert L.btc_runner_run(None, 0, None) == -1
    assert L.btc_runner_create(None, None) == -2
    assert L.btc_runner_query(None) == -1
    assert L.btc_factor_batched(None, 0, None, None, None) == -1
    assert L.btc_solve_batched(None, 0, None, None, None, 1) == -1
    assert L.btc_refine_info(None, None) == -1
    L.btc_runner_destroy(None)
    assert "argument" in lib.btc_error_string(-3)
    assert "positive definite" in lib.btc_error_string(lib.BTC_ERR_NOT_SPD)
