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
                 "btc_runner_create", "btc_runner_run", "btc_factor_batched", "btc_solve_batched",
                 "btc_set_allocator"):
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
    assert L.btc_factor_batched(None, 0, None, None, None, None) == -1
    assert L.btc_solve_batched(None, 0, None, None, None, None, None) == -1
    assert L.btc_refine_info(None, None) == -1
    L.btc_runner_destroy(None)
    # host-time counters and lanes: null handles are refused before any device work
    assert L.btc_runner_host_stats(None, None, None, None, 0) == -1
    assert L.btc_server_host_stats(None, None, None, 0) == -1
    assert not L.btc_server_lane_runner(None, 0)
    opt = lib.btc_server_options(0, 0, 0.0, 1 << 30, 0, 0, -1)  # negative lane count
    assert L.btc_server_create(ctypes.byref(opt), None, ctypes.byref(h)) == -1
    assert "argument" in lib.btc_error_string(-3)
    assert "positive definite" in lib.btc_error_string(lib.BTC_ERR_NOT_SPD)


# Off-diagonal factor blocks and fill blocks of the nested-dissection factor
# (counted independently from the dense structure of the permuted factor).
STRUCTURE = {16: (26, 11), 20: (33, 14), 64: (120, None), 256: (502, None), 1024: (2036, None),
             4096: (8178, 4083), 16384: (32752, None)}


@pytest.mark.parametrize("N", sorted(STRUCTURE))
def test_level_work_flops_match_operation_counts(lib, N):
    """Summed over the levels, the library's flop accounting equals the
    operation counts of section "Computational Complexity": factor
    n^3 (N/3 + 2 M_off + 2 F), both sweeps n^2 m (2N + 4 M_off)."""
    n, m = 24, 3
    L = int(np.floor(np.log2(N))) + 1
    fac = sum(lib.btc_level_work(lib.BTC_OP_FACTOR, 0, N, n, 0, l)[1] for l in range(L))
    fwd = sum(lib.btc_level_work(lib.BTC_OP_FORWARD, 0, N, n, m, l)[1] for l in range(L))
    bwd = sum(lib.btc_level_work(lib.BTC_OP_BACKWARD, 0, N, n, m, l)[1] for l in range(L))
    M_off, F = STRUCTURE[N]
    if F is None:  # every fill couples the two neighbours of a node that has both
        F = M_off - (N - 1)
    assert fac == pytest.approx(n ** 3 * (N / 3 + 2 * M_off + 2 * F), rel=1e-12)
    assert fwd + bwd == pytest.approx(n * n * m * (2 * N + 4 * M_off), rel=1e-12)


def test_level_work_bytes(lib):
    """Byte accounting: the residual reads every stored block of the matrix
    once; mixed precision halves the factor-block words; level-0 factor of
    N = 3: nodes 1 and 3, node 1 has a right neighbour, node 3 a left one."""
    n, N, m = 8, 37, 2
    b, f = lib.btc_level_work(lib.BTC_OP_RESIDUAL, 0, N, n, m, 0)
    assert b == 8 * n * n * (2 * N - 1) + 24 * N * n * m
    assert f == 2 * n * n * m * (3 * N - 2)
    b64, _ = lib.btc_level_work(lib.BTC_OP_FACTOR, 0, 3, n, 0, 0)
    # reads S_1, S_3, S_2 (node 1's right separator), C_21, C_32; writes L_11,
    # L_33, R_1, T_3, S_2
    assert b64 == 8 * n * n * (5 + 5)
    b32, _ = lib.btc_level_work(lib.BTC_OP_FACTOR, 1, 3, n, 0, 0)
    # FP64: S reads (3), coupling reads from the input (2), S_2 write; FP32: L, L, R, T
    assert b32 == n * n * (8 * (3 + 2 + 1) + 4 * 4)


def test_level_work_argument_errors(lib):
    L = lib.lib()
    import ctypes
    b, f = ctypes.c_double(), ctypes.c_double()
    assert L.btc_level_work(9, 0, 8, 4, 1, 0, ctypes.byref(b), ctypes.byref(f)) == -1
    assert L.btc_level_work(0, 7, 8, 4, 1, 0, ctypes.byref(b), ctypes.byref(f)) == -2
    assert L.btc_level_work(0, 0, 0, 4, 1, 0, ctypes.byref(b), ctypes.byref(f)) == -3
    assert L.btc_level_work(1, 0, 8, 4, 0, 0, ctypes.byref(b), ctypes.byref(f)) == -5
    assert L.btc_level_work(1, 0, 8, 4, 1, 4, ctypes.byref(b), ctypes.byref(f)) == -6
    assert L.btc_runner_profile(None, -1, -1) == -1


def test_graph_argument_errors(lib):
    L = lib.lib()
    assert L.btc_graph_begin(None) == -1
    assert L.btc_graph_end(None, None) == -1
    assert L.btc_graph_launch(None, None) == -1
    L.btc_graph_destroy(None)


def test_tune_table_host_only(lib):
    """The variant table is host state: defaults, set/get round trip, keys
    without a choice accept only variant 0, argument errors."""
    F, FW, R = lib.BTC_OP_FACTOR, lib.BTC_OP_FORWARD, lib.BTC_OP_RESIDUAL
    assert lib.btc_tune_get(F, 0, 24, 0) == 0
    assert lib.btc_tune_get(F, 1, 50, 0) == 1  # tile-parallel step by default at padded 64
    assert lib.btc_tune_get(F, 0, 64, 4) == 1
    lib.btc_tune_set(F, 0, 24, 3, 1)           # n 24 -> padded 32, levels >= 1
    assert lib.btc_tune_get(F, 0, 20, 5) == 1  # same padded size and bucket
    assert lib.btc_tune_get(F, 0, 24, 0) == 0  # level 0 bucket untouched
    lib.btc_tune_set(F, 0, 24, 3, 0)
    assert lib.btc_tune_get(F, 0, 24, 3) == 0
    lib.btc_tune_set(FW, 1, 64, 0, 1)
    assert lib.btc_tune_get(FW, 1, 50, 7) == 1
    lib.btc_tune_set(FW, 1, 64, 0, 0)
    lib.btc_tune_set(F, 1, 12, 0, 0)           # mixed factor at padded 16: single variant
    with pytest.raises(lib.BtcError) as ei:
        lib.btc_tune_set(F, 1, 12, 0, 1)
    assert ei.value.code == lib.BTC_ERR_UNSUPPORTED
    # padded 32: mixed, 0 or 1 (the tile-parallel step); FP64, 0, 1 or 2
    lib.btc_tune_set(F, 1, 24, 0, 1)
    assert lib.btc_tune_get(F, 1, 30, 0) == 1
    lib.btc_tune_set(F, 1, 24, 0, 0)
    lib.btc_tune_set(F, 0, 24, 0, 2)
    assert lib.btc_tune_get(F, 0, 24, 0) == 2
    lib.btc_tune_set(F, 0, 24, 0, 0)
    L = lib.lib()
    assert L.btc_tune_set(F, 0, 24, 0, 3) == -5
    assert L.btc_tune_set(F, 1, 24, 0, 2) == -5
    v = ctypes.c_int32()
    assert L.btc_tune_get(9, 0, 8, 0, ctypes.byref(v)) == -1
    assert L.btc_tune_get(0, 5, 8, 0, ctypes.byref(v)) == -2
    assert L.btc_tune_get(0, 0, 200, 0, ctypes.byref(v)) == -3
    assert L.btc_tune_get(0, 0, 8, -1, ctypes.byref(v)) == -4
    assert L.btc_tune_set(R, 0, 8, 0, 2) == -5
    assert L.btc_autotune(None, None, None, None, None, 1, 1, None) == -1


def test_allocator_hook_arguments(lib):
    """btc_set_allocator takes both functions or neither; loading the
    binding installs torch's caching allocator, and it can be switched back
    to HIP's own and on again (host state only, no device call)."""
    L = lib.lib()
    assert L.btc_set_allocator(lib._alloc_cb, ctypes.cast(None, lib._FREE_FN), None) == -1
    assert L.btc_set_allocator(ctypes.cast(None, lib._ALLOC_FN), lib._free_cb, None) == -1
    lib.btc_set_allocator(False)
    lib.btc_set_allocator(True)


def test_bf16_footprint_matches_mixed(lib):
    for n in (8, 40, 100):
        assert lib.btc_footprint_bytes(33, n, lib.BTC_BF16_IR, 2) == lib.btc_footprint_bytes(33, n, lib.BTC_FP32_IR, 2)
    assert lib.btc_footprint_bytes(33, 8, 3, 2) == 0


@pytest.mark.parametrize("N", [1, 2, 3, 16, 64, 100, 1000, 4096, 16384, 70000])
def test_sweep_ranges(lib, N):
    """Sweep level ranges: contiguous from level 0 to floor(log2 N)+1; levels
    with many nodes alone; in a multi-level range every level of a subtree
    has at most as many nodes as the workgroup has wavefronts (4), so the
    range takes one round of node steps per level."""
    b = lib.btc_sweep_ranges(N)
    L = int(np.floor(np.log2(N))) + 1
    assert b[0] == 0 and b[-1] == L and all(x < y for x, y in zip(b, b[1:]))
    nodes = lambda l: (N + (1 << l)) // (2 << l)
    for l0, l1 in zip(b, b[1:]):
        if nodes(l0) >= 4096:
            assert l1 == l0 + 1
        if l1 > l0 + 1:
            assert all(min(1 << (l1 - l - 1), nodes(l)) <= 4 for l in range(l0, l1))


def test_tune_cache_persists_across_processes(lib, tmp_path):
    """BTC_TUNE_CACHE: a variant set in one process is read back by the next
    (host state only); the sweep launch shape is a tune key with three
    variants."""
    import subprocess
    import sys
    cache = str(tmp_path / "tune.txt")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2601_03754_amd import btc\n"
            "S = btc.lib() and 6\n"
            "if sys.argv[1] == 'set':\n"
            "    btc.btc_tune_set(S, 1, 90, 0, 2)\n"
            "    btc.btc_tune_set(0, 0, 24, 3, 1)\n"
            "else:\n"
            "    print(btc.btc_tune_get(S, 1, 96, 0), btc.btc_tune_get(0, 0, 20, 1), btc.btc_tune_get(S, 0, 96, 0))\n"
            % ROOT)
    env = dict(os.environ, BTC_TUNE_CACHE=cache)
    subprocess.run([sys.executable, "-c", code, "set"], env=env, check=True)
    assert os.path.exists(cache)
    out = subprocess.run([sys.executable, "-c", code, "get"], env=env, check=True, capture_output=True,
                         text=True).stdout.split()
    assert out == ["2", "1", "0"]
    with pytest.raises(lib.BtcError):
        lib.btc_tune_set(6, 0, 40, 0, 3)


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU: any other count exits with a message before
    touching a device."""
    import subprocess, sys, os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_sums_lane_profiles_and_host_counters():
    """The served bench merges the launch profiles and host-time counters of
    the server's lane runners: equal keys add up, the order is by time."""
    import os, sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench

    class FakeBtc:
        prof = {1: [{"op": 0, "kind": 3, "np": 96, "part": 2, "launches": 2, "items": 10, "ms": 1.0, "bytes": 5.0,
                     "flops": 7.0}],
                2: [{"op": 0, "kind": 3, "np": 96, "part": 2, "launches": 1, "items": 4, "ms": 3.0, "bytes": 1.0,
                     "flops": 1.0},
                    {"op": 1, "kind": 1, "np": 32, "part": 0, "launches": 5, "items": 9, "ms": 2.0, "bytes": 2.0,
                     "flops": 3.0}]}
        host = {1: {"run_s": 1.0, "wait_s": 0.5, "calls": 3}, 2: {"run_s": 2.0, "wait_s": 0.25, "calls": 4}}

        def runner_profile_read(self, r):
            return self.prof[r]

        def runner_host_stats(self, r, reset=False):
            return self.host[r]

    f = FakeBtc()
    merged = bench.prof_read(f, [1, 2])
    assert [(m["op"], m["np"]) for m in merged] == [(0, 96), (1, 32)]
    assert merged[0]["launches"] == 3 and merged[0]["ms"] == 4.0 and merged[0]["bytes"] == 6.0
    assert merged[0]["items"] == 14 and merged[0]["flops"] == 8.0
    assert bench.host_stats(f, [1, 2]) == {"run_s": 3.0, "wait_s": 0.75, "calls": 7}


def test_auto_strategy_before_any_measurement(lib):
    """Without a measured choice, BTC_STRATEGY_AUTO takes the multi-stage
    order (measured the fastest also at the smallest shapes)."""
    for N, n, prec in ((7, 5, 0), (16, 8, 0), (31, 16, 0), (5000, 64, 1)):
        assert lib.btc_select_strategy(N, n, prec) == (lib.BTC_STRATEGY_MULTISTAGE, 0)
