// Kernel variants chosen by the autotuner: a process-wide table keyed by
// (operation, kernel family, padded block size, level bucket), and the tuner
// that times the candidates on a caller's instance.
//
// Tunable choices:
//   factor, FP64, padded size 16 or 32: 0 = matrix-core kernel, 1 = vector-ALU
//     kernel; padded size 64, every precision: 0 = one workgroup per node,
//     1 = the tile-parallel step (different rounding orders; level bucket 0 =
//     level 0, which has no deferred updates, 1 = the other levels)
//   forward / backward sweep and residual, nrhs > 1: 0 = four right-hand-side
//     columns per dependency chain group, 1 = one (bitwise identical results)
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "btc.h"
#include "btc_handle.h"
#include "btc_kernels.h"

namespace btc_host {
namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;
// measured elimination orders: (precision, N, padded n) -> (strategy, stages)
std::map<std::tuple<int, int64_t, int>, std::pair<int32_t, int32_t>> g_strategy;
bool g_loaded = false;

// The table file named by BTC_TUNE_CACHE: lines "v op kind np bucket
// variant" and "s precision N np strategy stages".  Called with the lock
// held.
void load_cache_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char* path = getenv("BTC_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char tag[4];
    while (fscanf(f, "%3s", tag) == 1) {
        if (tag[0] == 'v') {
            int op, kind, np, bucket, variant;
            if (fscanf(f, "%d %d %d %d %d", &op, &kind, &np, &bucket, &variant) != 5) break;
            g_tune[std::make_tuple(op, kind, np, bucket)] = variant;
        } else if (tag[0] == 's') {
            int prec, np, strategy, stages;
            long long N;
            if (fscanf(f, "%d %lld %d %d %d", &prec, &N, &np, &strategy, &stages) != 5) break;
            g_strategy[std::make_tuple(prec, (int64_t)N, np)] = {strategy, stages};
        } else {
            break;
        }
    }
    fclose(f);
}

}  // namespace

// Write the table to the BTC_TUNE_CACHE file (if set).
void save_tune_cache() {
    const char* path = getenv("BTC_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto& kv : g_tune)
        fprintf(f, "v %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                std::get<3>(kv.first), kv.second);
    for (auto& kv : g_strategy)
        fprintf(f, "s %d %lld %d %d %d\n", std::get<0>(kv.first), (long long)std::get<1>(kv.first),
                std::get<2>(kv.first), kv.second.first, kv.second.second);
    fclose(f);
    (void)rename(tmp.c_str(), path);
}

// Variant of a key nobody has set: measured on MI355X, the tile-parallel
// step beats the one-workgroup-per-node kernel at padded size 64 (it needs
// less LDS per workgroup, so several nodes share a compute unit); 0 elsewhere.
int default_variant(int op, int np) { return (op == BTC_OP_FACTOR && np == 64) ? 1 : 0; }

int tune_variant(int op, int kind, int np, int bucket) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tune.find(std::make_tuple(op, kind, np, bucket));
    return it == g_tune.end() ? default_variant(op, np) : it->second;
}

void tune_set(int op, int kind, int np, int bucket, int variant) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    g_tune[std::make_tuple(op, kind, np, bucket)] = variant;
}

void select_strategy(int64_t N, int64_t n, int32_t prec, int32_t* strategy, int32_t* stages) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        auto it = g_strategy.find(std::make_tuple((int)prec, N, btc::padded_block((int)n)));
        if (it != g_strategy.end()) {
            *strategy = it->second.first;
            *stages = it->second.second;
            return;
        }
    }
    // before any measurement: the multi-stage order (measured on MI355X
    // the fastest also for the smallest shapes, N = 16, n = 8: levels spread
    // over compute units beat a chain walked by one wavefront)
    (void)N;
    (void)n;
    (void)prec;
    *strategy = BTC_STRATEGY_MULTISTAGE;
    *stages = 0;
}

void strategy_set(int64_t N, int64_t n, int32_t prec, int32_t strategy, int32_t stages) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    g_strategy[std::make_tuple((int)prec, N, btc::padded_block((int)n))] = {strategy, stages};
}

}  // namespace btc_host

using namespace btc_host;

namespace {

// (kind, padded size) of a tunable family for a handle, or false.
bool tunable(int op, int32_t prec, int64_t n, int& kind, int& np, int& variants) {
    const bool mixed = is_mixed(prec);
    np = btc::padded_block((int)n);
    if (op == BTC_OP_FACTOR) {
        kind = mixed ? (prec == BTC_BF16_IR ? 2 : 1) : 0;
        // FP64 np 32: MFMA, VALU, tile-parallel; else two families
        variants = (!mixed && np == 32) ? 3 : 2;
        return np == 64 || np == 32 || (!mixed && np == 16);
    }
    if (op == BTC_OP_FORWARD || op == BTC_OP_BACKWARD) {
        kind = mixed ? 1 : 0;
        variants = 2;
        return true;
    }
    if (op == BTC_OP_RESIDUAL) {
        kind = 0;
        variants = 2;
        return true;
    }
    if (op == BTC_TUNE_SWEEP_SHAPE) {
        kind = mixed ? 1 : 0;
        variants = 3;
        return true;
    }
    return false;
}

// Level bucket of a key: the factor distinguishes level 0 from the others;
// the sweeps and the residual ignore the level.
int bucket_of(int op, int level) { return (op == BTC_OP_FACTOR && level > 0) ? 1 : 0; }

}  // namespace

extern "C" {

BTC_API int btc_tune_get(int32_t op, int32_t precision, int64_t n, int32_t level, int32_t* variant) {
    if (op < BTC_OP_FACTOR || op > BTC_TUNE_SWEEP_SHAPE) return -1;
    if (precision != BTC_FP64 && !is_mixed(precision)) return -2;
    if (n < 1 || n > BTC_MAX_BLOCK) return -3;
    if (level < 0) return -4;
    if (!variant) return -5;
    int kind, np, nv;
    *variant = tunable(op, precision, n, kind, np, nv) ? tune_variant(op, kind, np, bucket_of(op, level)) : 0;
    return BTC_OK;
}

BTC_API int btc_tune_set(int32_t op, int32_t precision, int64_t n, int32_t level, int32_t variant) {
    if (op < BTC_OP_FACTOR || op > BTC_TUNE_SWEEP_SHAPE) return -1;
    if (precision != BTC_FP64 && !is_mixed(precision)) return -2;
    if (n < 1 || n > BTC_MAX_BLOCK) return -3;
    if (level < 0) return -4;
    int kind, np, nv;
    if (!tunable(op, precision, n, kind, np, nv)) return variant == 0 ? BTC_OK : BTC_ERR_UNSUPPORTED;
    if (variant < 0 || variant >= nv) return -5;
    tune_set(op, kind, np, bucket_of(op, level), variant);
    save_tune_cache();
    return BTC_OK;
}

// Tune the table for a batch: every key the batch touches is tried variant
// by variant (the others at their current choice) on the whole batched
// factor + solve, and the fastest kept (coordinate descent, one pass, keys
// in the order factor, sweep shape, sweeps, residual).
BTC_API int btc_autotune_batched(btc_runner r, int32_t count, const btc_handle* h, const double* const* A_diag,
                                 const double* const* A_off, const double* const* B, double* const* X,
                                 const int64_t* nrhs, int32_t reps) {
    if (!r) return -1;
    if (count < 1) return -2;
    if (!h || !A_diag || !A_off) return -3;
    if (!B || !X) return -6;
    if (!nrhs) return -8;
    if (reps < 1) return -9;
    bool multi = false;
    for (int32_t k = 0; k < count; ++k) {
        if (!h[k] || !A_diag[k] || (h[k]->N > 1 && !A_off[k])) return -3;
        if (!B[k] || !X[k] || B[k] == X[k]) return -6;
        if (nrhs[k] < 1) return -8;
        multi = multi || nrhs[k] > 1;
    }
    struct Key {
        int op, kind, np, bucket, nv;
        bool operator<(const Key& o) const {
            return std::tie(op, kind, np, bucket) < std::tie(o.op, o.kind, o.np, o.bucket);
        }
    };
    std::map<Key, int> keys;  // key -> its place in the descent
    const int order[6] = {BTC_OP_FACTOR, BTC_TUNE_SWEEP_SHAPE, BTC_OP_FORWARD, BTC_OP_BACKWARD, BTC_OP_RESIDUAL, -1};
    for (int oi = 0; order[oi] >= 0; ++oi) {
        const int op = order[oi];
        if ((op == BTC_OP_FORWARD || op == BTC_OP_BACKWARD || op == BTC_OP_RESIDUAL) && !multi) continue;
        for (int32_t k = 0; k < count; ++k) {
            int kind, np, nv;
            if (!tunable(op, h[k]->precision, h[k]->n, kind, np, nv)) continue;
            const int nb = (op == BTC_OP_FACTOR && h[k]->levels > 1) ? 2 : 1;
            for (int b = 0; b < nb; ++b) keys.emplace(Key{op, kind, np, b, nv}, oi);
        }
    }
    std::vector<std::pair<int, Key>> seq;
    for (auto& kv : keys) seq.push_back({kv.second, kv.first});
    std::stable_sort(seq.begin(), seq.end(), [](const std::pair<int, Key>& a, const std::pair<int, Key>& b) {
        return a.first < b.first;
    });
    // median wall time of reps batched factor + solve calls (after one warm-up)
    auto run_once = [&]() -> int {
        int rc = btc_factor_batched(r, count, h, A_diag, A_off, nullptr);
        if (rc == BTC_OK) rc = btc_solve_batched(r, count, h, B, X, nrhs, nullptr);
        if (rc == BTC_OK) rc = btc_runner_sync(r);
        return rc;
    };
    auto time_batch = [&](double& ms) -> int {
        int rc = run_once();
        std::vector<double> t;
        for (int k = 0; k < reps && rc == BTC_OK; ++k) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = run_once();
            t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        if (rc != BTC_OK) return rc;
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return BTC_OK;
    };
    for (auto& e : seq) {
        const Key& k = e.second;
        double best = 1e300;
        int pick = tune_variant(k.op, k.kind, k.np, k.bucket);
        for (int v = 0; v < k.nv; ++v) {
            tune_set(k.op, k.kind, k.np, k.bucket, v);
            double ms = 0.0;
            const int rc = time_batch(ms);
            if (rc != BTC_OK) {
                tune_set(k.op, k.kind, k.np, k.bucket, pick);
                return rc;
            }
            if (ms < best) {
                best = ms;
                pick = v;
            }
        }
        tune_set(k.op, k.kind, k.np, k.bucket, pick);
    }
    save_tune_cache();
    // leave every instance factored and solved with the final choices
    return run_once();
}

BTC_API int btc_autotune(btc_handle h, const double* A_diag, const double* A_off, const double* B, double* X,
                         int64_t nrhs, int32_t reps, void* stream) {
    if (!h) return -1;
    if (!A_diag || (h->N > 1 && !A_off)) return -2;
    if (!B || !X || B == X) return -4;
    if (nrhs < 1) return -6;
    if (reps < 1) return -7;
    int kind, np, nv;
    // factor: per level bucket, the variant with the least summed level time
    if (tunable(BTC_OP_FACTOR, h->precision, h->n, kind, np, nv)) {
        double best[2] = {1e300, 1e300};
        int pick[2] = {0, 0};
        for (int v = 0; v < nv; ++v) {
            tune_set(BTC_OP_FACTOR, kind, np, 0, v);
            tune_set(BTC_OP_FACTOR, kind, np, 1, v);
            int rc = btc_refactor(h, A_diag, A_off, stream);  // warm-up
            if (rc == BTC_OK) rc = btc_profile(h, 1);
            for (int k = 0; k < reps && rc == BTC_OK; ++k) rc = btc_refactor(h, A_diag, A_off, stream);
            double ms[64] = {};
            if (rc == BTC_OK) rc = btc_profile_read(h, 0, ms, nullptr, 64) < 0 ? BTC_ERR_HIP : BTC_OK;
            btc_profile(h, 0);
            if (rc != BTC_OK) return rc;
            const double t[2] = {ms[0], [&] { double a = 0; for (int l = 1; l < h->levels; ++l) a += ms[l]; return a; }()};
            for (int b = 0; b < 2; ++b)
                if (t[b] < best[b]) {
                    best[b] = t[b];
                    pick[b] = v;
                }
        }
        tune_set(BTC_OP_FACTOR, kind, np, 0, pick[0]);
        tune_set(BTC_OP_FACTOR, kind, np, 1, pick[1]);
    }
    int rc = btc_refactor(h, A_diag, A_off, stream);
    if (rc != BTC_OK) return rc;
    // sweep launch shape: the whole solve timed per shape (results identical)
    {
        tunable(BTC_TUNE_SWEEP_SHAPE, h->precision, h->n, kind, np, nv);
        hipStream_t st = (hipStream_t)stream;
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            return BTC_ERR_HIP;
        }
        double best = 1e300;
        int pick = 0;
        for (int v = 0; v < nv && rc == BTC_OK; ++v) {
            tune_set(BTC_TUNE_SWEEP_SHAPE, kind, np, 0, v);
            rc = btc_solve(h, B, X, nrhs, stream, nullptr);  // warm-up
            float ms = 0.f;
            if (rc == BTC_OK && hipEventRecord(a, st) != hipSuccess) rc = BTC_ERR_HIP;
            for (int k = 0; k < reps && rc == BTC_OK; ++k) rc = btc_solve(h, B, X, nrhs, stream, nullptr);
            if (rc == BTC_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                                 hipEventElapsedTime(&ms, a, b) != hipSuccess))
                rc = BTC_ERR_HIP;
            if (rc == BTC_OK && ms < best) {
                best = ms;
                pick = v;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        tune_set(BTC_TUNE_SWEEP_SHAPE, kind, np, 0, pick);
        if (rc != BTC_OK) return rc;
    }
    // sweeps and residual: only with several right-hand sides
    if (nrhs > 1) {
        const int ops[3] = {BTC_OP_FORWARD, BTC_OP_BACKWARD, BTC_OP_RESIDUAL};
        double tot[3][2] = {};
        for (int v = 0; v < 2; ++v) {
            for (int op : ops) {
                tunable(op, h->precision, h->n, kind, np, nv);
                tune_set(op, kind, np, 0, v);
            }
            btc_solve_info info;
            rc = btc_solve(h, B, X, nrhs, stream, nullptr);  // warm-up
            if (rc == BTC_OK) rc = btc_profile(h, 1);
            for (int k = 0; k < reps && rc == BTC_OK; ++k) rc = btc_solve(h, B, X, nrhs, stream, &info);
            double ms[3][64] = {};
            for (int ph = 0; ph < 3 && rc == BTC_OK; ++ph)
                if (btc_profile_read(h, ph == 2 ? 3 : ph + 1, ms[ph], nullptr, 64) < 0) rc = BTC_ERR_HIP;
            btc_profile(h, 0);
            if (rc != BTC_OK) return rc;
            for (int ph = 0; ph < 3; ++ph)
                for (int l = 0; l < 64; ++l)
                    if (ph < 2 || l == 1) tot[ph][v] += ms[ph][l];  // refinement phase entry 1: residual
        }
        for (int k = 0; k < 3; ++k) {
            tunable(ops[k], h->precision, h->n, kind, np, nv);
            // the FP64 path forms a residual only when asked for it: keep the default
            const int v = (k == 2 && tot[2][0] == 0.0 && tot[2][1] == 0.0) ? 0 : (tot[k][1] < tot[k][0] ? 1 : 0);
            tune_set(ops[k], kind, np, 0, v);
        }
    }
    save_tune_cache();
    return BTC_OK;
}

BTC_API int btc_autotune_strategy(int64_t N, int64_t n, int32_t precision, const double* A_diag,
                                  const double* A_off, const double* B, double* X, int64_t nrhs, int32_t reps,
                                  void* stream, double* ms) {
    if (N < 1) return -1;
    if (n < 1 || n > BTC_MAX_BLOCK) return -2;
    if (precision != BTC_FP64 && !is_mixed(precision)) return -3;
    if (!A_diag || (N > 1 && !A_off)) return -4;
    if (!B || !X || B == X) return -6;
    if (nrhs < 1) return -8;
    if (reps < 1) return -9;
    hipStream_t st = (hipStream_t)stream;
    // candidates: multi-stage, k-stage with k = 0, 1, 2, partition with p = 2, 4
    constexpr int kCand = 6;
    double t[kCand] = {-1.0, -1.0, -1.0, -1.0, -1.0, -1.0};
    auto cand = [](int c, int32_t& strategy, int32_t& stages) {
        strategy = c == 0 ? BTC_STRATEGY_MULTISTAGE : c <= 3 ? BTC_STRATEGY_KSTAGE : BTC_STRATEGY_PARTITION;
        stages = c == 0 ? 0 : c <= 3 ? c - 1 : (c == 4 ? 2 : 4);
    };
    int best = -1;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return BTC_ERR_HIP;
    }
    int rc = BTC_OK;
    for (int c = 0; c < kCand && rc == BTC_OK; ++c) {
        btc_options o{};
        o.precision = precision;
        cand(c, o.strategy, o.stages);
        if (c > 0 && (precision != BTC_FP64 || n > 64)) continue;
        if (o.strategy == BTC_STRATEGY_KSTAGE && o.stages >= num_levels(N)) continue;
        int64_t n1 = 0, nk = 0;
        if (o.strategy == BTC_STRATEGY_PARTITION && !partition_sizes(N, o.stages, n1, nk)) continue;
        btc_handle h = nullptr;
        rc = btc_create(N, n, &o, &h);
        if (rc != BTC_OK) break;
        rc = btc_refactor(h, A_diag, A_off, stream);  // warm-up
        if (rc == BTC_OK) rc = btc_solve(h, B, X, nrhs, stream, nullptr);
        if (rc == BTC_OK && hipEventRecord(a, st) != hipSuccess) rc = BTC_ERR_HIP;
        for (int k = 0; k < reps && rc == BTC_OK; ++k) {
            rc = btc_refactor(h, A_diag, A_off, stream);
            if (rc == BTC_OK) rc = btc_solve(h, B, X, nrhs, stream, nullptr);
        }
        float ms1 = 0.f;
        if (rc == BTC_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                             hipEventElapsedTime(&ms1, a, b) != hipSuccess))
            rc = BTC_ERR_HIP;
        int64_t info = 0;
        if (rc == BTC_OK) rc = btc_status(h, &info);
        btc_destroy(h);
        if (rc == BTC_OK && info != 0) rc = BTC_ERR_NOT_SPD;
        if (rc != BTC_OK) break;
        t[c] = (double)ms1 / reps;
        if (best < 0 || t[c] < t[best]) best = c;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != BTC_OK) return rc;
    int32_t bs = BTC_STRATEGY_MULTISTAGE, bk = 0;
    cand(best < 0 ? 0 : best, bs, bk);
    strategy_set(N, n, precision, bs, bk);
    save_tune_cache();
    if (ms)
        for (int c = 0; c < kCand; ++c) ms[c] = t[c];
    return BTC_OK;
}

BTC_API int btc_select_strategy(int64_t N, int64_t n, int32_t precision, int32_t* strategy, int32_t* stages) {
    if (N < 1) return -1;
    if (n < 1 || n > BTC_MAX_BLOCK) return -2;
    if (precision != BTC_FP64 && !is_mixed(precision)) return -3;
    if (!strategy || !stages) return -4;
    select_strategy(N, n, precision, strategy, stages);
    if (*strategy == BTC_STRATEGY_KSTAGE && *stages >= num_levels(N)) *strategy = BTC_STRATEGY_MULTISTAGE;
    return BTC_OK;
}

}  // extern "C"
