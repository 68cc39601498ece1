// Host side of the libbtc C ABI (declared in include/btc.h): argument
// checking, device memory of a handle, the level schedule and the launches.
#include "btc.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <new>
#include <vector>

#include "btc_device.h"
#include "btc_kernels.h"

namespace {

constexpr unsigned long long kInfoOk = ~0ull;

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

}  // namespace

struct btc_handle_s {
    int64_t N = 0;
    int64_t n = 0;
    int32_t precision = BTC_FP64;
    int levels = 0;  // floor(log2 N) + 1
    int device = 0;
    double* Ld = nullptr;
    double* Rb = nullptr;
    double* Tb = nullptr;
    unsigned long long* info = nullptr;
    // solve workspace, grown on demand
    double* Y = nullptr;
    double* U = nullptr;
    double* V = nullptr;
    int64_t ws_m = 0;
    hipStream_t stream = nullptr;  // stream of the last call
    bool factored = false;
    bool failed_known = false;     // a btc_status call saw a breakdown
    const double* A_diag = nullptr;
    const double* A_off = nullptr;
    // optional per-launch timing
    struct Timed {
        hipEvent_t a, b;
        int phase, level;
    };
    bool prof = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[3][64] = {};
    int64_t prof_n[3][64] = {};
};

namespace {

int num_levels(int64_t N) {
    int L = 0;
    while ((((int64_t)1) << (L + 1)) <= N) ++L;
    return L + 1;
}

int64_t level_nodes(int64_t N, int l) {
    const int64_t s = (int64_t)1 << l;
    return (N + s) / (2 * s);
}

void free_all(btc_handle h) {
    if (!h) return;
    for (auto& t : h->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    h->pending.clear();
    for (auto e : h->pool) (void)hipEventDestroy(e);
    h->pool.clear();
    if (h->Ld) (void)hipFree(h->Ld);
    if (h->Rb) (void)hipFree(h->Rb);
    if (h->Tb) (void)hipFree(h->Tb);
    if (h->info) (void)hipFree(h->info);
    if (h->Y) (void)hipFree(h->Y);
    if (h->U) (void)hipFree(h->U);
    if (h->V) (void)hipFree(h->V);
}

hipEvent_t take_event(btc_handle h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrapper: brackets the launch with events when profiling is on.
template <class F>
hipError_t timed(btc_handle h, int phase, int level, hipStream_t st, F&& launch) {
    if (!h->prof) return launch();
    hipEvent_t a = take_event(h), b = take_event(h);
    if (!a || !b) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, st);
    hipError_t e = launch();
    (void)hipEventRecord(b, st);
    h->pending.push_back({a, b, phase, level});
    return e;
}

void drain_profile(btc_handle h) {
    for (auto& t : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess && t.level < 64) {
            h->prof_ms[t.phase][t.level] += ms;
            h->prof_n[t.phase][t.level] += 1;
        }
        h->pool.push_back(t.a);
        h->pool.push_back(t.b);
    }
    h->pending.clear();
}

int to_code(hipError_t e) {
    if (e == hipSuccess) return BTC_OK;
    if (e == hipErrorOutOfMemory) return BTC_ERR_OOM;
    return BTC_ERR_HIP;
}

int launch_factor(btc_handle h, const double* A_diag, const double* A_off, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, h->info, kInfoOk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return to_code(e);
    btc::FactorParams p{};
    p.A_diag = A_diag;
    p.A_off = A_off;
    p.Ld = h->Ld;
    p.Rb = h->Rb;
    p.Tb = h->Tb;
    p.info = h->info;
    p.N = h->N;
    p.n = (int32_t)h->n;
    for (int l = 0; l < h->levels; ++l) {
        p.level = l;
        const int64_t nodes = level_nodes(h->N, l);
        e = timed(h, 0, l, st, [&] {
            return btc::padded_block((int)h->n) >= 16 ? btc::launch_factor_level_mfma(p, nodes, st)
                                                      : btc::launch_factor_level_f64(p, nodes, st);
        });
        if (e != hipSuccess) return to_code(e);
    }
    h->A_diag = A_diag;
    h->A_off = A_off;
    h->stream = st;
    h->factored = true;
    h->failed_known = false;
    return BTC_OK;
}

int ensure_workspace(btc_handle h, int64_t m) {
    if (m <= h->ws_m) return BTC_OK;
    if (h->Y) (void)hipFree(h->Y);
    if (h->U) (void)hipFree(h->U);
    if (h->V) (void)hipFree(h->V);
    h->Y = h->U = h->V = nullptr;
    h->ws_m = 0;
    const size_t bytes = (size_t)h->N * (size_t)h->n * (size_t)m * sizeof(double);
    hipError_t e = hipMalloc(&h->Y, bytes);
    if (e == hipSuccess) e = hipMalloc(&h->U, bytes);
    if (e == hipSuccess) e = hipMalloc(&h->V, bytes);
    if (e != hipSuccess) return to_code(e);
    h->ws_m = m;
    return BTC_OK;
}

}  // namespace

extern "C" {

BTC_API int btc_version(void) { return 100; }

BTC_API const char* btc_error_string(int code) {
    switch (code) {
        case BTC_OK: return "ok";
        case BTC_ERR_HIP: return "HIP runtime error";
        case BTC_ERR_OOM: return "out of device memory";
        case BTC_ERR_NOT_SPD: return "matrix is not positive definite (factorization broke down)";
        case BTC_ERR_UNSUPPORTED: return "unsupported block size or option";
        default: break;
    }
    if (code < 0 && code > -100) return "invalid argument";
    return "unknown code";
}

BTC_API int btc_permutation(int64_t N, int64_t* order) {
    if (N < 1) return -1;
    if (!order) return -2;
    int64_t p = 0;
    for (int64_t s = 1; s <= N; s *= 2)
        for (int64_t i = s; i <= N; i += 2 * s) order[p++] = i;
    return BTC_OK;
}

BTC_API size_t btc_footprint_bytes(int64_t N, int64_t n, int32_t precision, int64_t nrhs) {
    if (N < 1 || n < 1 || n > BTC_MAX_BLOCK || nrhs < 0 || precision != BTC_FP64) return 0;
    const size_t nn = (size_t)n * (size_t)n;
    return 3 * (size_t)N * nn * sizeof(double) + sizeof(unsigned long long) +
           3 * (size_t)N * (size_t)n * (size_t)nrhs * sizeof(double);
}

BTC_API int btc_factor(const double* A_diag, const double* A_off, int64_t N, int64_t n,
                       const btc_options* opt, void* stream, btc_handle* out) {
    if (!A_diag) return -1;
    if (N > 1 && !A_off) return -2;
    if (N < 1) return -3;
    if (n < 1) return -4;
    if (n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    if (opt && opt->precision != BTC_FP64) return -5;
    if (!out) return -7;
    *out = nullptr;
    btc_handle h = new (std::nothrow) btc_handle_s();
    if (!h) return BTC_ERR_OOM;
    h->N = N;
    h->n = n;
    h->levels = num_levels(N);
    (void)hipGetDevice(&h->device);
    const size_t bytes = (size_t)N * (size_t)n * (size_t)n * sizeof(double);
    hipError_t e = hipMalloc(&h->Ld, bytes);
    if (e == hipSuccess) e = hipMalloc(&h->Rb, bytes);
    if (e == hipSuccess) e = hipMalloc(&h->Tb, bytes);
    if (e == hipSuccess) e = hipMalloc(&h->info, sizeof(unsigned long long));
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return to_code(e);
    }
    const int rc = launch_factor(h, A_diag, A_off, (hipStream_t)stream);
    if (rc != BTC_OK) {
        free_all(h);
        delete h;
        return rc;
    }
    *out = h;
    return BTC_OK;
}

BTC_API int btc_refactor(btc_handle h, const double* A_diag, const double* A_off, void* stream) {
    if (!h) return -1;
    if (!A_diag) return -2;
    if (h->N > 1 && !A_off) return -3;
    return launch_factor(h, A_diag, A_off, (hipStream_t)stream);
}

BTC_API int btc_solve(btc_handle h, const double* B, double* X, int64_t nrhs, void* stream,
                      btc_solve_info* info) {
    if (!h) return -1;
    if (!B) return -2;
    if (!X) return -3;
    if (nrhs < 0) return -4;
    if (!h->factored) return -1;
    if (h->failed_known) return BTC_ERR_NOT_SPD;
    if (nrhs == 0) return BTC_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_workspace(h, nrhs);
    if (rc != BTC_OK) return rc;
    btc::SolveParams p{};
    p.Ld = h->Ld;
    p.Rb = h->Rb;
    p.Tb = h->Tb;
    p.B = B;
    p.X = X;
    p.Y = h->Y;
    p.U = h->U;
    p.V = h->V;
    p.info = h->info;
    p.N = h->N;
    p.n = (int32_t)h->n;
    p.m = (int32_t)nrhs;
    for (int l = 0; l < h->levels; ++l) {
        p.level = l;
        hipError_t e = timed(h, 1, l, st, [&] { return btc::launch_solve_level_f64(p, level_nodes(h->N, l), false, st); });
        if (e != hipSuccess) return to_code(e);
    }
    for (int l = h->levels - 1; l >= 0; --l) {
        p.level = l;
        hipError_t e = timed(h, 2, l, st, [&] { return btc::launch_solve_level_f64(p, level_nodes(h->N, l), true, st); });
        if (e != hipSuccess) return to_code(e);
    }
    h->stream = st;
    if (info) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return to_code(e);
        unsigned long long v = 0;
        e = hipMemcpy(&v, h->info, sizeof(v), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return to_code(e);
        if (v != kInfoOk) {
            h->failed_known = true;
            return BTC_ERR_NOT_SPD;
        }
        info->steps = 0;
        info->converged = 1;
        info->relres = -1.0;
    }
    return BTC_OK;
}

BTC_API int btc_status(btc_handle h, int64_t* info) {
    if (!h) return -1;
    if (!info) return -2;
    if (!h->factored) return -1;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return to_code(e);
    unsigned long long v = 0;
    e = hipMemcpy(&v, h->info, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return to_code(e);
    *info = (v == kInfoOk) ? 0 : (int64_t)v;
    h->failed_known = (v != kInfoOk);
    return BTC_OK;
}

BTC_API void btc_destroy(btc_handle h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
}

BTC_API int btc_profile(btc_handle h, int enable) {
    if (!h) return -1;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drain_profile(h);
    h->prof = enable != 0;
    memset(h->prof_ms, 0, sizeof(h->prof_ms));
    memset(h->prof_n, 0, sizeof(h->prof_n));
    return BTC_OK;
}

BTC_API int btc_profile_read(btc_handle h, int phase, double* ms, int64_t* counts, int max_levels) {
    if (!h) return -1;
    if (phase < 0 || phase > 2) return -2;
    if (max_levels < 0) return -5;
    if (h->stream) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return to_code(e);
    }
    drain_profile(h);
    for (int l = 0; l < max_levels && l < 64; ++l) {
        if (ms) ms[l] = (l < h->levels) ? h->prof_ms[phase][l] : 0.0;
        if (counts) counts[l] = (l < h->levels) ? h->prof_n[phase][l] : 0;
    }
    return h->levels;
}

BTC_API int btc_export_factor(btc_handle h, double* Ld, double* Rb, double* Tb) {
    if (!h) return -1;
    if (!h->factored) return -1;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return to_code(e);
    const int64_t N = h->N;
    const size_t nn = (size_t)h->n * (size_t)h->n;
    std::vector<double> tmp(nn * (size_t)N);
    double* outs[3] = {Ld, Rb, Tb};
    const double* srcs[3] = {h->Ld, h->Rb, h->Tb};
    for (int a = 0; a < 3; ++a) {
        if (!outs[a]) continue;
        e = hipMemcpy(tmp.data(), srcs[a], nn * (size_t)N * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return to_code(e);
        for (int64_t i = 1; i <= N; ++i) {
            const int l = btc::level_of(i);
            const int64_t s = (int64_t)1 << l;
            const bool present = (a == 0) || (a == 1 && i + s <= N) || (a == 2 && i > s);
            double* dst = outs[a] + (size_t)(i - 1) * nn;
            if (present)
                memcpy(dst, tmp.data() + (size_t)btc::perm_pos(N, l, i) * nn, nn * sizeof(double));
            else
                memset(dst, 0, nn * sizeof(double));
        }
    }
    return BTC_OK;
}

}  // extern "C"
