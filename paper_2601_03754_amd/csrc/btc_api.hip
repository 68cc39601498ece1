// Host side of the libbtc C ABI (declared in include/btc.h): argument
// checking, the device memory of a handle, the level schedule and the
// launches, and the iterative-refinement driver of the mixed-precision path.
#include "btc.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <new>
#include <vector>

#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {
int padded_block_mixed(int n);
}

namespace {

constexpr unsigned long long kInfoOk = ~0ull;

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

}  // namespace

struct btc_handle_s {
    int64_t N = 0;
    int64_t n = 0;
    int32_t precision = BTC_FP64;
    int32_t max_refine = 0;
    double tol = 0.0;
    int levels = 0;  // floor(log2 N) + 1
    int device = 0;
    // FP64 factor (BTC_FP64)
    double* Ld = nullptr;
    double* Rb = nullptr;
    double* Tb = nullptr;
    // mixed factor (BTC_FP32_IR): FP64 Schur complements, FP32 factor
    double* S64 = nullptr;
    float* L32 = nullptr;
    float* R32 = nullptr;
    float* T32 = nullptr;
    unsigned long long* info = nullptr;
    // solve workspace, grown on demand (one allocation)
    void* ws = nullptr;
    int64_t ws_m = 0;
    hipStream_t stream = nullptr;  // stream of the last call
    bool factored = false;
    bool failed_known = false;     // a status check saw a breakdown
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
    double prof_ms[4][64] = {};
    int64_t prof_n[4][64] = {};
};

namespace {

bool is_mixed(int32_t p) { return p == BTC_FP32_IR; }

int num_levels(int64_t N) {
    int L = 0;
    while ((((int64_t)1) << (L + 1)) <= N) ++L;
    return L + 1;
}

int64_t level_nodes(int64_t N, int l) {
    const int64_t s = (int64_t)1 << l;
    return (N + s) / (2 * s);
}

int to_code(hipError_t e) {
    if (e == hipSuccess) return BTC_OK;
    if (e == hipErrorOutOfMemory) return BTC_ERR_OOM;
    return BTC_ERR_HIP;
}

template <class P>
void dfree(P*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
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
    dfree(h->Ld);
    dfree(h->Rb);
    dfree(h->Tb);
    dfree(h->S64);
    dfree(h->L32);
    dfree(h->R32);
    dfree(h->T32);
    dfree(h->info);
    dfree(h->ws);
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
// Phases: 0 factor, 1 forward sweep, 2 backward sweep, 3 residual/refinement.
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

size_t factor_bytes(int64_t N, int64_t n, int32_t prec) {
    const size_t nn = (size_t)N * (size_t)n * (size_t)n;
    if (is_mixed(prec)) return nn * (sizeof(double) + 3 * sizeof(float));
    return 3 * nn * sizeof(double);
}

// Solve workspace: FP64 path: Y, U, V (FP64); mixed: r, y, u, v, d (FP32);
// both: partial norms (FP64, N x m x 2) and the refinement state.
size_t workspace_bytes(int64_t N, int64_t n, int32_t prec, int64_t m) {
    const size_t v = (size_t)N * (size_t)n * (size_t)m;
    const size_t tail = 2 * (size_t)N * (size_t)m * sizeof(double) + 256 + 256 + 256;
    if (is_mixed(prec)) return 5 * v * sizeof(float) + tail;
    return 3 * v * sizeof(double) + tail;
}

struct Workspace {
    double *Y = nullptr, *U = nullptr, *V = nullptr;                              // FP64 path
    float *r = nullptr, *y = nullptr, *u = nullptr, *v = nullptr, *d = nullptr;  // mixed
    double* part = nullptr;
    btc::IrState* ir = nullptr;
};

Workspace carve(btc_handle h, int64_t m) {
    Workspace w;
    const size_t v = (size_t)h->N * (size_t)h->n * (size_t)m;
    char* p = (char*)h->ws;
    auto align = [](char* q) { return (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255); };
    if (is_mixed(h->precision)) {
        w.r = (float*)p;
        p += v * sizeof(float);
        w.y = (float*)p;
        p += v * sizeof(float);
        w.u = (float*)p;
        p += v * sizeof(float);
        w.v = (float*)p;
        p += v * sizeof(float);
        w.d = (float*)p;
        p += v * sizeof(float);
    } else {
        w.Y = (double*)p;
        p += v * sizeof(double);
        w.U = (double*)p;
        p += v * sizeof(double);
        w.V = (double*)p;
        p += v * sizeof(double);
    }
    p = align(p);
    w.part = (double*)p;
    p += 2 * (size_t)h->N * (size_t)m * sizeof(double);
    p = align(p);
    w.ir = (btc::IrState*)p;
    return w;
}

int ensure_workspace(btc_handle h, int64_t m) {
    if (m <= h->ws_m && h->ws) return BTC_OK;
    if (h->ws) {
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        dfree(h->ws);
    }
    h->ws_m = 0;
    hipError_t e = hipMalloc(&h->ws, workspace_bytes(h->N, h->n, h->precision, m));
    if (e != hipSuccess) {
        h->ws = nullptr;
        return to_code(e);
    }
    h->ws_m = m;
    return BTC_OK;
}

int launch_factor(btc_handle h, const double* A_diag, const double* A_off, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, h->info, kInfoOk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return to_code(e);
    if (is_mixed(h->precision)) {
        btc::FactorParamsMixed p{};
        p.A_diag = A_diag;
        p.A_off = A_off;
        p.S64 = h->S64;
        p.L32 = h->L32;
        p.R32 = h->R32;
        p.T32 = h->T32;
        p.info = h->info;
        p.N = h->N;
        p.n = (int32_t)h->n;
        for (int l = 0; l < h->levels; ++l) {
            p.level = l;
            const int64_t nodes = level_nodes(h->N, l);
            e = timed(h, 0, l, st, [&] { return btc::launch_factor_level_mixed(p, nodes, st); });
            if (e != hipSuccess) return to_code(e);
        }
    } else {
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
    }
    h->A_diag = A_diag;
    h->A_off = A_off;
    h->stream = st;
    h->factored = true;
    h->failed_known = false;
    return BTC_OK;
}

template <class T>
hipError_t sweeps(btc_handle h, btc::SweepParams<T> p, hipStream_t st) {
    for (int l = 0; l < h->levels; ++l) {
        p.level = l;
        hipError_t e = timed(h, 1, l, st, [&] { return btc::launch_sweep(p, level_nodes(h->N, l), false, st); });
        if (e != hipSuccess) return e;
    }
    for (int l = h->levels - 1; l >= 0; --l) {
        p.level = l;
        hipError_t e = timed(h, 2, l, st, [&] { return btc::launch_sweep(p, level_nodes(h->N, l), true, st); });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int read_info(btc_handle h, hipStream_t st, unsigned long long* v) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return to_code(e);
    e = hipMemcpy(v, h->info, sizeof(*v), hipMemcpyDeviceToHost);
    return to_code(e);
}

}  // namespace

extern "C" {

BTC_API int btc_version(void) { return 200; }

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
    if (N < 1 || n < 1 || n > BTC_MAX_BLOCK || nrhs < 0) return 0;
    if (precision != BTC_FP64 && !is_mixed(precision)) return 0;
    size_t b = factor_bytes(N, n, precision) + sizeof(unsigned long long);
    if (nrhs > 0) b += workspace_bytes(N, n, precision, nrhs);
    return b;
}

BTC_API int btc_factor(const double* A_diag, const double* A_off, int64_t N, int64_t n,
                       const btc_options* opt, void* stream, btc_handle* out) {
    if (!A_diag) return -1;
    if (N > 1 && !A_off) return -2;
    if (N < 1) return -3;
    if (n < 1) return -4;
    if (n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    const int32_t prec = opt ? opt->precision : BTC_FP64;
    if (prec != BTC_FP64 && !is_mixed(prec)) return -5;
    if (opt && (opt->max_refine < 0 || !(opt->tol >= 0.0))) return -5;
    if (!out) return -7;
    *out = nullptr;
    btc_handle h = new (std::nothrow) btc_handle_s();
    if (!h) return BTC_ERR_OOM;
    h->N = N;
    h->n = n;
    h->precision = prec;
    h->max_refine = (opt && opt->max_refine > 0) ? opt->max_refine : BTC_DEFAULT_MAX_REFINE;
    h->tol = (opt && opt->tol > 0.0) ? opt->tol : BTC_DEFAULT_TOL;
    h->levels = num_levels(N);
    (void)hipGetDevice(&h->device);
    const size_t nn = (size_t)N * (size_t)n * (size_t)n;
    hipError_t e = hipMalloc(&h->info, sizeof(unsigned long long));
    if (is_mixed(prec)) {
        if (e == hipSuccess) e = hipMalloc(&h->S64, nn * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&h->L32, nn * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&h->R32, nn * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&h->T32, nn * sizeof(float));
    } else {
        if (e == hipSuccess) e = hipMalloc(&h->Ld, nn * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&h->Rb, nn * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&h->Tb, nn * sizeof(double));
    }
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
    const bool mixed = is_mixed(h->precision);
    if (mixed && X == B) return -3;  // refinement reads b after x is written
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_workspace(h, nrhs);
    if (rc != BTC_OK) return rc;
    Workspace w = carve(h, nrhs);
    h->stream = st;
    hipError_t e = hipSuccess;
    btc::ResidualParams r{};
    r.A_diag = h->A_diag;
    r.A_off = h->A_off;
    r.B = B;
    r.X = X;
    r.part = w.part;
    r.state = w.ir;
    r.N = h->N;
    r.n = (int32_t)h->n;
    r.m = (int32_t)nrhs;

    if (!mixed) {
        btc::SweepParams<double> p{};
        p.Ld = h->Ld;
        p.Rb = h->Rb;
        p.Tb = h->Tb;
        p.B = B;
        p.X = X;
        p.Y = w.Y;
        p.U = w.U;
        p.V = w.V;
        p.info = h->info;
        p.N = h->N;
        p.n = (int32_t)h->n;
        p.m = (int32_t)nrhs;
        e = sweeps(h, p, st);
        if (e != hipSuccess) return to_code(e);
        if (!info) return BTC_OK;
        // FP64 residual of the solution, for the caller's information
        e = btc::launch_ir_init(w.ir, 0.0, 1, B, nullptr, 0, st);
        if (e == hipSuccess) e = btc::launch_residual(r, st);
        if (e == hipSuccess) e = btc::launch_ir_check(w.ir, w.part, h->N, (int)nrhs, st);
        if (e != hipSuccess) return to_code(e);
    } else {
        // iterative refinement: x_0 = solve_lo(b); repeat: r = b - Psi x in
        // FP64; stop when max_q ||r_q||/||b_q|| <= tol (or stalled, or the
        // budget is spent); x += solve_lo(r).  Every launch after the stop
        // returns at once (device flag), so no host synchronisation is needed.
        const size_t count = (size_t)h->N * (size_t)h->n * (size_t)nrhs;
        e = timed(h, 3, 0, st, [&] {
            return btc::launch_ir_init(w.ir, h->tol, 1 + h->max_refine, B, w.r, count, st);
        });
        if (e != hipSuccess) return to_code(e);
        btc::SweepParams<float> p{};
        p.Ld = h->L32;
        p.Rb = h->R32;
        p.Tb = h->T32;
        p.B = w.r;
        p.X = w.d;
        p.Y = w.y;
        p.U = w.u;
        p.V = w.v;
        p.X64 = X;
        p.info = h->info;
        p.skip = &w.ir->done;
        p.N = h->N;
        p.n = (int32_t)h->n;
        p.m = (int32_t)nrhs;
        r.R32 = w.r;
        for (int it = 0; it <= h->max_refine; ++it) {
            p.first = (it == 0);
            e = sweeps(h, p, st);
            if (e == hipSuccess) e = timed(h, 3, 1, st, [&] { return btc::launch_residual(r, st); });
            if (e == hipSuccess)
                e = timed(h, 3, 2, st, [&] { return btc::launch_ir_check(w.ir, w.part, h->N, (int)nrhs, st); });
            if (e != hipSuccess) return to_code(e);
        }
        if (!info) return BTC_OK;
    }
    unsigned long long v = 0;
    rc = read_info(h, st, &v);
    if (rc != BTC_OK) return rc;
    if (v != kInfoOk) {
        h->failed_known = true;
        return BTC_ERR_NOT_SPD;
    }
    btc::IrState s{};
    e = hipMemcpy(&s, w.ir, sizeof(s), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return to_code(e);
    info->steps = mixed ? s.steps - 1 : 0;
    info->converged = mixed ? s.converged : 1;
    info->relres = s.relres;
    return BTC_OK;
}

BTC_API int btc_status(btc_handle h, int64_t* info) {
    if (!h) return -1;
    if (!info) return -2;
    if (!h->factored) return -1;
    unsigned long long v = 0;
    const int rc = read_info(h, h->stream, &v);
    if (rc != BTC_OK) return rc;
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
    if (phase < 0 || phase > 3) return -2;
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
    std::vector<float> tmp32;
    double* outs[3] = {Ld, Rb, Tb};
    const bool mixed = is_mixed(h->precision);
    const double* srcs[3] = {h->Ld, h->Rb, h->Tb};
    const float* srcs32[3] = {h->L32, h->R32, h->T32};
    if (mixed) tmp32.resize(nn * (size_t)N);
    for (int a = 0; a < 3; ++a) {
        if (!outs[a]) continue;
        if (mixed) {
            e = hipMemcpy(tmp32.data(), srcs32[a], nn * (size_t)N * sizeof(float), hipMemcpyDeviceToHost);
            for (size_t k = 0; k < tmp.size(); ++k) tmp[k] = (double)tmp32[k];
        } else {
            e = hipMemcpy(tmp.data(), srcs[a], nn * (size_t)N * sizeof(double), hipMemcpyDeviceToHost);
        }
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
