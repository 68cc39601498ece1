// Host side of the libbtc C ABI (declared in include/btc.h): argument
// checking, the device memory of a handle, the level schedule and the
// launches, and the iterative-refinement driver of the mixed-precision path.
#include "btc.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "btc_device.h"
#include "btc_handle.h"
#include "btc_kernels.h"

namespace btc_host {
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;
}  // namespace

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}
}  // namespace btc_host

using namespace btc_host;

extern "C" {

BTC_API int btc_version(void) { return 300; }

BTC_API int btc_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*, void*), void* ctx) {
    if ((alloc == nullptr) != (free_ == nullptr)) return -1;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free_ = free_;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return BTC_OK;
}

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

BTC_API int btc_create(int64_t N, int64_t n, const btc_options* opt, btc_handle* out) {
    if (N < 1) return -1;
    if (n < 1) return -2;
    if (n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    const int32_t prec = opt ? opt->precision : BTC_FP64;
    if (prec != BTC_FP64 && !is_mixed(prec)) return -3;
    if (opt && (opt->max_refine < 0 || !(opt->tol >= 0.0))) return -3;
    if (!out) return -4;
    *out = nullptr;
    btc_handle h = new (std::nothrow) btc_handle_s();
    if (!h) return BTC_ERR_OOM;
    h->N = N;
    h->n = n;
    h->precision = prec;
    h->max_refine = (opt && opt->max_refine > 0) ? opt->max_refine
                                                  : (is_bf16(prec) ? BTC_DEFAULT_MAX_REFINE_BF16 : BTC_DEFAULT_MAX_REFINE);
    h->tol = (opt && opt->tol > 0.0) ? opt->tol : BTC_DEFAULT_TOL;
    h->levels = num_levels(N);
    (void)hipGetDevice(&h->device);
    h->alloc = current_allocator();
    const size_t nn = (size_t)N * (size_t)n * (size_t)n;
    auto get = [h](auto*& p, size_t bytes) { return dev_alloc(h->alloc, (void**)&p, bytes, h->stream); };
    hipError_t e = get(h->info, sizeof(unsigned long long));
    if (is_mixed(prec)) {
        if (e == hipSuccess) e = get(h->S64, nn * sizeof(double));
        if (e == hipSuccess) e = get(h->L32, nn * sizeof(float));
        if (e == hipSuccess) e = get(h->R32, nn * sizeof(float));
        if (e == hipSuccess) e = get(h->T32, nn * sizeof(float));
    } else {
        if (e == hipSuccess) e = get(h->Ld, nn * sizeof(double));
        if (e == hipSuccess) e = get(h->Rb, nn * sizeof(double));
        if (e == hipSuccess) e = get(h->Tb, nn * sizeof(double));
    }
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return to_code(e);
    }
    *out = h;
    return BTC_OK;
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
    btc_handle h = nullptr;
    int rc = btc_create(N, n, opt, &h);
    if (rc != BTC_OK) return rc;
    rc = launch_factor(h, A_diag, A_off, (hipStream_t)stream);
    if (rc != BTC_OK) {
        btc_destroy(h);
        return rc;
    }
    *out = h;
    return BTC_OK;
}

BTC_API int btc_refine_info(btc_handle h, btc_solve_info* info) {
    if (!h) return -1;
    if (!info) return -2;
    if (!h->ws) return -1;
    unsigned long long v = 0;
    int rc = read_info(h, h->stream, &v);
    if (rc != BTC_OK) return rc;
    if (v != kInfoOk) {
        h->failed_known = true;
        return BTC_ERR_NOT_SPD;
    }
    const Workspace w = carve(h, h->ws_m);
    btc::IrState s{};
    const hipError_t e = hipMemcpy(&s, w.ir, sizeof(s), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return to_code(e);
    const bool mixed = is_mixed(h->precision);
    info->steps = mixed ? s.steps - 1 : 0;
    info->converged = mixed ? s.converged : 1;
    info->relres = s.relres;
    return BTC_OK;
}

BTC_API int btc_refactor(btc_handle h, const double* A_diag, const double* A_off, void* stream) {
    if (!h) return -1;
    if (!A_diag) return -2;
    if (h->N > 1 && !A_off) return -3;
    return launch_factor(h, A_diag, A_off, (hipStream_t)stream);
}

}  // extern "C"

namespace btc_host {

// Enqueue a solve (and, for the mixed paths, its refinement) with the
// workspace w; fills *info (synchronising) when it is not NULL.  Allocates
// nothing.
int solve_with(btc_handle h, const Workspace& w, const double* B, double* X, int64_t nrhs, hipStream_t st,
               btc_solve_info* info) {
    const bool mixed = is_mixed(h->precision);
    hipError_t e = hipSuccess;
    const int np = btc::padded_block((int)h->n);
    if (!mixed) {
        e = sweeps(h, sweep_desc64(h, w, B, X, nrhs), st);
        if (e != hipSuccess) return to_code(e);
        if (!info) return BTC_OK;
        // FP64 residual of the solution, for the caller's information
        btc::Launch<btc::IrDesc> I{};
        I.single = ir_desc(h, w, nrhs, 0.0, 1);
        btc::Launch<btc::ResidualDesc> R{};
        R.single = residual_desc(h, w, B, X, nrhs, false);
        e = btc::launch_ir_init(I, 1, st);
        if (e == hipSuccess)
            e = timed(h, 3, 1, st, [&] { return btc::launch_residual(R, np, h->N, sweep_mc(BTC_OP_RESIDUAL, 0, np, nrhs), st); });
        if (e == hipSuccess) e = btc::launch_ir_check(I, 1, st);
        if (e != hipSuccess) return to_code(e);
    } else {
        // iterative refinement: x_0 = solve_lo(b); repeat: r = b - Psi x in
        // FP64; stop when max_q ||r_q||/||b_q|| <= tol (or stalled, or the
        // budget is spent); x += solve_lo(r).  Every launch after the stop
        // returns at once (device flag), so no host synchronisation is needed.
        btc::Launch<btc::IrDesc> I{};
        I.single = ir_desc(h, w, nrhs, h->tol, 1 + h->max_refine);
        btc::Launch<btc::ResidualDesc> R{};
        R.single = residual_desc(h, w, B, X, nrhs, true);
        e = timed(h, 3, 0, st, [&] { return btc::launch_ir_init(I, 1, st); });
        if (e != hipSuccess) return to_code(e);
        for (int it = 0; it <= h->max_refine; ++it) {
            e = sweeps(h, sweep_desc32(h, w, B, X, nrhs, it == 0), st);
            if (e == hipSuccess)
                e = timed(h, 3, 1, st, [&] { return btc::launch_residual(R, np, h->N, sweep_mc(BTC_OP_RESIDUAL, 0, np, nrhs), st); });
            if (e == hipSuccess) e = timed(h, 3, 2, st, [&] { return btc::launch_ir_check(I, 1, st); });
            if (e != hipSuccess) return to_code(e);
        }
        if (!info) return BTC_OK;
    }
    unsigned long long v = 0;
    int rc = read_info(h, st, &v);
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

// Argument checks shared by btc_solve and btc_solve_noalloc (0: go on,
// 1: nothing to do, < 0: error code).
int check_solve(btc_handle h, const double* B, double* X, int64_t nrhs) {
    if (!h) return -1;
    if (!B) return -2;
    if (!X) return -3;
    if (nrhs < 0) return -4;
    if (!h->factored) return -1;
    if (h->failed_known) return BTC_ERR_NOT_SPD;
    if (nrhs == 0) return 1;
    if (is_mixed(h->precision) && X == B) return -3;  // refinement reads b after x is written
    return 0;
}

void note_stream(btc_handle h, hipStream_t st) {
    for (hipStream_t s : h->streams)
        if (s == st) return;
    h->streams.push_back(st);
}

}  // namespace btc_host

extern "C" {

BTC_API int btc_solve(btc_handle h, const double* B, double* X, int64_t nrhs, void* stream,
                      btc_solve_info* info) {
    int rc = check_solve(h, B, X, nrhs);
    if (rc != 0) return rc < 0 ? rc : BTC_OK;
    hipStream_t st = (hipStream_t)stream;
    note_stream(h, st);
    // the handle's workspace serves solves on its stream, and solves on
    // another stream once the last solve that used it has finished; a solve
    // that would overlap one still running elsewhere gets a workspace of its
    // own for the duration of the call (stream-ordered)
    bool own = true;
    if (h->ws && h->ws_stream != st) {
        if (!h->ws_ev_valid) {
            own = false;
        } else {
            const hipError_t q = hipEventQuery(h->ws_ev);
            own = q == hipSuccess;
        }
    }
    if (own && nrhs > h->ws_m) {
        // growing the workspace synchronises with the streams that used it
        h->stream = st;
        rc = ensure_workspace(h, nrhs);
        if (rc != BTC_OK) return rc;
    }
    if (own) {
        const Workspace w = carve(h, h->ws_m);  // one layout per allocation
        h->stream = st;
        rc = solve_with(h, w, B, X, nrhs, st, info);
        if (!h->ws_ev && hipEventCreateWithFlags(&h->ws_ev, hipEventDisableTiming) != hipSuccess) h->ws_ev = nullptr;
        h->ws_stream = st;
        h->ws_ev_valid = h->ws_ev && hipEventRecord(h->ws_ev, st) == hipSuccess;
        return rc;
    }
    void* mem = nullptr;
    const Allocator a = current_allocator();
    hipError_t e = dev_alloc_async(a, &mem, workspace_bytes(h->N, h->n, h->precision, nrhs), st);
    if (e != hipSuccess) return to_code(e);
    const Workspace w = carve_at(mem, h->N, h->n, h->precision, nrhs);
    h->stream = st;
    rc = solve_with(h, w, B, X, nrhs, st, info);
    dev_free_async(a, mem, st);
    return rc;
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
    // wait for the handle's work on every stream it was used on
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (hipStream_t s : h->streams) (void)hipStreamSynchronize(s);
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
