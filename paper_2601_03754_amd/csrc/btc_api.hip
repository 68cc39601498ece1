// Host side of the libbtc C ABI (declared in include/btc.h): argument
// checking, the device memory of a handle, the level schedule and the
// launches, and the iterative-refinement driver of the mixed-precision path.
#include "btc.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cmath>
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
    if (opt && (opt->refine < BTC_REFINE_CLASSIC || opt->refine > BTC_REFINE_GMRES)) return -3;
    if (opt && (opt->gmres_m < 0 || opt->gmres_m > 200)) return -3;
    if (opt && (opt->strategy < BTC_STRATEGY_MULTISTAGE || opt->strategy > BTC_STRATEGY_PARTITION || opt->stages < 0))
        return -3;
    if (!out) return -4;
    int32_t strategy = opt ? opt->strategy : BTC_STRATEGY_MULTISTAGE, stages = opt ? opt->stages : 0;
    if (strategy == BTC_STRATEGY_AUTO) select_strategy(N, n, prec, &strategy, &stages);
    if (strategy == BTC_STRATEGY_KSTAGE && stages >= num_levels(N)) strategy = BTC_STRATEGY_MULTISTAGE;
    if (strategy == BTC_STRATEGY_KSTAGE && (prec != BTC_FP64 || n > 64)) return BTC_ERR_UNSUPPORTED;
    int64_t part_n1 = 0, part_nk = 0;
    if (strategy == BTC_STRATEGY_PARTITION &&
        (prec != BTC_FP64 || n > 64 || !partition_sizes(N, stages, part_n1, part_nk)))
        return BTC_ERR_UNSUPPORTED;
    *out = nullptr;
    btc_handle h = new (std::nothrow) btc_handle_s();
    if (!h) return BTC_ERR_OOM;
    h->N = N;
    h->n = n;
    h->precision = prec;
    h->max_refine = (opt && opt->max_refine > 0) ? opt->max_refine
                                                  : (is_bf16(prec) ? BTC_DEFAULT_MAX_REFINE_BF16 : BTC_DEFAULT_MAX_REFINE);
    h->tol = (opt && opt->tol > 0.0) ? opt->tol : BTC_DEFAULT_TOL;
    h->refine = opt ? opt->refine : BTC_REFINE_CLASSIC;
    h->gmres_m = (opt && opt->gmres_m > 0) ? opt->gmres_m : BTC_DEFAULT_GMRES_M;
    h->levels = num_levels(N);
    h->strategy = strategy;
    h->nd_levels = strategy == BTC_STRATEGY_KSTAGE ? stages : strategy == BTC_STRATEGY_PARTITION ? 0 : h->levels;
    if (strategy == BTC_STRATEGY_PARTITION) {
        h->parts = stages;
        h->part_n1 = part_n1;
        h->part_nk = part_nk;
    }
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
    if (opt && (opt->refine < BTC_REFINE_CLASSIC || opt->refine > BTC_REFINE_GMRES)) return -5;
    if (opt && (opt->gmres_m < 0 || opt->gmres_m > 200)) return -5;
    if (opt && (opt->strategy < BTC_STRATEGY_MULTISTAGE || opt->strategy > BTC_STRATEGY_PARTITION || opt->stages < 0))
        return -5;
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
    info->inner = 0;
    info->pad = 0;
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
int solve_gmres(btc_handle h, const Workspace& w, const double* B, double* X, int64_t m, hipStream_t st,
                btc_solve_info* info);

int solve_with(btc_handle h, const Workspace& w, const double* B, double* X, int64_t nrhs, hipStream_t st,
               btc_solve_info* info) {
    const bool mixed = is_mixed(h->precision);
    if (mixed && h->refine == BTC_REFINE_GMRES) return solve_gmres(h, w, B, X, nrhs, st, info);
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
        // A caller that asks for the outcome waits for the solve anyway: then
        // every round after the first correction is enqueued only if the
        // refinement has not stopped yet (one small read per round), instead
        // of launches that would exit at once.
        for (int it = 0; it <= h->max_refine; ++it) {
            e = sweeps(h, sweep_desc32(h, w, B, X, nrhs, it == 0), st);
            if (e == hipSuccess)
                e = timed(h, 3, 1, st, [&] { return btc::launch_residual(R, np, h->N, sweep_mc(BTC_OP_RESIDUAL, 0, np, nrhs), st); });
            if (e == hipSuccess) e = timed(h, 3, 2, st, [&] { return btc::launch_ir_check(I, 1, st); });
            if (e != hipSuccess) return to_code(e);
            if (info && it >= 1 && it < h->max_refine) {
                int32_t done = 0;
                e = hipMemcpyAsync(&done, &w.ir->done, sizeof(done), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return to_code(e);
                if (done) break;
            }
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
    info->inner = 0;
    info->pad = 0;
    return BTC_OK;
}

// Preconditioner of the GMRES correction: out = (L L^T)^{-1} in with the
// low-precision factor (FP64 in and out, FP32 sweeps in between).
hipError_t precond(btc_handle h, const Workspace& w, const double* in, double* out, int64_t m, hipStream_t st) {
    btc::SweepDesc<float> d = sweep_desc32(h, w, in, out, m, true);
    d.skip = nullptr;
    return sweeps(h, d, st);
}

// out = Psi x in FP64 (the residual kernels with a zero right-hand side,
// negated).
hipError_t matvec(btc_handle h, const Workspace& w, const double* zero, const double* x, double* out, int64_t m,
                  hipStream_t st) {
    const int np = btc::padded_block((int)h->n);
    btc::Launch<btc::ResidualDesc> R{};
    R.single = residual_desc(h, w, zero, x, m, false);
    R.single.state = nullptr;
    R.single.R64 = out;
    R.single.neg = 1;
    return btc::launch_residual(R, np, h->N, sweep_mc(BTC_OP_RESIDUAL, 0, np, m), st);
}

// Mixed-precision solve refined with GMRES corrections (BTC_REFINE_GMRES).
// x0 = (L L^T)^{-1} b; then per correction: r = b - Psi x (FP64, with the
// convergence test of classic refinement), and d from at most gmres_m
// iterations of GMRES on (L L^T)^{-1} Psi d = (L L^T)^{-1} r starting from
// d = 0 (Arnoldi with two classical Gram-Schmidt passes per vector, Givens
// rotations on the host, one synchronisation per iteration); x += d.
// Columns of B are independent problems that share the kernels.
int solve_gmres(btc_handle h, const Workspace& w, const double* B, double* X, int64_t m, hipStream_t st,
                btc_solve_info* info) {
    const int64_t rows = h->N * h->n;
    const size_t vs = (size_t)rows * (size_t)m;
    const int K = h->gmres_m;
    const double tau = 1e-8;
    const size_t small = (size_t)(K + 2) * (size_t)m;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = al((size_t)(K + 1) * vs * 8) + 3 * al(vs * 8) +
                         al((size_t)btc::kGmresBlocks * small * 8) + 3 * al(small * 8);
    const Allocator a = current_allocator();
    void* mem = nullptr;
    hipError_t e = dev_alloc_async(a, &mem, bytes, st);
    if (e != hipSuccess) return to_code(e);
    char* p = (char*)mem;
    auto take = [&](size_t b) { char* q = p; p += al(b); return (double*)q; };
    double* V = take((size_t)(K + 1) * vs * 8);
    double* z = take(vs * 8);
    double* r = take(vs * 8);
    double* zero = take(vs * 8);
    double* part = take((size_t)btc::kGmresBlocks * small * 8);
    double* hd = take(small * 8);
    double* h2d = take(small * 8);
    double* sd = take(small * 8);
    int rc = BTC_OK;
    int inner = 0;
    std::vector<double> H((size_t)(K + 1) * K * m), cs((size_t)K * m), sn((size_t)K * m), g((size_t)(K + 1) * m);
    std::vector<double> hv(small), h2v(small), sv(small), y((size_t)K * m);
    std::vector<int> kq((size_t)m);
    btc::Launch<btc::IrDesc> I{};
    I.single = ir_desc(h, w, m, h->tol, 1 + h->max_refine);
    btc::Launch<btc::ResidualDesc> Rs{};
    Rs.single = residual_desc(h, w, B, X, m, false);
    Rs.single.state = nullptr;
    Rs.single.R64 = r;
    const int np = btc::padded_block((int)h->n);
    auto fail = [&](hipError_t err) {
        rc = to_code(err);
        return rc;
    };
    e = btc::launch_fill(zero, 0.0, (int64_t)vs, st);
    if (e == hipSuccess) e = btc::launch_ir_init(I, 1, st);
    if (e == hipSuccess) {
        btc::SweepDesc<float> d = sweep_desc32(h, w, B, X, m, true);  // x0 = (L L^T)^{-1} b into X
        d.skip = nullptr;
        e = sweeps(h, d, st);
    }
    if (e != hipSuccess) {
        fail(e);
        dev_free_async(a, mem, st);
        return rc;
    }
    btc::IrState s{};
    for (int it = 0; it <= h->max_refine + 1 && rc == BTC_OK; ++it) {
        // residual of the current iterate and the convergence test
        e = btc::launch_residual(Rs, np, h->N, sweep_mc(BTC_OP_RESIDUAL, 0, np, m), st);
        if (e == hipSuccess) e = btc::launch_ir_check(I, 1, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&s, w.ir, sizeof(s), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            fail(e);
            break;
        }
        if (s.done) break;
        // GMRES on the preconditioned correction equation, d0 = 0
        e = precond(h, w, r, z, m, st);
        if (e == hipSuccess) e = btc::launch_gmres_dots(V, 0, z, true, rows, m, part, hd, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hv.data(), hd, (size_t)m * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            fail(e);
            break;
        }
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        std::vector<double> beta((size_t)m);
        for (int q = 0; q < m; ++q) {
            beta[q] = sqrt(hv[q]);
            g[(size_t)q * (K + 1)] = beta[q];
            sv[q] = beta[q] > 0.0 ? 1.0 / beta[q] : 0.0;
            kq[q] = beta[q] > 0.0 ? -1 : 0;  // -1: still iterating
        }
        e = hipMemcpyAsync(sd, sv.data(), (size_t)m * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = btc::launch_gmres_scale(z, sd, V, rows, m, st);
        int j = 0;
        for (; j < K && e == hipSuccess; ++j) {
            bool any = false;
            for (int q = 0; q < m; ++q) any = any || kq[q] < 0;
            if (!any) break;
            double* vj = V + (size_t)j * vs;
            e = matvec(h, w, zero, vj, r, m, st);
            if (e == hipSuccess) e = precond(h, w, r, z, m, st);
            // two classical Gram-Schmidt passes, then the norm
            if (e == hipSuccess) e = btc::launch_gmres_dots(V, j + 1, z, false, rows, m, part, hd, st);
            if (e == hipSuccess) e = btc::launch_gmres_update(V, j + 1, hd, z, rows, m, st);
            if (e == hipSuccess) e = btc::launch_gmres_dots(V, j + 1, z, true, rows, m, part, h2d, st);
            if (e == hipSuccess) e = btc::launch_gmres_update(V, j + 1, h2d, z, rows, m, st);
            if (e == hipSuccess) e = btc::launch_gmres_dots(V, 0, z, true, rows, m, part, sd, st);
            if (e == hipSuccess) e = hipMemcpyAsync(hv.data(), hd, (size_t)(j + 1) * m * 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(h2v.data(), h2d, (size_t)(j + 1) * m * 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(sv.data(), sd, (size_t)m * 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) break;
            ++inner;
            for (int q = 0; q < m; ++q) {
                double* Hq = &H[(size_t)q * (K + 1) * K];  // column-major (K+1) x K
                auto Hat = [&](int row, int col) -> double& { return Hq[(size_t)col * (K + 1) + row]; };
                for (int i = 0; i <= j; ++i) Hat(i, j) = hv[(size_t)i * m + q] + h2v[(size_t)i * m + q];
                const double hn = sqrt(fmax(sv[q], 0.0));
                Hat(j + 1, j) = hn;
                // earlier rotations, then a new one that zeroes H(j+1, j)
                for (int i = 0; i < j; ++i) {
                    const double c = cs[(size_t)q * K + i], sgn = sn[(size_t)q * K + i];
                    const double t = c * Hat(i, j) + sgn * Hat(i + 1, j);
                    Hat(i + 1, j) = -sgn * Hat(i, j) + c * Hat(i + 1, j);
                    Hat(i, j) = t;
                }
                const double a0 = Hat(j, j), b0 = Hat(j + 1, j);
                const double rr = hypot(a0, b0);
                const double c = rr > 0.0 ? a0 / rr : 1.0, sgn = rr > 0.0 ? b0 / rr : 0.0;
                cs[(size_t)q * K + j] = c;
                sn[(size_t)q * K + j] = sgn;
                Hat(j, j) = rr;
                Hat(j + 1, j) = 0.0;
                double* gq = &g[(size_t)q * (K + 1)];
                gq[j + 1] = -sgn * gq[j];
                gq[j] = c * gq[j];
                if (kq[q] < 0 && (fabs(gq[j + 1]) <= tau * beta[q] || hn == 0.0 || j + 1 == K)) kq[q] = j + 1;
                // next basis vector (zero for a column that has stopped)
                sv[q] = (kq[q] < 0 && hn > 0.0) ? 1.0 / hn : 0.0;
            }
            e = hipMemcpyAsync(sd, sv.data(), (size_t)m * 8, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = btc::launch_gmres_scale(z, sd, V + (size_t)(j + 1) * vs, rows, m, st);
        }
        if (e != hipSuccess) {
            fail(e);
            break;
        }
        // y from the triangular system of each column's first kq iterations
        std::fill(y.begin(), y.end(), 0.0);
        int kmax = 0;
        for (int q = 0; q < m; ++q) {
            const int k = kq[q] < 0 ? j : kq[q];
            kmax = std::max(kmax, k);
            const double* Hq = &H[(size_t)q * (K + 1) * K];
            const double* gq = &g[(size_t)q * (K + 1)];
            for (int i = k - 1; i >= 0; --i) {
                double t = gq[i];
                for (int c = i + 1; c < k; ++c) t -= Hq[(size_t)c * (K + 1) + i] * y[(size_t)c * m + q];
                const double dgn = Hq[(size_t)i * (K + 1) + i];
                y[(size_t)i * m + q] = dgn != 0.0 ? t / dgn : 0.0;
            }
        }
        e = hipMemcpyAsync(hd, y.data(), (size_t)std::max(kmax, 1) * m * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && kmax > 0) e = btc::launch_gmres_combine(V, kmax, hd, X, rows, m, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vectors are reused next round
        if (e != hipSuccess) fail(e);
    }
    if (rc == BTC_OK && info) {
        unsigned long long v = 0;
        rc = read_info(h, st, &v);
        if (rc == BTC_OK && v != kInfoOk) {
            h->failed_known = true;
            rc = BTC_ERR_NOT_SPD;
        }
        if (rc == BTC_OK) {
            e = hipMemcpy(&s, w.ir, sizeof(s), hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = to_code(e);
        }
        if (rc == BTC_OK) {
            info->steps = s.steps - 1;
            info->converged = s.converged;
            info->relres = s.relres;
            info->inner = inner;
            info->pad = 0;
        }
    }
    dev_free_async(a, mem, st);
    return rc;
}

// Argument checks shared by the solve entry points (0: go on,
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
        if (h->strategy == BTC_STRATEGY_PARTITION) {
            // stored by original block: chunk blocks (R to the next block or
            // the right separator, T to the left separator), separators (R'
            // to the next separator; their T slot holds a chunk's fill)
            for (int64_t i = 1; i <= N; ++i) {
                bool sep = false, last = false, has_l = false;
                int64_t j = 0;  // chunk of i, or separator index
                if (i <= h->part_n1) {
                    j = 0;
                    last = i == h->part_n1;
                } else {
                    const int64_t off = i - h->part_n1 - 1, per = h->part_nk + 1;
                    j = off / per + 1;
                    sep = off % per == 0;
                    last = !sep && off % per == h->part_nk;
                    has_l = !sep;
                }
                bool present = a == 0;
                if (a == 1) present = sep ? j + 1 < h->parts : (!last || j + 1 < h->parts);
                if (a == 2) present = has_l;
                double* dst = outs[a] + (size_t)(i - 1) * nn;
                if (present)
                    memcpy(dst, tmp.data() + (size_t)(i - 1) * nn, nn * sizeof(double));
                else
                    memset(dst, 0, nn * sizeof(double));
            }
            continue;
        }
        for (int64_t i = 1; i <= N; ++i) {
            const int l = btc::level_of(i);
            const int64_t s = (int64_t)1 << l;
            bool present = (a == 0) || (a == 1 && i + s <= N) || (a == 2 && i > s);
            if (l >= h->nd_levels) {
                // a block of the chain of a k-stage order: right slot = the
                // factor block at (next chain block, i), no left block
                const int64_t sc = (int64_t)1 << h->nd_levels;
                present = (a == 0) || (a == 1 && i + sc <= N);
            }
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
