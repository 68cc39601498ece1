// Iterative-refinement control of the mixed-precision solve: set-up of the
// refinement state and the convergence test over the per-block-row partial
// norms that the residual kernel leaves (reduced in a fixed order, so the
// decision is deterministic).
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {
namespace {

constexpr unsigned long long kInfoOk = ~0ull;

// Reduce the partial norms of one instance in a fixed order, form
// max_q ||r_q||/||b_q|| and advance its refinement state: converged when
// <= tol, stalled when the residual fell by less than 2x in the last step,
// done when either holds or the step budget is spent.
__global__ __launch_bounds__(256) void k_ir_check(Launch<IrDesc> L) {
    __shared__ double red[2][256];
    IrDesc P;
    int lvl_unused;
    int64_t k_unused;
    fetch_item(L, P, lvl_unused, k_unused);
    IrState* st = P.state;
    if (st->done) return;
    const int64_t N = P.N;
    const int m = P.m;
    double worst = 0.0;
    for (int q = 0; q < m; ++q) {
        double rr = 0.0, bb = 0.0;
        for (int64_t i = threadIdx.x; i < N; i += 256) {
            rr += P.part[((size_t)i * m + q) * 2 + 0];
            bb += P.part[((size_t)i * m + q) * 2 + 1];
        }
        red[0][threadIdx.x] = rr;
        red[1][threadIdx.x] = bb;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                red[0][threadIdx.x] += red[0][threadIdx.x + h];
                red[1][threadIdx.x] += red[1][threadIdx.x + h];
            }
            __syncthreads();
        }
        const double rn = sqrt(red[0][0]), bn = sqrt(red[1][0]);
        const double rel = (bn > 0.0) ? rn / bn : rn;
        worst = fmax(worst, rel);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->steps += 1;
        st->relres = worst;
        if (!(worst == worst)) {  // NaN: give up
            st->done = 1;
        } else if (worst <= st->tol) {
            st->converged = 1;
            st->done = 1;
        } else if (st->steps >= st->max_steps) {
            st->done = 1;
        } else if (worst > 0.5 * st->prev) {
            st->stalled = 1;
            st->done = 1;
        }
        st->prev = worst;
    }
}

// Reset the refinement state of one instance.
__global__ void k_ir_init(Launch<IrDesc> L) {
    IrDesc P;
    int lvl_unused;
    int64_t k_unused;
    fetch_item(L, P, lvl_unused, k_unused);
    if (threadIdx.x == 0) {
        IrState* st = P.state;
        st->done = 0;
        st->steps = 0;
        st->converged = 0;
        st->stalled = 0;
        st->relres = -1.0;
        st->prev = __builtin_inf();
        st->tol = P.tol;
        st->max_steps = P.max_steps;
    }
}

}  // namespace

hipError_t launch_ir_check(const Launch<IrDesc>& p, int64_t items, hipStream_t st) {
    hipLaunchKernelGGL(k_ir_check, dim3((unsigned)items), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_ir_init(const Launch<IrDesc>& p, int64_t items, hipStream_t st) {
    hipLaunchKernelGGL(k_ir_init, dim3((unsigned)items), dim3(64), 0, st, p);
    return hipGetLastError();
}

}  // namespace btc
