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

// ---------------------------------------------------------------------------
// GMRES vector kernels (FP64).  One workgroup of 256 threads per slice of
// rows; columns q of the m right-hand sides are independent.

constexpr int kGT = 256;

// Block-sum of `v` over the workgroup (fixed order); valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kGT / 64; ++k) t += red[k];
    return t;
}

// part[(b*(k+1) + i)*m + q]: workgroup b's share of dot (V_i or z, z) for column q.
__global__ __launch_bounds__(kGT) void k_gmres_dots(const double* __restrict__ V, int k, const double* __restrict__ z,
                                                    int self, int64_t rows, int m, double* __restrict__ part) {
    __shared__ double red[kGT / 64];
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < rows ? r0 + per : rows;
    const size_t vs = (size_t)rows * m;
    const int kk = k + (self ? 1 : 0);
    for (int i = 0; i < kk; ++i) {
        const double* a = i < k ? V + (size_t)i * vs : z;
        for (int q = 0; q < m; ++q) {
            double acc = 0.0;
            for (int64_t r = r0 + threadIdx.x; r < r1; r += kGT) {
                const size_t e = (size_t)r * m + q;
                acc = fma(a[e], z[e], acc);
            }
            const double t = block_sum(acc, red);
            if (threadIdx.x == 0) part[((size_t)blockIdx.x * (k + 1) + i) * m + q] = t;
        }
    }
}

// h[i*m + q] = sum over workgroups b (in order) of part[(b*(k+1) + i)*m + q].
__global__ void k_gmres_dots_fin(const double* __restrict__ part, int nb, int k, int self, int m,
                                 double* __restrict__ h) {
    const int kk = k + (self ? 1 : 0);
    for (int e = threadIdx.x; e < kk * m; e += blockDim.x) {
        const int i = e / m, q = e % m;
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += part[((size_t)b * (k + 1) + i) * m + q];
        h[(size_t)i * m + q] = t;
    }
}

__global__ __launch_bounds__(kGT) void k_gmres_update(const double* __restrict__ V, int k,
                                                      const double* __restrict__ h, double* __restrict__ z,
                                                      int64_t rows, int m) {
    const size_t total = (size_t)rows * m, vs = total;
    for (size_t e = (size_t)blockIdx.x * kGT + threadIdx.x; e < total; e += (size_t)gridDim.x * kGT) {
        const int q = (int)(e % m);
        double acc = z[e];
        for (int i = 0; i < k; ++i) acc = fma(-h[(size_t)i * m + q], V[(size_t)i * vs + e], acc);
        z[e] = acc;
    }
}

__global__ __launch_bounds__(kGT) void k_gmres_scale(const double* __restrict__ src, const double* __restrict__ sc,
                                                     double* __restrict__ dst, int64_t rows, int m) {
    const size_t total = (size_t)rows * m;
    for (size_t e = (size_t)blockIdx.x * kGT + threadIdx.x; e < total; e += (size_t)gridDim.x * kGT)
        dst[e] = src[e] * sc[e % m];
}

__global__ __launch_bounds__(kGT) void k_gmres_combine(const double* __restrict__ V, int k,
                                                       const double* __restrict__ y, double* __restrict__ x,
                                                       int64_t rows, int m) {
    const size_t total = (size_t)rows * m, vs = total;
    for (size_t e = (size_t)blockIdx.x * kGT + threadIdx.x; e < total; e += (size_t)gridDim.x * kGT) {
        const int q = (int)(e % m);
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(y[(size_t)j * m + q], V[(size_t)j * vs + e], acc);
        x[e] += acc;
    }
}

__global__ __launch_bounds__(kGT) void k_fill(double* __restrict__ x, double v, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * kGT + threadIdx.x; e < count; e += (int64_t)gridDim.x * kGT) x[e] = v;
}

unsigned grid_for(int64_t elems) {
    const int64_t g = (elems + kGT - 1) / kGT;
    return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_gmres_dots(const double* V, int k, const double* z, bool self, int64_t rows, int m, double* part,
                             double* h, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_dots, dim3(kGmresBlocks), dim3(kGT), 0, st, V, k, z, self ? 1 : 0, rows, m, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gmres_dots_fin, dim3(1), dim3(kGT), 0, st, part, kGmresBlocks, k, self ? 1 : 0, m, h);
    return hipGetLastError();
}

hipError_t launch_gmres_update(const double* V, int k, const double* h, double* z, int64_t rows, int m,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_update, dim3(grid_for(rows * m)), dim3(kGT), 0, st, V, k, h, z, rows, m);
    return hipGetLastError();
}

hipError_t launch_gmres_scale(const double* src, const double* s, double* dst, int64_t rows, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_scale, dim3(grid_for(rows * m)), dim3(kGT), 0, st, src, s, dst, rows, m);
    return hipGetLastError();
}

hipError_t launch_gmres_combine(const double* V, int k, const double* y, double* x, int64_t rows, int m,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_gmres_combine, dim3(grid_for(rows * m)), dim3(kGT), 0, st, V, k, y, x, rows, m);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, double v, int64_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(kGT), 0, st, x, v, count);
    return hipGetLastError();
}

hipError_t launch_ir_check(const Launch<IrDesc>& p, int64_t items, hipStream_t st) {
    hipLaunchKernelGGL(k_ir_check, dim3((unsigned)items), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_ir_init(const Launch<IrDesc>& p, int64_t items, hipStream_t st) {
    hipLaunchKernelGGL(k_ir_init, dim3((unsigned)items), dim3(64), 0, st, p);
    return hipGetLastError();
}

}  // namespace btc
