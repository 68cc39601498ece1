// Level sweeps of the solve (section "Cholesky Solve", Algorithm 6), templated
// on the storage type of the factor (FP64 for the plain path, FP32 for the
// low-precision solves of iterative refinement), plus the FP64 residual and
// the refinement control used by the mixed-precision path.
//
// Sweeps: one workgroup per node; wavefront w handles right-hand-side columns
// q = w, w + nwaves, ...; lane r owns row r of the block.
//   forward (levels ascending): y_i = L_ii^{-1}(b_i - pulled contributions),
//     u_i = R_i y_i (left for the right neighbour), v_i = T_i^T y_i (left for
//     the left neighbour).  Rather than two nodes subtracting into the same y
//     concurrently, node i pulls the u/v vectors that its children at every
//     lower level left for it, in a fixed order (deterministic).
//   backward (levels descending): x_i = L_ii^{-T}(y_i - R_i^T x_{i+s} - T_i x_{i-s}).
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {
namespace {

constexpr unsigned long long kInfoOk = ~0ull;

template <int NP>
struct SweepCfg {
    static constexpr int NT = (NP >= 64) ? 256 : (NP >= 32 ? 128 : 64);
};

__device__ __forceinline__ double bcast(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <class T>
__device__ __forceinline__ bool skip_launch(const SweepDesc<T>& P) {
    if (*P.info != kInfoOk) return true;
    if (P.skip && *P.skip) return true;
    return false;
}

template <int NP, int NT, class T>
__global__ __launch_bounds__(NT) void k_forward(Launch<SweepDesc<T>> L) {
    constexpr int LD = NP + 1;
    constexpr int NW = NT / kWave;
    __shared__ T sL[NP * LD];
    __shared__ T sR[NP * LD];
    __shared__ T sT[NP * LD];
    __shared__ T invd[NP];
    __shared__ T sy[NW][NP];

    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_launch(P)) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);

    {
        Stage<NP, NT, T> a, b, c;
        a.fetch(P.Ld + (size_t)pi * nn, n, true, 1.0, tid);
        if (has_r) b.fetch(P.Rb + (size_t)pi * nn, n, false, 0.0, tid);
        if (has_l) c.fetch(P.Tb + (size_t)pi * nn, n, false, 0.0, tid);
        a.put(sL, tid);
        if (has_r) b.put(sR, tid);
        if (has_l) c.put(sT, tid);
    }
    __syncthreads();
    if (tid < NP) invd[tid] = T(1) / sL[tid * LD + tid];
    __syncthreads();

    for (int q = w; q < m; q += NW) {
        // right-hand side minus the contributions of the children at every
        // lower level, gathered eight levels at a time so the loads overlap
        T acc = T(0);
        if (lane < n) {
            const size_t bidx = ((size_t)(i - 1) * n + lane) * m + q;
            acc = P.B64 ? (T)P.B64[bidx] : P.B[bidx];
            for (int l0 = 0; l0 < lvl; l0 += 8) {
                T pu[8], pv[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int l2 = l0 + k;
                    const int64_t s2 = (int64_t)1 << l2;
                    pu[k] = (l2 < lvl) ? P.U[(size_t)perm_pos(N, l2, i - s2) * nm + (size_t)lane * m + q] : T(0);
                    pv[k] = (l2 < lvl && i + s2 <= N)
                                ? P.V[(size_t)perm_pos(N, l2, i + s2) * nm + (size_t)lane * m + q]
                                : T(0);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) acc -= pu[k] + pv[k];
            }
        }
        // y = L^{-1} acc: column sweep, pivot broadcast by readlane
#pragma unroll 8
        for (int j = 0; j < NP; ++j) {
            const T yj = bcast(acc, j) * invd[j];
            if (lane == j) acc = yj;
            if (lane > j && lane < NP) acc = fma(-sL[lane * LD + j], yj, acc);
        }
        if (lane < NP) sy[w][lane] = acc;
        wave_lds_sync();
        if (lane < n) {
            P.Y[(size_t)pi * nm + (size_t)lane * m + q] = acc;
            if (has_r) {
                T u = T(0);
                for (int c = 0; c < n; ++c) u = fma(sR[lane * LD + c], sy[w][c], u);
                P.U[(size_t)pi * nm + (size_t)lane * m + q] = u;
            }
            if (has_l) {
                T v = T(0);
                for (int c = 0; c < n; ++c) v = fma(sT[c * LD + lane], sy[w][c], v);
                P.V[(size_t)pi * nm + (size_t)lane * m + q] = v;
            }
        }
        wave_lds_sync();
    }
}

template <int NP, int NT, class T>
__global__ __launch_bounds__(NT) void k_backward(Launch<SweepDesc<T>> L) {
    constexpr int LD = NP + 1;
    constexpr int NW = NT / kWave;
    __shared__ T sL[NP * LD];
    __shared__ T sR[NP * LD];
    __shared__ T sT[NP * LD];
    __shared__ T invd[NP];
    __shared__ T sxr[NW][NP];
    __shared__ T sxl[NW][NP];

    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_launch(P)) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);

    {
        Stage<NP, NT, T> a, b, c;
        a.fetch(P.Ld + (size_t)pi * nn, n, true, 1.0, tid);
        if (has_r) b.fetch(P.Rb + (size_t)pi * nn, n, false, 0.0, tid);
        if (has_l) c.fetch(P.Tb + (size_t)pi * nn, n, false, 0.0, tid);
        a.put(sL, tid);
        if (has_r) b.put(sR, tid);
        if (has_l) c.put(sT, tid);
    }
    __syncthreads();
    if (tid < NP) invd[tid] = T(1) / sL[tid * LD + tid];
    __syncthreads();

    for (int q = w; q < m; q += NW) {
        T acc = T(0);
        if (lane < NP) {
            sxr[w][lane] = (has_r && lane < n) ? P.X[((size_t)(i + s - 1) * n + lane) * m + q] : T(0);
            sxl[w][lane] = (has_l && lane < n) ? P.X[((size_t)(i - s - 1) * n + lane) * m + q] : T(0);
        }
        wave_lds_sync();
        if (lane < n) {
            acc = P.Y[(size_t)pi * nm + (size_t)lane * m + q];
            if (has_r)
                for (int c = 0; c < n; ++c) acc = fma(-sR[c * LD + lane], sxr[w][c], acc);
            if (has_l)
                for (int c = 0; c < n; ++c) acc = fma(-sT[lane * LD + c], sxl[w][c], acc);
        }
        // x = L^{-T} acc: backward column sweep
#pragma unroll 8
        for (int j = NP - 1; j >= 0; --j) {
            const T xj = bcast(acc, j) * invd[j];
            if (lane == j) acc = xj;
            if (lane < j) acc = fma(-sL[j * LD + lane], xj, acc);
        }
        if (lane < n) {
            const size_t idx = ((size_t)(i - 1) * n + lane) * m + q;
            P.X[idx] = acc;
            if (P.X64) P.X64[idx] = P.first ? (double)acc : P.X64[idx] + (double)acc;
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Large blocks (padded 96 and 128): lane owns rows lane and lane + 64; only
// L_ii is staged in LDS, R_i and T_i are streamed from global memory (the
// product with T_i^T reads whole rows across the lanes, the one with R_i one
// row per lane, which stays in the vector cache).

template <int NP, class T>
__device__ __forceinline__ void stage_L(T* __restrict__ sL, const T* __restrict__ src, int n, int tid, int nt) {
    constexpr int LD = NP + 1;
    constexpr int CH = 8;
    for (int base = 0; base < NP * NP; base += nt * CH) {
        T v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = base + tid + nt * u, r = e / NP, c = e % NP;
            T x = (r == c) ? T(1) : T(0);
            if (e < NP * NP && r < n && c <= r) x = src[(size_t)r * n + c];
            v[u] = x;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = base + tid + nt * u;
            if (e < NP * NP) sL[(e / NP) * LD + e % NP] = v[u];
        }
    }
}

template <int NP, int NT, class T>
__global__ __launch_bounds__(NT) void k_forward_big(Launch<SweepDesc<T>> L) {
    constexpr int LD = NP + 1;
    constexpr int NW = NT / kWave;
    constexpr int RPL = (NP + kWave - 1) / kWave;
    __shared__ T sL[NP * LD];
    __shared__ T invd[NP];
    __shared__ T sy[NW][RPL * kWave];
    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_launch(P)) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);
    stage_L<NP, T>(sL, P.Ld + (size_t)pi * nn, n, tid, NT);
    __syncthreads();
    if (tid < NP) invd[tid] = T(1) / sL[tid * LD + tid];
    __syncthreads();
    const T* Rg = P.Rb + (size_t)pi * nn;
    const T* Tg = P.Tb + (size_t)pi * nn;
    for (int q = w; q < m; q += NW) {
        T acc[RPL];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int row = lane + kWave * rr;
            T a = T(0);
            if (row < n) {
                const size_t bidx = ((size_t)(i - 1) * n + row) * m + q;
                a = P.B64 ? (T)P.B64[bidx] : P.B[bidx];
                for (int l2 = 0; l2 < lvl; ++l2) {
                    const int64_t s2 = (int64_t)1 << l2;
                    a -= P.U[(size_t)perm_pos(N, l2, i - s2) * nm + (size_t)row * m + q];
                    if (i + s2 <= N) a -= P.V[(size_t)perm_pos(N, l2, i + s2) * nm + (size_t)row * m + q];
                }
            }
            acc[rr] = a;
        }
        for (int j = 0; j < NP; ++j) {
            const int jr = j / kWave;
            T piv = acc[0];
#pragma unroll
            for (int rr = 1; rr < RPL; ++rr) piv = (jr == rr) ? acc[rr] : piv;
            const T yj = bcast(piv, j % kWave) * invd[j];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                const int row = lane + kWave * rr;
                if (row == j) acc[rr] = yj;
                if (row > j && row < NP) acc[rr] = fma(-sL[row * LD + j], yj, acc[rr]);
            }
        }
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) sy[w][lane + kWave * rr] = acc[rr];
        wave_lds_sync();
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int row = lane + kWave * rr;
            if (row >= n) continue;
            P.Y[(size_t)pi * nm + (size_t)row * m + q] = acc[rr];
            if (has_r) {
                T u = T(0);
                for (int c = 0; c < n; ++c) u = fma(Rg[(size_t)row * n + c], sy[w][c], u);
                P.U[(size_t)pi * nm + (size_t)row * m + q] = u;
            }
            if (has_l) {
                T v = T(0);
                for (int c = 0; c < n; ++c) v = fma(Tg[(size_t)c * n + row], sy[w][c], v);
                P.V[(size_t)pi * nm + (size_t)row * m + q] = v;
            }
        }
        wave_lds_sync();
    }
}

template <int NP, int NT, class T>
__global__ __launch_bounds__(NT) void k_backward_big(Launch<SweepDesc<T>> L) {
    constexpr int LD = NP + 1;
    constexpr int NW = NT / kWave;
    constexpr int RPL = (NP + kWave - 1) / kWave;
    __shared__ T sL[NP * LD];
    __shared__ T invd[NP];
    __shared__ T sxr[NW][RPL * kWave];
    __shared__ T sxl[NW][RPL * kWave];
    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_launch(P)) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);
    stage_L<NP, T>(sL, P.Ld + (size_t)pi * nn, n, tid, NT);
    __syncthreads();
    if (tid < NP) invd[tid] = T(1) / sL[tid * LD + tid];
    __syncthreads();
    const T* Rg = P.Rb + (size_t)pi * nn;
    const T* Tg = P.Tb + (size_t)pi * nn;
    for (int q = w; q < m; q += NW) {
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int row = lane + kWave * rr;
            sxr[w][row] = (has_r && row < n) ? P.X[((size_t)(i + s - 1) * n + row) * m + q] : T(0);
            sxl[w][row] = (has_l && row < n) ? P.X[((size_t)(i - s - 1) * n + row) * m + q] : T(0);
        }
        wave_lds_sync();
        T acc[RPL];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int row = lane + kWave * rr;
            T a = T(0);
            if (row < n) {
                a = P.Y[(size_t)pi * nm + (size_t)row * m + q];
                if (has_r)
                    for (int c = 0; c < n; ++c) a = fma(-Rg[(size_t)c * n + row], sxr[w][c], a);
                if (has_l)
                    for (int c = 0; c < n; ++c) a = fma(-Tg[(size_t)row * n + c], sxl[w][c], a);
            }
            acc[rr] = a;
        }
        for (int j = NP - 1; j >= 0; --j) {
            const int jr = j / kWave;
            T piv = acc[0];
#pragma unroll
            for (int rr = 1; rr < RPL; ++rr) piv = (jr == rr) ? acc[rr] : piv;
            const T xj = bcast(piv, j % kWave) * invd[j];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                const int row = lane + kWave * rr;
                if (row == j) acc[rr] = xj;
                if (row < j) acc[rr] = fma(-sL[j * LD + row], xj, acc[rr]);
            }
        }
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int row = lane + kWave * rr;
            if (row < n) {
                const size_t idx = ((size_t)(i - 1) * n + row) * m + q;
                P.X[idx] = acc[rr];
                if (P.X64) P.X64[idx] = P.first ? (double)acc[rr] : P.X64[idx] + (double)acc[rr];
            }
        }
        wave_lds_sync();
    }
}

template <int NP, class T>
hipError_t launch_sweep_np(const Launch<SweepDesc<T>>& p, int64_t items, bool backward, hipStream_t st) {
    constexpr int NT = SweepCfg<NP>::NT;
    if (backward)
        hipLaunchKernelGGL((k_backward<NP, NT, T>), dim3((unsigned)items), dim3(NT), 0, st, p);
    else
        hipLaunchKernelGGL((k_forward<NP, NT, T>), dim3((unsigned)items), dim3(NT), 0, st, p);
    return hipGetLastError();
}

template <class T>
hipError_t launch_sweep_t(const Launch<SweepDesc<T>>& p, int np, int64_t items, bool backward, hipStream_t st) {
    switch (np) {
        case 8: return launch_sweep_np<8, T>(p, items, backward, st);
        case 16: return launch_sweep_np<16, T>(p, items, backward, st);
        case 32: return launch_sweep_np<32, T>(p, items, backward, st);
        case 64: return launch_sweep_np<64, T>(p, items, backward, st);
        case 96:
        case 128: {
            const dim3 g((unsigned)items);
            if (np == 96) {
                if (backward)
                    hipLaunchKernelGGL((k_backward_big<96, 256, T>), g, dim3(256), 0, st, p);
                else
                    hipLaunchKernelGGL((k_forward_big<96, 256, T>), g, dim3(256), 0, st, p);
            } else {
                if (backward)
                    hipLaunchKernelGGL((k_backward_big<128, 256, T>), g, dim3(256), 0, st, p);
                else
                    hipLaunchKernelGGL((k_forward_big<128, 256, T>), g, dim3(256), 0, st, p);
            }
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// FP64 residual r = b - Psi x, one workgroup (one wavefront) per block row i,
// lane r owning row r: r_i = b_i - E_{i-1} x_{i-1} - D_i x_i - E_i^T x_{i+1}
// with D_i symmetric from its lower triangle.  Writes r rounded to FP32 (the
// right-hand side of the next low-precision solve) and the per-row-block
// squared column norms of r and b, reduced later in a fixed order.

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_residual(Launch<ResidualDesc> L) {
    constexpr int LD = NP + 1;
    constexpr int NW = NT / kWave;
    __shared__ double sDg[NP * LD];
    __shared__ double sEl[NP * LD];
    __shared__ double sEr[NP * LD];
    __shared__ double sx[NW][3][kWave];

    ResidualDesc P;
    int lvl_unused;
    int64_t row;
    fetch_item(L, P, lvl_unused, row);
    if (P.state && P.state->done) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n;
    const int64_t i = row + 1;
    const bool lft = i > 1, rgt = i < N;
    {
        Stage<NP, NT> a, b, c;
        a.fetch(P.A_diag + (size_t)(i - 1) * nn, n, true, 0.0, tid);
        if (lft) b.fetch(P.A_off + (size_t)(i - 2) * nn, n, false, 0.0, tid);
        if (rgt) c.fetch(P.A_off + (size_t)(i - 1) * nn, n, false, 0.0, tid);
        a.put(sDg, tid);
        if (lft) b.put(sEl, tid);
        if (rgt) c.put(sEr, tid);
    }
    __syncthreads();
    for (int q = w; q < m; q += NW) {
        const bool act = lane < n;
        sx[w][0][lane] = (act && lft) ? P.X[((size_t)(i - 2) * n + lane) * m + q] : 0.0;
        sx[w][1][lane] = act ? P.X[((size_t)(i - 1) * n + lane) * m + q] : 0.0;
        sx[w][2][lane] = (act && rgt) ? P.X[((size_t)i * n + lane) * m + q] : 0.0;
        wave_lds_sync();
        double b = 0.0, acc = 0.0;
        if (act) {
            b = P.B[((size_t)(i - 1) * n + lane) * m + q];
            acc = b;
            for (int c = 0; c < n; ++c) {
                const double dv = (c <= lane) ? sDg[lane * LD + c] : sDg[c * LD + lane];
                acc = fma(-dv, sx[w][1][c], acc);
            }
            if (lft)
                for (int c = 0; c < n; ++c) acc = fma(-sEl[lane * LD + c], sx[w][0][c], acc);
            if (rgt)
                for (int c = 0; c < n; ++c) acc = fma(-sEr[c * LD + lane], sx[w][2][c], acc);
            if (P.R32) P.R32[((size_t)(i - 1) * n + lane) * m + q] = (float)acc;
        }
        double rr = acc * acc, bb = b * b;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rr += __shfl_xor(rr, off);
            bb += __shfl_xor(bb, off);
        }
        if (lane == 0) {
            P.part[((size_t)(i - 1) * m + q) * 2 + 0] = rr;
            P.part[((size_t)(i - 1) * m + q) * 2 + 1] = bb;
        }
        wave_lds_sync();
    }
}

// Residual for large blocks: lane owns rows lane and lane + 64; the blocks
// are read from global memory (column walks are coalesced across the lanes,
// row walks stay in the vector cache).
template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_residual_big(Launch<ResidualDesc> L) {
    constexpr int NW = NT / kWave;
    constexpr int RPL = (NP + kWave - 1) / kWave;
    __shared__ double sx[NW][3][RPL * kWave];
    ResidualDesc P;
    int lvl_unused;
    int64_t row0;
    fetch_item(L, P, lvl_unused, row0);
    if (P.state && P.state->done) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n;
    const int64_t i = row0 + 1;
    const bool lft = i > 1, rgt = i < N;
    const double* Dg = P.A_diag + (size_t)(i - 1) * nn;
    const double* El = lft ? P.A_off + (size_t)(i - 2) * nn : nullptr;
    const double* Er = rgt ? P.A_off + (size_t)(i - 1) * nn : nullptr;
    for (int q = w; q < m; q += NW) {
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
            const bool act = r < n;
            sx[w][0][r] = (act && lft) ? P.X[((size_t)(i - 2) * n + r) * m + q] : 0.0;
            sx[w][1][r] = act ? P.X[((size_t)(i - 1) * n + r) * m + q] : 0.0;
            sx[w][2][r] = (act && rgt) ? P.X[((size_t)i * n + r) * m + q] : 0.0;
        }
        wave_lds_sync();
        double rr2 = 0.0, bb2 = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
            if (r >= n) continue;
            const double b = P.B[((size_t)(i - 1) * n + r) * m + q];
            double acc = b;
            for (int c = 0; c <= r; ++c) acc = fma(-Dg[(size_t)r * n + c], sx[w][1][c], acc);
            for (int c = r + 1; c < n; ++c) acc = fma(-Dg[(size_t)c * n + r], sx[w][1][c], acc);
            if (lft)
                for (int c = 0; c < n; ++c) acc = fma(-El[(size_t)r * n + c], sx[w][0][c], acc);
            if (rgt)
                for (int c = 0; c < n; ++c) acc = fma(-Er[(size_t)c * n + r], sx[w][2][c], acc);
            if (P.R32) P.R32[((size_t)(i - 1) * n + r) * m + q] = (float)acc;
            rr2 += acc * acc;
            bb2 += b * b;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rr2 += __shfl_xor(rr2, off);
            bb2 += __shfl_xor(bb2, off);
        }
        if (lane == 0) {
            P.part[((size_t)(i - 1) * m + q) * 2 + 0] = rr2;
            P.part[((size_t)(i - 1) * m + q) * 2 + 1] = bb2;
        }
        wave_lds_sync();
    }
}

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

hipError_t launch_sweep(const Launch<SweepDesc<double>>& p, int np, int64_t items, bool backward, hipStream_t st) {
    return launch_sweep_t<double>(p, np, items, backward, st);
}

hipError_t launch_sweep(const Launch<SweepDesc<float>>& p, int np, int64_t items, bool backward, hipStream_t st) {
    return launch_sweep_t<float>(p, np, items, backward, st);
}

hipError_t launch_residual(const Launch<ResidualDesc>& p, int np, int64_t items, hipStream_t st) {
    const dim3 g((unsigned)items);
    switch (np) {
        case 8: hipLaunchKernelGGL((k_residual<8, SweepCfg<8>::NT>), g, dim3(SweepCfg<8>::NT), 0, st, p); break;
        case 16: hipLaunchKernelGGL((k_residual<16, SweepCfg<16>::NT>), g, dim3(SweepCfg<16>::NT), 0, st, p); break;
        case 32: hipLaunchKernelGGL((k_residual<32, SweepCfg<32>::NT>), g, dim3(SweepCfg<32>::NT), 0, st, p); break;
        case 64: hipLaunchKernelGGL((k_residual<64, SweepCfg<64>::NT>), g, dim3(SweepCfg<64>::NT), 0, st, p); break;
        case 96: hipLaunchKernelGGL((k_residual_big<96, 256>), g, dim3(256), 0, st, p); break;
        case 128: hipLaunchKernelGGL((k_residual_big<128, 256>), g, dim3(256), 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
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
