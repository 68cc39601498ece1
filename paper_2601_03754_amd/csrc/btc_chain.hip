// Sequential elimination of a chain of blocks in one wavefront (the
// sequential part of the k-stage strategies of section "Parallel Cholesky
// Factorization": Algorithm 1 on the whole chain for k = 0, on the blocks
// that remain after k levels of the multi-stage permutation otherwise; the
// single-stage permutation is k = 1, the two-stage variant k = 2).
//
// The chain is c_j = j s, j = 1 .. floor(N / s), s = 2^k.  After the first k
// levels (run by the level kernels) the Schur complement of c_j sits in the
// factor array at c_j's permuted position, minus the update its right child
// c_j + s/2 left deferred (T^T T, applied here), and the coupling between
// c_j and c_{j+1} is the fill of level k-1, stored in the slot of whichever
// of the two is an odd multiple of s (its right or left coupling slot).  For
// k = 0 they are D_j and E_j.  Per chain block (Algorithm 1):
//   S_j -= R'_{j-1} R'_{j-1}^T;  L_j = chol(S_j);  R'_j = C_{j+1,j} L_j^{-T}
// with L_j stored at c_j's diagonal slot and R'_j (the factor block at row
// c_{j+1}, column c_j) at c_j's right slot.
//
// The solve walks the chain in one launch: forward y_j = L_j^{-1} (b_j minus
// the contributions of c_j's descendants in the first k levels, minus
// R'_{j-1} y_{j-1}), then backward x_j = L_j^{-T} (y_j - R'_j^T x_{j+1}),
// so the level sweeps of the first k levels run before (forward) and after
// (backward) it.
//
// Lane r owns row r of every n x n block (n <= 64); blocks pass through LDS
// with row stride NP+1.
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {
namespace {

constexpr unsigned long long kInfoOk = ~0ull;

// S (LDS, lower triangle used) -> L in place; false if a pivot is not
// positive (or not finite).
template <int NP>
__device__ __forceinline__ bool chol_lds(double* S, int n, int lane) {
    constexpr int LD = NP + 1;
    for (int j = 0; j < n; ++j) {
        const double d = S[j * LD + j];
        if (!(d > 0.0) || !isfinite(d)) return false;
        const double p = sqrt(d);
        const double inv = 1.0 / p;
        double l = 0.0;
        if (lane > j && lane < n) {
            l = S[lane * LD + j] * inv;
            S[lane * LD + j] = l;
        }
        wave_lds_sync();
        if (lane == j) S[j * LD + j] = p;
        // trailing update of row lane: S[lane][c] -= l_lane l_c, j < c <= lane
        if (lane > j && lane < n)
            for (int c = j + 1; c <= lane; ++c) S[lane * LD + c] = fma(-l, S[c * LD + j], S[lane * LD + c]);
        wave_lds_sync();
    }
    return true;
}

// Chain node j (1-based) of a k-stage factor: original block index.
__device__ __forceinline__ int64_t chain_block(int k, int64_t j) { return j << k; }

template <int NP>
__global__ __launch_bounds__(kWave) void k_chain_factor(ChainDesc P) {
    constexpr int LD = NP + 1;
    __shared__ double sS[NP * LD];  // S_j -> L_j
    __shared__ double sR[NP * LD];  // R'_{j-1}, then R'_j
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int n = P.n, k = P.k;
    const int64_t N = P.N, s = (int64_t)1 << k, M = N >> k;
    const size_t nn = (size_t)n * n;
    for (int64_t j = 1; j <= M; ++j) {
        const int64_t c = chain_block(k, j);
        const int lc = level_of(c);
        const int64_t pc = perm_pos(N, lc, c);
        // S_j: the input block (k = 0) or the Schur complement left by the
        // level kernels, full symmetric from its lower triangle
        const double* src = k == 0 ? P.A_diag + (size_t)(c - 1) * nn : P.Ld + (size_t)pc * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc) {
                const int a = cc <= lane ? lane : cc, b = cc <= lane ? cc : lane;
                sS[lane * LD + cc] = src[(size_t)a * n + b];
            }
        wave_lds_sync();
        double acc[NP];
        // deferred update of the last level-kernel step: T_m^T T_m, m = c + s/2
        if (k > 0 && c + s / 2 <= N) {
            const int64_t m = c + s / 2;
            const double* T = P.Tb + (size_t)perm_pos(N, k - 1, m) * nn;
            if (lane < n) {
#pragma unroll
                for (int cc = 0; cc < NP; ++cc) acc[cc] = 0.0;
                for (int q = 0; q < n; ++q) {
                    const double tl = T[(size_t)q * n + lane];
#pragma unroll
                    for (int cc = 0; cc < NP; ++cc)
                        if (cc < n) acc[cc] = fma(tl, T[(size_t)q * n + cc], acc[cc]);
                }
#pragma unroll
                for (int cc = 0; cc < NP; ++cc)
                    if (cc < n) sS[lane * LD + cc] -= acc[cc];
            }
            wave_lds_sync();
        }
        // Algorithm 1: S_j -= R'_{j-1} R'_{j-1}^T
        if (j > 1) {
            if (lane < n) {
#pragma unroll
                for (int cc = 0; cc < NP; ++cc) acc[cc] = 0.0;
                for (int q = 0; q < n; ++q) {
                    const double rl = sR[lane * LD + q];
#pragma unroll
                    for (int cc = 0; cc < NP; ++cc)
                        if (cc < n) acc[cc] = fma(rl, sR[cc * LD + q], acc[cc]);
                }
#pragma unroll
                for (int cc = 0; cc < NP; ++cc)
                    if (cc < n) sS[lane * LD + cc] -= acc[cc];
            }
            wave_lds_sync();
        }
        if (!chol_lds<NP>(sS, n, lane)) {
            if (lane == 0) atomicMin(P.info, (unsigned long long)c);
            return;
        }
        double* Lout = P.Ld + (size_t)pc * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc) Lout[(size_t)lane * n + cc] = cc <= lane ? sS[lane * LD + cc] : 0.0;
        if (j == M) break;
        // coupling C_{c+s, c}: k = 0: E_c; else the fill stored in the right
        // slot of c (c an odd multiple of s) or the left slot of c + s
        const int64_t cn = c + s;
        const double* C;
        if (k == 0)
            C = P.A_off + (size_t)(c - 1) * nn;
        else if (lc == k)
            C = P.Rb + (size_t)pc * nn;
        else
            C = P.Tb + (size_t)perm_pos(N, level_of(cn), cn) * nn;
        // R'_j = C L_j^{-T}: row lane solves x L^T = C[lane]
        if (lane < n) {
#pragma unroll
            for (int cc = 0; cc < NP; ++cc) acc[cc] = cc < n ? C[(size_t)lane * n + cc] : 0.0;
#pragma unroll
            for (int jj = 0; jj < NP; ++jj) {
                if (jj < n) {
                    double v = acc[jj];
#pragma unroll
                    for (int q = 0; q < jj; ++q) v = fma(-acc[q], sS[jj * LD + q], v);
                    acc[jj] = v / sS[jj * LD + jj];
                }
            }
        }
        wave_lds_sync();
        double* Rout = P.Rb + (size_t)pc * nn;
        if (lane < n) {
#pragma unroll
            for (int cc = 0; cc < NP; ++cc)
                if (cc < n) {
                    sR[lane * LD + cc] = acc[cc];
                    Rout[(size_t)lane * n + cc] = acc[cc];
                }
        }
        wave_lds_sync();
    }
}

// Solve along the chain (after the forward level sweeps of the first k
// levels, before their backward sweeps).  y of chain block c goes to the
// forward-sweep array Y at c's permuted position (unused by the level
// kernels for these blocks), x to X.
template <int NP>
__global__ __launch_bounds__(kWave) void k_chain_solve(ChainDesc P) {
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int n = P.n, k = P.k, m = P.m;
    const int64_t N = P.N, s = (int64_t)1 << k, M = N >> k;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    for (int q = 0; q < m; ++q) {
        double yprev = 0.0;
        // forward
        for (int64_t j = 1; j <= M; ++j) {
            const int64_t c = chain_block(k, j);
            const int64_t pc = perm_pos(N, level_of(c), c);
            double a = 0.0;
            if (lane < n) {
                a = P.B[((size_t)(c - 1) * n + lane) * m + q];
                // contributions of c's descendants in the first k levels
                for (int l2 = 0; l2 < k; ++l2) {
                    const int64_t s2 = (int64_t)1 << l2;
                    const size_t off = (size_t)lane * m + q;
                    a -= P.U[(size_t)perm_pos(N, l2, c - s2) * nm + off];
                    if (c + s2 <= N) a -= P.V[(size_t)perm_pos(N, l2, c + s2) * nm + off];
                }
            }
            if (j > 1) {
                // - R'_{j-1} y_{j-1}
                const double* R = P.Rb + (size_t)perm_pos(N, level_of(c - s), c - s) * nn;
                double v = 0.0;
                for (int t = 0; t < n; ++t) {
                    const double yt = readlane_d(yprev, t);
                    if (lane < n) v = fma(R[(size_t)lane * n + t], yt, v);
                }
                a -= v;
            }
            // y = L^{-1} a, column sweep with the pivot values broadcast
            const double* L = P.Ld + (size_t)pc * nn;
            const double lrow_dummy = 0.0;
            (void)lrow_dummy;
            for (int t = 0; t < n; ++t) {
                const double yt = readlane_d(a, t) / L[(size_t)t * n + t];
                if (lane == t) a = yt;
                else if (lane > t && lane < n) a = fma(-L[(size_t)lane * n + t], yt, a);
            }
            if (lane < n) P.Y[(size_t)pc * nm + (size_t)lane * m + q] = a;
            yprev = a;
        }
        // backward
        double xnext = 0.0;
        for (int64_t j = M; j >= 1; --j) {
            const int64_t c = chain_block(k, j);
            const int64_t pc = perm_pos(N, level_of(c), c);
            double a = lane < n ? P.Y[(size_t)pc * nm + (size_t)lane * m + q] : 0.0;
            if (j < M) {
                // - R'_j^T x_{j+1}
                const double* R = P.Rb + (size_t)pc * nn;
                double v = 0.0;
                for (int t = 0; t < n; ++t) {
                    const double xt = readlane_d(xnext, t);
                    if (lane < n) v = fma(R[(size_t)t * n + lane], xt, v);
                }
                a -= v;
            }
            const double* L = P.Ld + (size_t)pc * nn;
            for (int t = n - 1; t >= 0; --t) {
                const double xt = readlane_d(a, t) / L[(size_t)t * n + t];
                if (lane == t) a = xt;
                else if (lane < t) a = fma(-L[(size_t)t * n + lane], xt, a);
            }
            if (lane < n) P.X[((size_t)(c - 1) * n + lane) * m + q] = a;
            xnext = a;
        }
    }
}

}  // namespace

hipError_t launch_chain_factor(const ChainDesc& p, int np, hipStream_t st) {
    const dim3 g(1), b(kWave);
    switch (np) {
        case 8: hipLaunchKernelGGL(k_chain_factor<8>, g, b, 0, st, p); break;
        case 16: hipLaunchKernelGGL(k_chain_factor<16>, g, b, 0, st, p); break;
        case 32: hipLaunchKernelGGL(k_chain_factor<32>, g, b, 0, st, p); break;
        case 64: hipLaunchKernelGGL(k_chain_factor<64>, g, b, 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_chain_solve(const ChainDesc& p, int np, hipStream_t st) {
    const dim3 g(1), b(kWave);
    switch (np) {
        case 8: hipLaunchKernelGGL(k_chain_solve<8>, g, b, 0, st, p); break;
        case 16: hipLaunchKernelGGL(k_chain_solve<16>, g, b, 0, st, p); break;
        case 32: hipLaunchKernelGGL(k_chain_solve<32>, g, b, 0, st, p); break;
        case 64: hipLaunchKernelGGL(k_chain_solve<64>, g, b, 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace btc
