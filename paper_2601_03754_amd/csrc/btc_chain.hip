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
    constexpr int LD = NP + 1;
    // the blocks of the current chain step, staged by the whole wavefront
    // (one round of loads instead of one dependent load per column)
    __shared__ double sL[NP * LD];
    __shared__ double sR[NP * LD];
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int n = P.n, k = P.k, m = P.m;
    const int64_t N = P.N, s = (int64_t)1 << k, M = N >> k;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    auto stage = [&](const double* L, const double* R) {
        wave_lds_sync();  // the previous step's reads are done
        for (int e = lane; e < n * n; e += kWave) {
            sL[(e / n) * LD + e % n] = L[e];
            if (R) sR[(e / n) * LD + e % n] = R[e];
        }
        wave_lds_sync();
    };
    for (int q = 0; q < m; ++q) {
        double yprev = 0.0;
        // forward
        for (int64_t j = 1; j <= M; ++j) {
            const int64_t c = chain_block(k, j);
            const int64_t pc = perm_pos(N, level_of(c), c);
            stage(P.Ld + (size_t)pc * nn, j > 1 ? P.Rb + (size_t)perm_pos(N, level_of(c - s), c - s) * nn : nullptr);
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
                double v = 0.0;
                for (int t = 0; t < n; ++t) {
                    const double yt = readlane_d(yprev, t);
                    if (lane < n) v = fma(sR[lane * LD + t], yt, v);
                }
                a -= v;
            }
            // y = L^{-1} a, column sweep with the pivot values broadcast
            for (int t = 0; t < n; ++t) {
                const double yt = readlane_d(a, t) / sL[t * LD + t];
                if (lane == t) a = yt;
                else if (lane > t && lane < n) a = fma(-sL[lane * LD + t], yt, a);
            }
            if (lane < n) P.Y[(size_t)pc * nm + (size_t)lane * m + q] = a;
            yprev = a;
        }
        // backward
        double xnext = 0.0;
        for (int64_t j = M; j >= 1; --j) {
            const int64_t c = chain_block(k, j);
            const int64_t pc = perm_pos(N, level_of(c), c);
            stage(P.Ld + (size_t)pc * nn, j < M ? P.Rb + (size_t)pc * nn : nullptr);
            double a = lane < n ? P.Y[(size_t)pc * nm + (size_t)lane * m + q] : 0.0;
            if (j < M) {
                // - R'_j^T x_{j+1}
                double v = 0.0;
                for (int t = 0; t < n; ++t) {
                    const double xt = readlane_d(xnext, t);
                    if (lane < n) v = fma(sR[t * LD + lane], xt, v);
                }
                a -= v;
            }
            for (int t = n - 1; t >= 0; --t) {
                const double xt = readlane_d(a, t) / sL[t * LD + t];
                if (lane == t) a = xt;
                else if (lane < t) a = fma(-sL[t * LD + lane], xt, a);
            }
            if (lane < n) P.X[((size_t)(c - 1) * n + lane) * m + q] = a;
            xnext = a;
        }
    }
}

// ---------------------------------------------------------------------------
// Partition order (section "Partition Permutation", Algorithm 2): chunk 1 =
// blocks 1 .. N_1, separator s_1 = N_1 + 1, chunk 2 = the next N_k blocks,
// separator s_2, ..., chunk p.  Every chunk is eliminated in natural order by
// its own wavefront, all chunks at once; then the separators, in order, by
// one wavefront.  Within chunk j (0-based) with left separator sl = s_j
// (j >= 1) and right separator sr = s_{j+1} (j <= p-2), block i:
//   S_i = D_i - R_{i-1} R_{i-1}^T (within the chunk);  L_i = chol(S_i)
//   R_i = C_{i+1,i} L_i^{-T}                 (next block, or sr for the last)
//   T_i = L_i^{-1} H_i, H_i = block (i, sl)  (the input coupling for the first
//                                            block, then the fill below)
//   G  += T_i^T T_i                          (sl's Schur complement)
//   H_{i+1} = -R_i T_i                       (fill: block (i+1, sl), or
//                                            (sr, sl) after the last block)
// The factor is stored by original block: L_i in Ld, R_i in Rb, T_i in Tb.
// A chunk leaves its contributions where its separators' own factor blocks
// go later: R_last R_last^T (to sr) in Ld[sr], G (to sl) in Rb[sl], and the
// fill (sr, sl) in Tb[sr]; the separator chain reads them first:
//   S_{s_j} = D_{s_j} - Ld[s_j] - Rb[s_j] - R'_{j-1} R'_{j-1}^T
//   L = chol(S);  R'_j = Tb[s_{j+1}] L^{-T}  (stored in Rb[s_j])
// The solve: forward through every chunk at once (y_i, and the chunk's
// contributions to its separators: sum of T_i^T y_i left in V[sl],
// R_last y_last in U[sr]), forward and backward along the separators, then
// backward through every chunk at once.

__device__ __forceinline__ int64_t part_sep(const ChainDesc& P, int j) {  // s_j, j = 1 .. p-1
    return P.n1 + 1 + (int64_t)(j - 1) * (P.nk + 1);
}
__device__ __forceinline__ void part_chunk(const ChainDesc& P, int j, int64_t& b0, int64_t& b1) {
    b0 = j == 0 ? 1 : part_sep(P, j) + 1;
    b1 = j == 0 ? P.n1 : b0 + P.nk - 1;
}

// sS <- the symmetric n x n block src (lower triangle read), padded with 0
template <int NP>
__device__ __forceinline__ void load_sym(double* sS, const double* __restrict__ src, int n, int lane) {
    constexpr int LD = NP + 1;
    if (lane < n)
        for (int cc = 0; cc < n; ++cc) {
            const int a = cc <= lane ? lane : cc, b = cc <= lane ? cc : lane;
            sS[lane * LD + cc] = src[(size_t)a * n + b];
        }
    wave_lds_sync();
}

// sS[lane][c] -= sum_q A[lane][q] A[c][q] (A in LDS, row stride NP+1)
template <int NP>
__device__ __forceinline__ void sub_aat_lds(double* sS, const double* sA, int n, int lane) {
    constexpr int LD = NP + 1;
    double acc[NP];
    if (lane < n) {
#pragma unroll
        for (int cc = 0; cc < NP; ++cc) acc[cc] = 0.0;
        for (int q = 0; q < n; ++q) {
            const double al = sA[lane * LD + q];
#pragma unroll
            for (int cc = 0; cc < NP; ++cc)
                if (cc < n) acc[cc] = fma(al, sA[cc * LD + q], acc[cc]);
        }
#pragma unroll
        for (int cc = 0; cc < NP; ++cc)
            if (cc < n) sS[lane * LD + cc] -= acc[cc];
    }
    wave_lds_sync();
}

// row lane of X = C L^{-T} (C given by rows through `crow`), into sX
template <int NP, class RowFn>
__device__ __forceinline__ void right_solve_lt(double* sX, const double* sL, int n, int lane, RowFn crow) {
    constexpr int LD = NP + 1;
    double acc[NP];
    if (lane < n) {
#pragma unroll
        for (int cc = 0; cc < NP; ++cc) acc[cc] = cc < n ? crow(cc) : 0.0;
#pragma unroll
        for (int jj = 0; jj < NP; ++jj) {
            if (jj < n) {
                double v = acc[jj];
#pragma unroll
                for (int q = 0; q < jj; ++q) v = fma(-acc[q], sL[jj * LD + q], v);
                acc[jj] = v / sL[jj * LD + jj];
            }
        }
    }
    wave_lds_sync();
    if (lane < n) {
#pragma unroll
        for (int cc = 0; cc < NP; ++cc)
            if (cc < n) sX[lane * LD + cc] = acc[cc];
    }
    wave_lds_sync();
}

template <int NP>
__global__ __launch_bounds__(kWave) void k_part_chunks(ChainDesc P) {
    constexpr int LD = NP + 1;
    __shared__ double sS[NP * LD];  // S_i -> L_i
    __shared__ double sR[NP * LD];  // R_{i-1}, then R_i
    __shared__ double sH[NP * LD];  // H_i (block (i, sl)), then the fill H_{i+1}
    __shared__ double sT[NP * LD];  // T_i^T (row r = column r of T_i)
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int j = blockIdx.x, p = P.parts, n = P.n;
    const size_t nn = (size_t)n * n;
    int64_t b0, b1;
    part_chunk(P, j, b0, b1);
    const bool has_l = j >= 1, has_r = j + 1 < p;
    const int64_t sl = has_l ? b0 - 1 : 0, sr = has_r ? b1 + 1 : 0;
    for (int64_t i = b0; i <= b1; ++i) {
        load_sym<NP>(sS, P.A_diag + (size_t)(i - 1) * nn, n, lane);
        if (i > b0) sub_aat_lds<NP>(sS, sR, n, lane);
        if (!chol_lds<NP>(sS, n, lane)) {
            if (lane == 0) atomicMin(P.info, (unsigned long long)i);
            return;
        }
        double* Lout = P.Ld + (size_t)(i - 1) * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc) Lout[(size_t)lane * n + cc] = cc <= lane ? sS[lane * LD + cc] : 0.0;
        if (has_l) {
            // H_i: the input coupling (b0, sl) for the first block
            if (i == b0) {
                const double* E = P.A_off + (size_t)(sl - 1) * nn;
                if (lane < n)
                    for (int cc = 0; cc < n; ++cc) sH[lane * LD + cc] = E[(size_t)lane * n + cc];
                wave_lds_sync();
            }
            // T_i^T = H_i^T L_i^{-T}: row r from column r of H_i
            right_solve_lt<NP>(sT, sS, n, lane, [&](int q) { return sH[q * LD + lane]; });
            double* Tout = P.Tb + (size_t)(i - 1) * nn;
            if (lane < n)
                for (int q = 0; q < n; ++q) Tout[(size_t)q * n + lane] = sT[lane * LD + q];
            // G += T_i^T T_i (row lane), kept in Rb[sl]
            double* G = P.Rb + (size_t)(sl - 1) * nn;
            if (lane < n)
                for (int cc = 0; cc < n; ++cc) {
                    double v = 0.0;
                    for (int q = 0; q < n; ++q) v = fma(sT[lane * LD + q], sT[cc * LD + q], v);
                    G[(size_t)lane * n + cc] = (i == b0 ? 0.0 : G[(size_t)lane * n + cc]) + v;
                }
        }
        const bool rn = i < b1 || has_r;
        if (rn) {
            // R_i = C_{i+1,i} L_i^{-T} (the next block or sr: both i + 1)
            const double* C = P.A_off + (size_t)(i - 1) * nn;
            right_solve_lt<NP>(sR, sS, n, lane, [&](int q) { return C[(size_t)lane * n + q]; });
            double* Rout = P.Rb + (size_t)(i - 1) * nn;
            if (lane < n)
                for (int cc = 0; cc < n; ++cc) Rout[(size_t)lane * n + cc] = sR[lane * LD + cc];
            if (has_l) {
                // fill -R_i T_i: block (i+1, sl), row lane
                double f[NP];
                if (lane < n) {
#pragma unroll
                    for (int cc = 0; cc < NP; ++cc) {
                        double v = 0.0;
                        if (cc < n)
                            for (int q = 0; q < n; ++q) v = fma(sR[lane * LD + q], sT[cc * LD + q], v);
                        f[cc] = -v;
                    }
                }
                wave_lds_sync();
                if (lane < n) {
#pragma unroll
                    for (int cc = 0; cc < NP; ++cc)
                        if (cc < n) sH[lane * LD + cc] = f[cc];
                }
                wave_lds_sync();
            }
        }
        wave_lds_sync();
    }
    if (has_r) {
        // R_last R_last^T for sr (in Ld[sr]), and the fill (sr, sl) in Tb[sr]
        double* RR = P.Ld + (size_t)(sr - 1) * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc) {
                double v = 0.0;
                for (int q = 0; q < n; ++q) v = fma(sR[lane * LD + q], sR[cc * LD + q], v);
                RR[(size_t)lane * n + cc] = v;
            }
        if (has_l) {
            double* F = P.Tb + (size_t)(sr - 1) * nn;
            if (lane < n)
                for (int cc = 0; cc < n; ++cc) F[(size_t)lane * n + cc] = sH[lane * LD + cc];
        }
    }
}

template <int NP>
__global__ __launch_bounds__(kWave) void k_part_chain(ChainDesc P) {
    constexpr int LD = NP + 1;
    __shared__ double sS[NP * LD];
    __shared__ double sR[NP * LD];
    __shared__ double sC[NP * LD];
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int p = P.parts, n = P.n;
    const size_t nn = (size_t)n * n;
    for (int j = 1; j < p; ++j) {
        const int64_t s = part_sep(P, j);
        load_sym<NP>(sS, P.A_diag + (size_t)(s - 1) * nn, n, lane);
        // the chunks' contributions: R R^T of the chunk on the left, G of the
        // chunk on the right (both full symmetric blocks)
        const double* RR = P.Ld + (size_t)(s - 1) * nn;
        const double* G = P.Rb + (size_t)(s - 1) * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc)
                sS[lane * LD + cc] -= RR[(size_t)lane * n + cc] + G[(size_t)lane * n + cc];
        wave_lds_sync();
        if (j > 1) sub_aat_lds<NP>(sS, sR, n, lane);
        if (!chol_lds<NP>(sS, n, lane)) {
            if (lane == 0) atomicMin(P.info, (unsigned long long)s);
            return;
        }
        double* Lout = P.Ld + (size_t)(s - 1) * nn;
        if (lane < n)
            for (int cc = 0; cc < n; ++cc) Lout[(size_t)lane * n + cc] = cc <= lane ? sS[lane * LD + cc] : 0.0;
        if (j + 1 < p) {
            // R'_j = F L^{-T}, F = block (s_{j+1}, s_j) left by chunk j
            const double* F = P.Tb + (size_t)(part_sep(P, j + 1) - 1) * nn;
            if (lane < n)
                for (int cc = 0; cc < n; ++cc) sC[lane * LD + cc] = F[(size_t)lane * n + cc];
            wave_lds_sync();
            right_solve_lt<NP>(sR, sS, n, lane, [&](int q) { return sC[lane * LD + q]; });
            double* Rout = P.Rb + (size_t)(s - 1) * nn;
            if (lane < n)
                for (int cc = 0; cc < n; ++cc) Rout[(size_t)lane * n + cc] = sR[lane * LD + cc];
        }
        wave_lds_sync();
    }
}

// y = L^{-1} a (lane r holds row r), L row-major n x n in global memory
__device__ __forceinline__ double lower_solve(const double* __restrict__ L, double a, int n, int lane) {
    for (int t = 0; t < n; ++t) {
        const double yt = readlane_d(a, t) / L[(size_t)t * n + t];
        if (lane == t) a = yt;
        else if (lane > t && lane < n) a = fma(-L[(size_t)lane * n + t], yt, a);
    }
    return a;
}
// x = L^{-T} a
__device__ __forceinline__ double upper_solve(const double* __restrict__ L, double a, int n, int lane) {
    for (int t = n - 1; t >= 0; --t) {
        const double xt = readlane_d(a, t) / L[(size_t)t * n + t];
        if (lane == t) a = xt;
        else if (lane < t) a = fma(-L[(size_t)t * n + lane], xt, a);
    }
    return a;
}
// lane r: sum_t M[r][t] v[t] (TR: sum_t M[t][r] v[t]); v held one row per lane
template <bool TR>
__device__ __forceinline__ double matvec_lanes(const double* __restrict__ M, double v, int n, int lane) {
    double acc = 0.0;
    for (int t = 0; t < n; ++t) {
        const double vt = readlane_d(v, t);
        if (lane < n) acc = fma(TR ? M[(size_t)t * n + lane] : M[(size_t)lane * n + t], vt, acc);
    }
    return acc;
}

// phase 0: forward through the chunks; 1: along the separators (forward and
// backward); 2: backward through the chunks.  Y, U, V, X indexed by
// original block ([N][n][m]).
template <int NP, int PHASE>
__global__ __launch_bounds__(kWave) void k_part_solve(ChainDesc P) {
    const int lane = threadIdx.x;
    if (*P.info != kInfoOk) return;
    const int p = P.parts, n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    auto vec = [&](const double* base, int64_t i, int q) {
        return lane < n ? base[(size_t)(i - 1) * nm + (size_t)lane * m + q] : 0.0;
    };
    auto put = [&](double* base, int64_t i, int q, double v) {
        if (lane < n) base[(size_t)(i - 1) * nm + (size_t)lane * m + q] = v;
    };
    for (int q = 0; q < m; ++q) {
        if (PHASE == 0 || PHASE == 2) {
            const int j = blockIdx.x;
            int64_t b0, b1;
            part_chunk(P, j, b0, b1);
            const bool has_l = j >= 1, has_r = j + 1 < p;
            const int64_t sl = has_l ? b0 - 1 : 0, sr = has_r ? b1 + 1 : 0;
            if (PHASE == 0) {
                double y = 0.0, g = 0.0;
                for (int64_t i = b0; i <= b1; ++i) {
                    double a = vec(P.B, i, q);
                    if (i > b0) a -= matvec_lanes<false>(P.Rb + (size_t)(i - 2) * nn, y, n, lane);
                    y = lower_solve(P.Ld + (size_t)(i - 1) * nn, a, n, lane);
                    put(P.Y, i, q, y);
                    if (has_l) g += matvec_lanes<true>(P.Tb + (size_t)(i - 1) * nn, y, n, lane);
                }
                if (has_l) put(const_cast<double*>(P.V), sl, q, g);
                if (has_r) put(const_cast<double*>(P.U), sr, q, matvec_lanes<false>(P.Rb + (size_t)(b1 - 1) * nn, y, n, lane));
            } else {
                const double xl = has_l ? vec(P.X, sl, q) : 0.0;
                double x = has_r ? vec(P.X, sr, q) : 0.0;
                for (int64_t i = b1; i >= b0; --i) {
                    double a = vec(P.Y, i, q);
                    if (i < b1 || has_r) a -= matvec_lanes<true>(P.Rb + (size_t)(i - 1) * nn, x, n, lane);
                    if (has_l) a -= matvec_lanes<false>(P.Tb + (size_t)(i - 1) * nn, xl, n, lane);
                    x = upper_solve(P.Ld + (size_t)(i - 1) * nn, a, n, lane);
                    put(P.X, i, q, x);
                }
            }
        } else {
            double y = 0.0;
            for (int j = 1; j < p; ++j) {
                const int64_t s = part_sep(P, j);
                double a = vec(P.B, s, q) - vec(P.U, s, q) - vec(P.V, s, q);
                if (j > 1) a -= matvec_lanes<false>(P.Rb + (size_t)(part_sep(P, j - 1) - 1) * nn, y, n, lane);
                y = lower_solve(P.Ld + (size_t)(s - 1) * nn, a, n, lane);
                put(P.Y, s, q, y);
            }
            double x = 0.0;
            for (int j = p - 1; j >= 1; --j) {
                const int64_t s = part_sep(P, j);
                double a = vec(P.Y, s, q);
                if (j + 1 < p) a -= matvec_lanes<true>(P.Rb + (size_t)(s - 1) * nn, x, n, lane);
                x = upper_solve(P.Ld + (size_t)(s - 1) * nn, a, n, lane);
                put(P.X, s, q, x);
            }
        }
    }
}

}  // namespace

hipError_t launch_part_factor(const ChainDesc& p, int np, hipStream_t st) {
    const dim3 g((unsigned)p.parts), b(kWave);
    switch (np) {
        case 8: hipLaunchKernelGGL(k_part_chunks<8>, g, b, 0, st, p); hipLaunchKernelGGL(k_part_chain<8>, dim3(1), b, 0, st, p); break;
        case 16: hipLaunchKernelGGL(k_part_chunks<16>, g, b, 0, st, p); hipLaunchKernelGGL(k_part_chain<16>, dim3(1), b, 0, st, p); break;
        case 32: hipLaunchKernelGGL(k_part_chunks<32>, g, b, 0, st, p); hipLaunchKernelGGL(k_part_chain<32>, dim3(1), b, 0, st, p); break;
        case 64: hipLaunchKernelGGL(k_part_chunks<64>, g, b, 0, st, p); hipLaunchKernelGGL(k_part_chain<64>, dim3(1), b, 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_part_solve(const ChainDesc& p, int np, hipStream_t st) {
    const dim3 g((unsigned)p.parts), b(kWave);
    switch (np) {
#define BTC_PART_SOLVE(NPV)                                                   \
    case NPV:                                                                 \
        hipLaunchKernelGGL((k_part_solve<NPV, 0>), g, b, 0, st, p);           \
        hipLaunchKernelGGL((k_part_solve<NPV, 1>), dim3(1), b, 0, st, p);     \
        hipLaunchKernelGGL((k_part_solve<NPV, 2>), g, b, 0, st, p);           \
        break;
        BTC_PART_SOLVE(8)
        BTC_PART_SOLVE(16)
        BTC_PART_SOLVE(32)
        BTC_PART_SOLVE(64)
#undef BTC_PART_SOLVE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

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
