// Matrix-core tile helpers shared by the factorization kernels (gfx950).
//
// Blocks are staged in LDS padded to NP x NP with an odd row stride and split
// into 16 x 16 tiles; block products run on MFMA instructions whose operand
// and accumulator lane layouts are:
//   v_mfma_f64_16x16x4f64 : A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//                           accumulator register v of lane l = element
//                           (4v + l/16, l%16)
//   v_mfma_f32_16x16x4f32 : same operand layout (one float per lane),
//                           accumulator register v of lane l = element
//                           (4(l/16) + v, l%16)
#pragma once

#include "btc_device.h"

namespace btc {
namespace tiles {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;       // tile side
constexpr int kLDI = kT + 1; // row stride of an inverted diagonal tile in LDS

// f64 16x16x4 accumulator layout: register v of lane l holds tile element
// (4v + l/16, l%16).  Operand layouts: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k.
__device__ __forceinline__ int acc_r(int v, int lane) { return 4 * v + (lane >> 4); }
__device__ __forceinline__ int acc_c(int lane) { return lane & 15; }

// acc += (NEG ? -1 : 1) * sum_{kk<K} opA[ra+i][ka+kk] * opB[kb+kk][cb+j]
//   opA[r][k] = TA ? A[k][r] : A[r][k],  opB[k][c] = TB ? B[c][k] : B[k][c]
template <int LDA, int LDB, bool TA, bool TB, bool NEG>
__device__ __forceinline__ void mma_tile(d4& acc, const double* __restrict__ A, int ra, int ka,
                                         const double* __restrict__ B, int cb, int kb, int K) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, q = lane >> 4;
    auto opa = [&](int kk) {
        const int k1 = ka + kk + q;
        const double a = TA ? A[k1 * LDA + ra + i] : A[(ra + i) * LDA + k1];
        return NEG ? -a : a;
    };
    auto opb = [&](int kk) {
        const int k2 = kb + kk + q;
        return TB ? B[(cb + i) * LDB + k2] : B[k2 * LDB + cb + i];
    };
    if (K >= 16 && K % 8 == 0) {
        // two independent accumulation chains (hides the matrix-core latency)
        d4 acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int kk = 0; kk < K; kk += 8) {
            const double a0 = opa(kk), b0 = opb(kk), a1 = opa(kk + 4), b1 = opb(kk + 4);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
        }
        acc += acc1;
        return;
    }
#pragma unroll 4
    for (int kk = 0; kk < K; kk += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opa(kk), opb(kk), acc, 0, 0, 0);
}

template <int LD>
__device__ __forceinline__ void acc_load_lds(d4& acc, const double* __restrict__ S, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = S[(r0 + acc_r(v, lane)) * LD + c0 + acc_c(lane)];
}

template <int LD>
__device__ __forceinline__ void acc_store_lds(const d4& acc, double* __restrict__ S, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(r0 + acc_r(v, lane)) * LD + c0 + acc_c(lane)] = acc[v];
}

// Load a tile of an n x n global block (lower triangle only, identity padding).
__device__ __forceinline__ void acc_load_sym(d4& acc, const double* __restrict__ src, int n, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + acc_r(v, lane), c = c0 + acc_c(lane);
        double x = (r == c) ? 1.0 : 0.0;
        if (r < n && c < n && c <= r) x = src[(size_t)r * n + c];
        acc[v] = x;
    }
}

__device__ __forceinline__ void acc_store_global(const d4& acc, double* __restrict__ dst, int n, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + acc_r(v, lane), c = c0 + acc_c(lane);
        if (r < n && c < n) dst[(size_t)r * n + c] = acc[v];
    }
}

// LDS layouts of the lower triangle of an NP x NP block, addressed by
// 16 x 16 tiles; tile (a, b) has row stride LDT.
// Row-major square layout, row stride LD.
template <int LD>
struct SquareLds {
    static constexpr int LDT = LD;
    template <class T>
    __device__ static T* tile(T* A, int a, int b) { return A + (kT * a) * LD + kT * b; }
};
// Lower tiles only (about half the LDS): tile (a, b), b <= a, at position
// a(a+1)/2 + b, rows of kLDI elements (conflict-free 16 x 4 operand reads).
struct PackedLds {
    static constexpr int LDT = kLDI;
    static constexpr int kTile = kT * kLDI;
    template <class T>
    __device__ static T* tile(T* A, int a, int b) { return A + (a * (a + 1) / 2 + b) * kTile; }
};
template <int NP>
constexpr int packed_lds_elems() { return (NP / kT) * (NP / kT + 1) / 2 * PackedLds::kTile; }

// k-th lower-triangle tile (a, b), b <= a, in row-major order of the triangle.
__device__ __forceinline__ void tri_tile(int k, int& a, int& b) {
    a = 0;
    while ((a + 1) * (a + 2) / 2 <= k) ++a;
    b = k - a * (a + 1) / 2;
}

// 1/sqrt(p): hardware estimate r refined by one third-order step.  With
// e = 1 - p r^2, 1/sqrt(p) = r (1 - e)^(-1/2) = r (1 + e/2 + 3e^2/8 + ...);
// the estimate's e of about 1e-7 leaves a truncation term near 1e-22, and
// the chain is four dependent operations instead of two Newton steps' six.
__device__ __forceinline__ double rsqrt_refined(double p) {
    const double r = __builtin_amdgcn_rsq(p);
    const double e = fma(-p * r, r, 1.0);
    return fma(r * e, fma(e, 0.375, 0.5), r);
}

// Cholesky of a 16-column panel held one row per lane: lanes 0..NC-1 hold
// the rows of the NC x NC diagonal tile (zeros above the diagonal), any other
// lane a row below it (or zeros).  Column j: the pivot row's lane forms
// L_jj, every lane below it its multiplier a_rj / L_jj (for the rows below
// the tile this is the triangular solve x L_pp^T = a), and the multipliers of
// the pivot rows reach the later columns by readlane broadcasts (no LDS round
// trip on the chain).  On return a holds the rows of L, myinv 1/L_rr on lane
// r < NC; false on a non-positive or NaN pivot.
template <int NC>
__device__ __forceinline__ bool chol_rows(double (&a)[NC], double& myinv) {
    const int lane = threadIdx.x & (kWave - 1);
    double piv = readlane_d(a[0], 0);
    double r = rsqrt_refined(piv);
    myinv = 1.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        ok = ok && (piv > 0.0);
        double l = a[j] * r;
        l = (lane == j) ? piv * r : l;
        l = (lane < j) ? 0.0 : l;
        myinv = (lane == j) ? r : myinv;
        a[j] = l;
        if (j + 1 < NC) {
            // the next pivot first: its reciprocal square root overlaps the
            // rest of this column's update
            a[j + 1] = fma(-l, readlane_d(l, j + 1), a[j + 1]);
            piv = readlane_d(a[j + 1], j + 1);
            const double rn = rsqrt_refined(piv);
            double lc[NC];
#pragma unroll
            for (int c = j + 2; c < NC; ++c) lc[c] = readlane_d(l, c);
#pragma unroll
            for (int c = j + 2; c < NC; ++c) a[c] = fma(-l, lc[c], a[c]);
            r = rn;
        }
    }
    return ok;
}

// Cholesky of the lower triangle of an NP x NP LDS tile (NP <= 16, row
// stride LD) by one wavefront with lane r holding row r: writes L back (zero
// strict upper part) and 1/L_jj to invd; false on a non-positive or NaN
// pivot.
template <int NP, int LD = NP + 1>
__device__ __forceinline__ bool potrf_small(double* __restrict__ A, double* __restrict__ invd) {
    static_assert(NP <= 16, "small tiles only");
    const int lane = threadIdx.x & (kWave - 1);
    double a[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) a[c] = (lane < NP && c <= lane) ? A[lane * LD + c] : 0.0;
    double myinv;
    const bool ok = chol_rows<NP>(a, myinv);
    if (lane < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) A[lane * LD + c] = (c <= lane) ? a[c] : 0.0;
        invd[lane] = myinv;
    }
    return ok;
}

// Inverse of the 16 x 16 lower-triangular diagonal tile of L starting at
// (r0, r0) into Dinv (row stride kLDI): lane c (< 16) forward-substitutes the
// unit vector e_c.
template <int LD, class TOut>
__device__ __forceinline__ void tile_inverse(const double* __restrict__ L, int r0, const double* __restrict__ invd,
                                             TOut* __restrict__ Dinv) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 15;
    double x[kT];
#pragma unroll
    for (int j = 0; j < kT; ++j) x[j] = (j == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < kT; ++j) {
        x[j] *= invd[r0 + j];
#pragma unroll
        for (int k = j + 1; k < kT; ++k) x[k] = fma(-L[(r0 + k) * LD + r0 + j], x[j], x[k]);
    }
    if (lane < kT) {
#pragma unroll
        for (int j = 0; j < kT; ++j) Dinv[j * kLDI + c] = (TOut)x[j];
    }
}


// Inverse of the 16 x 16 lower-triangular tile T (row stride LD) by one
// wavefront, written transposed into the tile's strict upper triangle: the
// strict lower part of the inverse at T[c][j] for c < j (its diagonal is
// invd).  Lane c (< 16) forward-substitutes e_c; the reads (lower part) and
// the writes (upper part) never touch the same element.
template <int LD>
__device__ __forceinline__ void tile_inverse_upper(double* T, const double* __restrict__ invd) {
    static_assert(LD > kT, "the tile rows need a padding column");
    const int lane = threadIdx.x & 63;
    const int c = lane & 15;
    double x[kT];
#pragma unroll
    for (int j = 0; j < kT; ++j) x[j] = (j == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < kT; ++j) {
        x[j] *= invd[j];
#pragma unroll
        for (int k = j + 1; k < kT; ++k) x[k] = fma(-T[k * LD + j], x[j], x[k]);
    }
    if (lane < kT) {
        // entries on or below the diagonal go to the row's padding column
        // (index kT; LD > kT), so every store is unconditional
#pragma unroll
        for (int j = 1; j < kT; ++j) T[c * LD + (j > c ? j : kT)] = x[j];
    }
}

// Blocked Cholesky of the lower triangle of an NP x NP LDS tile (row stride
// LD) by all NW wavefronts of the workgroup (every thread must call it), in
// 16-column panels.  A panel is factored in registers, one row per lane, by
// chol_rows: each panel wavefront holds the 16 rows of the diagonal tile in
// lanes 0..15 (every panel wavefront repeats that part of the chain, so no
// wavefront waits on another inside a panel) and up to 48 rows below it in
// lanes 16..63, whose multipliers are the triangular solve L_tp = A_tp
// L_pp^{-T}.  Look-ahead: the panel wavefronts of panel p+1 apply panel p's
// update to their own tiles of column p+1 (A_ap -= L_ap L_(p+1)p^T; the
// diagonal tile into the wavefront's scratch tile when two or more
// wavefronts share the panel) and factor it at once, while the other
// wavefronts update the trailing tiles right of column p+1 (matrix cores).
// The 16 x 16 diagonal tiles are inverted at
// the end, spread over the wavefronts.  On return: L in the lower triangle
// (strict upper part of each diagonal tile zeroed, tiles above the diagonal
// untouched), 1/L_jj in invd, the inverted diagonal tiles in inv[NP/16] (row
// stride kLDI).  *fail (LDS, 0 on entry) becomes 1 on a non-positive or NaN
// pivot; the result is then false for every thread.
// INV: where the inverted diagonal tiles go: 1 the array inv (row stride
// kLDI), 2 transposed into the strict upper part of each diagonal tile.
// scr: one 16 x kLDI tile per panel wavefront, needed when a panel has more
// than 48 rows below its diagonal tile (NP > 64).
template <int NP, int LD, int NW, class Lay = SquareLds<LD>, int INV = 1>
__device__ __forceinline__ bool potrf_blocked(double* __restrict__ A, double* __restrict__ invd,
                                              double (*__restrict__ inv)[kT * kLDI], int* fail,
                                              double (*__restrict__ scr)[kT * kLDI] = nullptr) {
    constexpr int NTL = NP / kT;
    constexpr int LT = Lay::LDT;
    constexpr int kBelow = kWave - kT;  // rows below the diagonal tile per panel wavefront
    // wavefronts that factor panel q
    constexpr auto pwaves = [](int q) { return NP - (q + 1) * kT <= 0 ? 1 : (NP - (q + 1) * kT + kBelow - 1) / kBelow; };
    static_assert(pwaves(0) <= NW, "too few wavefronts for the first panel");
    static_assert(NTL <= 2 || pwaves(1) < NW, "the trailing update needs a wavefront outside the panel");
    static_assert(kBelow % kT == 0, "whole tiles per panel wavefront");
    constexpr int kTilesBelow = kBelow / kT;
    constexpr bool kShared = pwaves(0) > 1;  // some panel has two or more wavefronts
    const int tid = threadIdx.x;
    const int w = wave_id();
    const int lane = tid & 63;
    double a[kT];
    double myinv = 1.0;
    // this wavefront's rows of panel q into registers (lanes 0..15 from the
    // diagonal tile at D with row stride ldd, the others from the tiles below)
    auto load_rows = [&](int q, const double* D, int ldd) {
        const int below = NP - (q + 1) * kT;
        const int rb = kBelow * w + lane - kT;
        const bool diag = lane < kT;
        const bool has = diag || (lane - kT < kBelow && rb < below);
        // every lane loads from a valid row (a lane without a row reads the
        // diagonal tile's first row and keeps zeros)
        const double* row = diag ? D + lane * ldd : has ? Lay::tile(A, q + 1 + rb / kT, q) + (rb % kT) * LT : D;
#pragma unroll
        for (int c = 0; c < kT; ++c) {
            const double x = row[c];
            a[c] = (has && (!diag || c <= lane)) ? x : 0.0;
        }
    };
    // wavefront 0's rows of the factored diagonal tile q: into the tile
    // itself when it factored the panel alone (no other wavefront reads that
    // tile), else into its scratch tile, copied into place after the barrier
    // (the other panel wavefronts read the unfactored tile before it)
    auto store_diag = [&](int q) {
        if (w == 0 && lane < kT) {
            const bool alone = !kShared || pwaves(q) == 1;
            double* row = alone ? Lay::tile(A, q, q) + lane * LT : scr[0] + lane * kLDI;
#pragma unroll
            for (int c = 0; c < kT; ++c) row[c] = (c <= lane) ? a[c] : 0.0;
        }
    };
    auto place_diag = [&](int q) {
        if (kShared && pwaves(q) > 1 && w == 0) {
            wave_lds_sync();
            for (int e = lane; e < kT * kT; e += kWave)
                Lay::tile(A, q, q)[(e / kT) * LT + e % kT] = scr[0][(e / kT) * kLDI + e % kT];
            wave_lds_sync();
        }
    };
    // factor panel q (rows loaded), store the rows below the diagonal tile
    // and 1/L_jj
    auto factor_rows = [&](int q) {
        const bool ok = chol_rows<kT>(a, myinv);
        if (!ok && lane == 0) *fail = 1;
        const int below = NP - (q + 1) * kT;
        const int rb = kBelow * w + lane - kT;
        if (lane >= kT && lane - kT < kBelow && rb < below) {
            double* row = Lay::tile(A, q + 1 + rb / kT, q) + (rb % kT) * LT;
#pragma unroll
            for (int c = 0; c < kT; ++c) row[c] = a[c];
        }
        if (w == 0 && lane < kT) invd[q * kT + lane] = myinv;
        store_diag(q);
    };
    // A_ab -= L_ap L_bp^T
    auto update = [&](int ta, int tb, int p) {
        double* Tab = Lay::tile(A, ta, tb);
        d4 acc;
        acc_load_lds<LT>(acc, Tab, 0, 0);
        mma_tile<LT, LT, false, true, true>(acc, Lay::tile(A, ta, p), 0, 0, Lay::tile(A, tb, p), 0, 0, kT);
        acc_store_lds<LT>(acc, Tab, 0, 0);
    };
    if (w < pwaves(0)) {
        load_rows(0, Lay::tile(A, 0, 0), LT);
        factor_rows(0);
    }
    __syncthreads();
    if (*fail) return false;
#pragma unroll 1
    for (int p = 0; p + 1 < NTL; ++p) {
        const int q = p + 1;
        const int pw = kShared ? pwaves(q) : 1;
        place_diag(p);
        if (w < pw) {
            // this wavefront's tiles of column q below the diagonal tile
#pragma unroll 1
            for (int t = 0; t < kTilesBelow; ++t) {
                const int ta = q + 1 + kTilesBelow * w + t;
                if (ta < NTL) update(ta, q, p);
            }
            // the diagonal tile: in place when this wavefront factors the
            // panel alone, else into its scratch tile
            d4 acc;
            acc_load_lds<LT>(acc, Lay::tile(A, q, q), 0, 0);
            mma_tile<LT, LT, false, true, true>(acc, Lay::tile(A, q, p), 0, 0, Lay::tile(A, q, p), 0, 0, kT);
            if (!kShared || pw == 1) {
                acc_store_lds<LT>(acc, Lay::tile(A, q, q), 0, 0);
                wave_lds_sync();
                load_rows(q, Lay::tile(A, q, q), LT);
            } else {
                acc_store_lds<kLDI>(acc, scr[w], 0, 0);
                wave_lds_sync();
                load_rows(q, scr[w], kLDI);
            }
            factor_rows(q);
        } else {
            // the trailing tiles right of column q
            const int m = NTL - 1 - q;
            for (int k = w - pw; k < m * (m + 1) / 2; k += NW - pw) {
                int ta, tb;
                tri_tile(k, ta, tb);
                update(q + 1 + ta, q + 1 + tb, p);
            }
        }
        __syncthreads();
        if (*fail) return false;
    }
    place_diag(NTL - 1);
    __syncthreads();
    if (INV == 1)
        for (int t = w; t < NTL; t += NW) tile_inverse<LT, double>(Lay::tile(A, t, t), 0, invd + t * kT, inv[t]);
    else
        for (int t = w; t < NTL; t += NW) tile_inverse_upper<LT>(Lay::tile(A, t, t), invd + t * kT);
    __syncthreads();
    return true;
}



// ---------------------------------------------------------------------------
// FP32 tiles

__device__ __forceinline__ int acc32_r(int v, int lane) { return 4 * (lane >> 4) + v; }

// acc += (NEG ? -1 : 1) * sum_{kk<K} opA[ra+i][ka+kk] * opB[kb+kk][cb+j] in FP32
template <int LDA, int LDB, bool TA, bool TB, bool NEG>
__device__ __forceinline__ void mma_tile32(f4& acc, const float* __restrict__ A, int ra, int ka,
                                           const float* __restrict__ B, int cb, int kb, int K) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, q = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < K; kk += 4) {
        const int k1 = ka + kk + q, k2 = kb + kk + q;
        float a = TA ? A[k1 * LDA + ra + i] : A[(ra + i) * LDA + k1];
        const float b = TB ? B[(cb + i) * LDB + k2] : B[k2 * LDB + cb + i];
        if (NEG) a = -a;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
}

// acc += (NEG ? -1 : 1) * sum_{kk<K} opA[ra+i][ka+kk] * opB[kb+kk][cb+j] with the
// operands rounded to BF16 (round to nearest even) and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)+e] and
// B[8(l/16)+e][l%16], e < 8; accumulator layout as the FP32 tiles).  K is
// padded with zeros to a multiple of 32.
template <int LDA, int LDB, bool TA, bool TB, bool NEG>
__device__ __forceinline__ void mma_tile_bf16(f4& acc, const float* __restrict__ A, int ra, int ka,
                                              const float* __restrict__ B, int cb, int kb, int K) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, q = lane >> 4;
    for (int kk = 0; kk < K; kk += 32) {
        bf8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kk + 8 * q + e;
            float av = 0.f, bv = 0.f;
            if (k < K) {
                av = TA ? A[(ka + k) * LDA + ra + i] : A[(ra + i) * LDA + ka + k];
                bv = TB ? B[(cb + i) * LDB + kb + k] : B[(kb + k) * LDB + cb + i];
            }
            a[e] = (__bf16)(NEG ? -av : av);
            b[e] = (__bf16)bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
}

// Schur / fill product of the mixed kernels: FP32 or BF16 operands.
template <bool BF16, int LDA, int LDB, bool TA, bool TB, bool NEG>
__device__ __forceinline__ void mma_prod(f4& acc, const float* __restrict__ A, int ra, int ka,
                                         const float* __restrict__ B, int cb, int kb, int K) {
    if constexpr (BF16)
        mma_tile_bf16<LDA, LDB, TA, TB, NEG>(acc, A, ra, ka, B, cb, kb, K);
    else
        mma_tile32<LDA, LDB, TA, TB, NEG>(acc, A, ra, ka, B, cb, kb, K);
}

template <int LD>
__device__ __forceinline__ void acc32_load_lds(f4& acc, const float* __restrict__ S, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = S[(r0 + acc32_r(v, lane)) * LD + c0 + acc_c(lane)];
}

template <int LD>
__device__ __forceinline__ void acc32_store_lds(const f4& acc, float* __restrict__ S, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(r0 + acc32_r(v, lane)) * LD + c0 + acc_c(lane)] = acc[v];
}

// FP64 LDS tile -= FP32 accumulator (Schur update of an FP64 block by a
// product formed in lower precision)
template <int LD>
__device__ __forceinline__ void acc32_sub_from_lds64(const f4& acc, double* __restrict__ S, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(r0 + acc32_r(v, lane)) * LD + c0 + acc_c(lane)] -= (double)acc[v];
}

__device__ __forceinline__ void acc32_store_global(const f4& acc, float* __restrict__ dst, int n, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + acc32_r(v, lane), c = c0 + acc_c(lane);
        if (r < n && c < n) dst[(size_t)r * n + c] = acc[v];
    }
}

}  // namespace tiles
}  // namespace btc
