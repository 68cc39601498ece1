// FP64 factorization level kernel on matrix cores, for padded block sizes
// NP in {16, 32, 64} (block sizes 9 <= n <= 64).  One workgroup of W = NP/16
// wavefronts per node; every n x n block is treated as W x W tiles of 16 x 16
// and every block product runs on v_mfma_f64_16x16x4f64.
//
// Per node i of level l (stride s), the same steps as the VALU kernel
// (Algorithm 4, hybrid left/right-looking, deterministic ownership):
//   P1  stage S_i, S_{i+s} and the deferred T blocks in LDS
//   P2  S_i -= T'^T T',  S_{i+s} -= T''^T T''       (deferred syrk, MFMA;
//       lower-triangle tiles only, spread round-robin over the wavefronts)
//   P3  the couplings C_{i+s,i}, C_{i,i-s} (loads issued before P2) go to
//       LDS; L_ii = chol(S_i) blocked in 16-column panels by all wavefronts
//       (wavefront 0 factors and inverts each diagonal tile, the panel and
//       trailing updates run on the matrix cores)
//   P5  R_i = C_{i+s,i} L_ii^{-T} and T_i = L_ii^{-1} C_{i,i-s} as a blocked
//       triangular solve over the tiles: each step is a tile product with the
//       already solved tiles followed by a product with an inverted diagonal
//       tile, all MFMA; wavefront w owns tile-row w of R and tile-column w of T,
//       so no workgroup barrier is needed inside the solve
//   P6  S_{i+s} -= R_i R_i^T (into the accumulators), fill -R_i T_i; stores.
#include "btc_device.h"
#include "btc_kernels.h"
#include "btc_tiles.h"

namespace btc {
namespace {

using namespace tiles;
constexpr unsigned long long kInfoOk = ~0ull;

template <int NP>
struct MfmaCfg {
    static constexpr int W = NP / kT;             // wavefronts = tile rows
    static constexpr int NT = W * kWave;
    static constexpr int NTRI = W * (W + 1) / 2;  // lower-triangle tiles
    static constexpr int TPW = (NTRI + W - 1) / W; // lower tiles per wavefront
};

template <int NP>
__global__ __launch_bounds__(MfmaCfg<NP>::NT) void k_factor_level_mfma(Launch<FactorDesc> L) {
    using Cfg = MfmaCfg<NP>;
    constexpr int W = Cfg::W, NT = Cfg::NT, LD = NP + 1;
    __shared__ double sS[NP * LD];         // S_i -> L_ii
    __shared__ double sB[NP * LD];         // T' -> C_{i+s,i} -> R_i
    __shared__ double sD[NP * LD];         // T'' -> C_{i,i-s} -> T_i
    __shared__ double sC[NP * LD];         // S_{i+s}
    __shared__ double sInv[W][kT * kLDI];  // inverted diagonal tiles of L_ii (W = NP/16)
    __shared__ double invd[NP];
    __shared__ int fail;

    FactorDesc P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (*P.info != kInfoOk) return;  // an earlier level broke down

    const int tid = threadIdx.x;
    const int w = wave_id();
    const int64_t N = P.N;
    const int n = P.n;
    const size_t nn = (size_t)n * n;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t h = s >> 1;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N;
    const bool has_l = i > s;
    const bool def_self = lvl > 0 && i + h <= N;
    const bool def_sep = lvl > 0 && has_r && i + 3 * h <= N;
    const int64_t pi = perm_pos(N, lvl, i);
    const int64_t pr = has_r ? perm_pos(N, level_of(i + s), i + s) : 0;
    const double* Ssep = (lvl == 0) ? P.A_diag + (size_t)(i + s - 1) * nn : P.Ld + (size_t)pr * nn;

    // P1: stage S_i, S_{i+s} and the deferred T blocks (all loads in flight)
    {
        Stage<NP, NT> a, b, c, d;
        a.fetch(lvl == 0 ? P.A_diag + (size_t)(i - 1) * nn : P.Ld + (size_t)pi * nn, n, true, 1.0, tid);
        if (def_self) b.fetch(P.Tb + (size_t)perm_pos(N, lvl - 1, i + h) * nn, n, false, 0.0, tid);
        if (has_r) c.fetch(Ssep, n, true, 1.0, tid);
        if (def_sep) d.fetch(P.Tb + (size_t)perm_pos(N, lvl - 1, i + 3 * h) * nn, n, false, 0.0, tid);
        a.put(sS, tid);
        if (def_self) b.put(sB, tid);
        if (has_r) c.put(sC, tid);
        if (def_sep) d.put(sD, tid);
    }
    if (tid == 0) fail = 0;
    __syncthreads();

    // coupling loads go out now and land in LDS after P2 (their buffers hold
    // the deferred T blocks until then)
    const double* Cr = (lvl == 0) ? P.A_off + (size_t)(i - 1) * nn : P.Rb + (size_t)pi * nn;
    const double* Cl = (lvl == 0) ? P.A_off + (size_t)(i - 2) * nn : P.Tb + (size_t)pi * nn;
    Stage<NP, NT> cr, cl;
    if (has_r) cr.fetch(Cr, n, false, 0.0, tid);
    else cr.fetch(Cr, 0, false, 0.0, tid);
    if (has_l) cl.fetch(Cl, n, false, 0.0, tid);
    else cl.fetch(Cl, 0, false, 0.0, tid);

    // P2: deferred syrk updates (lower tiles, round-robin over wavefronts)
#pragma unroll
    for (int t = 0; t < Cfg::TPW; ++t) {
        const int k = w + W * t;
        if (k < Cfg::NTRI) {
            int ta, tb;
            tri_tile(k, ta, tb);
            if (def_self) {
                d4 acc;
                acc_load_lds<LD>(acc, sS, ta * kT, tb * kT);
                mma_tile<LD, LD, true, false, true>(acc, sB, ta * kT, 0, sB, tb * kT, 0, NP);
                acc_store_lds<LD>(acc, sS, ta * kT, tb * kT);
            }
            if (def_sep) {
                d4 acc;
                acc_load_lds<LD>(acc, sC, ta * kT, tb * kT);
                mma_tile<LD, LD, true, false, true>(acc, sD, ta * kT, 0, sD, tb * kT, 0, NP);
                acc_store_lds<LD>(acc, sC, ta * kT, tb * kT);
            }
        }
    }
    __syncthreads();

    // P3: stage the couplings (their loads were issued before P2), then the
    // blocked Cholesky of S_i by all wavefronts: L_ii, 1/diag, inverted
    // diagonal tiles
    cr.put(sB, tid);
    cl.put(sD, tid);
    const bool ok = potrf_blocked<NP, LD, W>(sS, invd, sInv, &fail);
    if (!ok) {
        if (tid == 0) atomicMin(P.info, (unsigned long long)i);
        return;
    }

    // P5: blocked triangular solves; wavefront w owns tile-row w of R and
    // tile-column w of T
    if (has_r) {
#pragma unroll
        for (int p = 0; p < W; ++p) {
            d4 acc;
            acc_load_lds<LD>(acc, sB, w * kT, p * kT);
#pragma unroll
            for (int q = 0; q < p; ++q)  // - R[w,q] L[p,q]^T
                mma_tile<LD, LD, false, true, true>(acc, sB, w * kT, q * kT, sS, p * kT, q * kT, kT);
            acc_store_lds<LD>(acc, sB, w * kT, p * kT);
            d4 out = {0.0, 0.0, 0.0, 0.0};  // Y Dinv_p^T
            mma_tile<LD, kLDI, false, true, false>(out, sB, w * kT, p * kT, sInv[p], 0, 0, kT);
            acc_store_lds<LD>(out, sB, w * kT, p * kT);
        }
    }
    if (has_l) {
#pragma unroll
        for (int p = 0; p < W; ++p) {
            d4 acc;
            acc_load_lds<LD>(acc, sD, p * kT, w * kT);
#pragma unroll
            for (int q = 0; q < p; ++q)  // - L[p,q] T[q,w]
                mma_tile<LD, LD, false, false, true>(acc, sS, p * kT, q * kT, sD, w * kT, q * kT, kT);
            acc_store_lds<LD>(acc, sD, p * kT, w * kT);
            d4 out = {0.0, 0.0, 0.0, 0.0};  // Dinv_p Y
            mma_tile<kLDI, LD, false, false, false>(out, sInv[p], 0, 0, sD, w * kT, p * kT, kT);
            acc_store_lds<LD>(out, sD, p * kT, w * kT);
        }
    }
    __syncthreads();

    // P6: separator update S_{i+s} -= R R^T, fill -R T, stores
    if (has_r) {
#pragma unroll
        for (int t = 0; t < Cfg::TPW; ++t) {
            const int k = w + W * t;
            if (k < Cfg::NTRI) {
                int ta, tb;
                tri_tile(k, ta, tb);
                d4 acc;
                acc_load_lds<LD>(acc, sC, ta * kT, tb * kT);
                mma_tile<LD, LD, false, true, true>(acc, sB, ta * kT, 0, sB, tb * kT, 0, NP);
                acc_store_global(acc, P.Ld + (size_t)pr * nn, n, ta * kT, tb * kT);
            }
        }
    }
    if (has_r && has_l) {
        const int64_t lft = i - s, rgt = i + s;
        double* dst = (((lft >> (lvl + 1)) & 1) != 0) ? P.Rb + (size_t)perm_pos(N, lvl + 1, lft) * nn
                                                      : P.Tb + (size_t)perm_pos(N, lvl + 1, rgt) * nn;
#pragma unroll
        for (int t = 0; t < W; ++t) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            mma_tile<LD, LD, false, false, true>(acc, sB, w * kT, 0, sD, t * kT, 0, NP);
            acc_store_global(acc, dst, n, w * kT, t * kT);
        }
    }
    lds_store<NP>(P.Ld + (size_t)pi * nn, sS, n, true, tid, NT);
    if (has_r) lds_store<NP>(P.Rb + (size_t)pi * nn, sB, n, false, tid, NT);
    if (has_l) lds_store<NP>(P.Tb + (size_t)pi * nn, sD, n, false, tid, NT);
}

}  // namespace

hipError_t launch_factor_mfma(const Launch<FactorDesc>& p, int np, int64_t items, hipStream_t st) {
    const dim3 g((unsigned)items);
    switch (np) {
        case 16: hipLaunchKernelGGL(k_factor_level_mfma<16>, g, dim3(MfmaCfg<16>::NT), 0, st, p); break;
        case 32: hipLaunchKernelGGL(k_factor_level_mfma<32>, g, dim3(MfmaCfg<32>::NT), 0, st, p); break;
        case 64: hipLaunchKernelGGL(k_factor_level_mfma<64>, g, dim3(MfmaCfg<64>::NT), 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace btc
