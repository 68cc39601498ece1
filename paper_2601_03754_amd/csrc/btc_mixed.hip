// Mixed-precision factorization level kernel (padded block sizes 16, 32, 64).
//
// Same elimination as the FP64 kernels (Algorithm 4, deterministic
// ownership of the separators), with the arithmetic split by precision:
//   * the running Schur complements S_j stay FP64 in HBM and in LDS, and the
//     Cholesky factorization of every pivot block runs in FP64;
//   * the factor blocks are rounded to FP32: L_ii (for the sweeps), R_i, T_i
//     and the fill-in couplings;
//   * the triangular solves and the Schur/fill products run on FP32 matrix
//     cores (v_mfma_f32_16x16x4f32, FP32 accumulation); each FP32 Schur
//     product is subtracted into the FP64 block it updates;
//   * BF16 variant: the Schur/fill products (syrk, gemm) take BF16 operands
//     rounded to nearest even (v_mfma_f32_16x16x32_bf16, FP32 accumulation);
//     the triangular solves stay FP32.
// The accuracy lost to FP32 is won back by FP64 iterative refinement of the
// solution (residual computed in FP64 from the original blocks).
#include "btc_device.h"
#include "btc_kernels.h"
#include "btc_tiles.h"

namespace btc {
namespace {

using namespace tiles;
constexpr unsigned long long kInfoOk = ~0ull;

template <int NP>
struct MixCfg {
    static constexpr int W = NP / kT;
    static constexpr int NT = W * kWave;
    static constexpr int NTRI = W * (W + 1) / 2;
    static constexpr int TPW = (NTRI + W - 1) / W;
};

// Store the elements of FP64 LDS tile (r0, c0) that lane holds in the FP32
// accumulator layout.
template <int LD>
__device__ __forceinline__ void tile64_store_global_acc32(const double* __restrict__ S, double* __restrict__ dst,
                                                          int n, int r0, int c0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + acc32_r(v, lane), c = c0 + acc_c(lane);
        if (r < n && c < n) dst[(size_t)r * n + c] = S[r * LD + c];
    }
}

template <int NP, bool BF16>
__global__ __launch_bounds__(MixCfg<NP>::NT) void k_factor_level_mixed(Launch<FactorDesc> L) {
    using Cfg = MixCfg<NP>;
    constexpr int W = Cfg::W, NT = Cfg::NT, LD = NP + 1;
    __shared__ double sS[NP * LD];  // S_i -> L_ii (FP64)
    __shared__ double sC[NP * LD];  // S_{i+s} (FP64)
    __shared__ float fB[NP * LD];   // T' -> C_{i+s,i} -> R_i
    __shared__ float fD[NP * LD];   // T'' -> C_{i,i-s} -> T_i
    __shared__ float fL[NP * LD];   // L_ii rounded to FP32
    __shared__ float fInv[W][kT * kLDI];
    __shared__ double sInv[W][kT * kLDI];  // inverted diagonal tiles (FP64, W = NP/16)
    __shared__ double invd[NP];
    __shared__ int fail;

    FactorDesc P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (*P.info != kInfoOk) return;

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

    // P1: stage S_i, S_{i+s} (FP64) and the deferred T blocks (FP32)
    {
        Stage<NP, NT> a, c;
        Stage<NP, NT, float> b, d;
        a.fetch(lvl == 0 ? P.A_diag + (size_t)(i - 1) * nn : P.Ld + (size_t)pi * nn, n, true, 1.0, tid);
        if (def_self) b.fetch(P.T32 + (size_t)perm_pos(N, lvl - 1, i + h) * nn, n, false, 0.0, tid);
        if (has_r) c.fetch(Ssep, n, true, 1.0, tid);
        if (def_sep) d.fetch(P.T32 + (size_t)perm_pos(N, lvl - 1, i + 3 * h) * nn, n, false, 0.0, tid);
        a.put(sS, tid);
        if (def_self) b.put(fB, tid);
        if (has_r) c.put(sC, tid);
        if (def_sep) d.put(fD, tid);
    }
    if (tid == 0) fail = 0;
    __syncthreads();

    // coupling loads (FP32) go out now and land in LDS after P2
    Stage<NP, NT, float> cr, cl;
    if (lvl == 0) {
        cr.fetch(P.A_off + (size_t)(i - 1) * nn, has_r ? n : 0, false, 0.0, tid);
        cl.fetch(P.A_off + (size_t)(i - 2) * nn, has_l ? n : 0, false, 0.0, tid);
    } else {
        cr.fetch(P.R32 + (size_t)pi * nn, has_r ? n : 0, false, 0.0, tid);
        cl.fetch(P.T32 + (size_t)pi * nn, has_l ? n : 0, false, 0.0, tid);
    }

    // P2: deferred syrk updates in FP32, subtracted into the FP64 blocks
#pragma unroll
    for (int t = 0; t < Cfg::TPW; ++t) {
        const int k = w + W * t;
        if (k < Cfg::NTRI) {
            int ta, tb;
            tri_tile(k, ta, tb);
            if (def_self) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                mma_prod<BF16, LD, LD, true, false, false>(acc, fB, ta * kT, 0, fB, tb * kT, 0, NP);
                acc32_sub_from_lds64<LD>(acc, sS, ta * kT, tb * kT);
            }
            if (def_sep) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                mma_prod<BF16, LD, LD, true, false, false>(acc, fD, ta * kT, 0, fD, tb * kT, 0, NP);
                acc32_sub_from_lds64<LD>(acc, sC, ta * kT, tb * kT);
            }
        }
    }
    __syncthreads();

    // P3: couplings to LDS; blocked FP64 Cholesky of S_i by all wavefronts
    cr.put(fB, tid);
    cl.put(fD, tid);
    const bool ok = potrf_blocked<NP, LD, W>(sS, invd, sInv, &fail);
    if (!ok) {
        if (tid == 0) atomicMin(P.info, (unsigned long long)i);
        return;
    }

    // P4: L_ii and the inverted diagonal tiles rounded to FP32
    for (int idx = tid; idx < NP * NP; idx += NT) {
        const int r = idx / NP, c = idx % NP;
        fL[r * LD + c] = (float)sS[r * LD + c];
    }
    for (int idx = tid; idx < W * kT * kLDI; idx += NT) fInv[idx / (kT * kLDI)][idx % (kT * kLDI)] =
        (float)sInv[idx / (kT * kLDI)][idx % (kT * kLDI)];
    __syncthreads();

    // P5: blocked FP32 triangular solves (wavefront w: tile-row w of R,
    // tile-column w of T)
    if (has_r) {
#pragma unroll
        for (int p = 0; p < W; ++p) {
            f4 acc;
            acc32_load_lds<LD>(acc, fB, w * kT, p * kT);
#pragma unroll
            for (int q = 0; q < p; ++q)
                mma_tile32<LD, LD, false, true, true>(acc, fB, w * kT, q * kT, fL, p * kT, q * kT, kT);
            acc32_store_lds<LD>(acc, fB, w * kT, p * kT);
            f4 out = {0.f, 0.f, 0.f, 0.f};
            mma_tile32<LD, kLDI, false, true, false>(out, fB, w * kT, p * kT, fInv[p], 0, 0, kT);
            acc32_store_lds<LD>(out, fB, w * kT, p * kT);
        }
    }
    if (has_l) {
#pragma unroll
        for (int p = 0; p < W; ++p) {
            f4 acc;
            acc32_load_lds<LD>(acc, fD, p * kT, w * kT);
#pragma unroll
            for (int q = 0; q < p; ++q)
                mma_tile32<LD, LD, false, false, true>(acc, fL, p * kT, q * kT, fD, w * kT, q * kT, kT);
            acc32_store_lds<LD>(acc, fD, p * kT, w * kT);
            f4 out = {0.f, 0.f, 0.f, 0.f};
            mma_tile32<kLDI, LD, false, false, false>(out, fInv[p], 0, 0, fD, w * kT, p * kT, kT);
            acc32_store_lds<LD>(out, fD, p * kT, w * kT);
        }
    }
    __syncthreads();

    // P6: S_{i+s} -= R R^T (FP32 product into the FP64 block), fill -R T
    if (has_r) {
#pragma unroll
        for (int t = 0; t < Cfg::TPW; ++t) {
            const int k = w + W * t;
            if (k < Cfg::NTRI) {
                int ta, tb;
                tri_tile(k, ta, tb);
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                mma_prod<BF16, LD, LD, false, true, false>(acc, fB, ta * kT, 0, fB, tb * kT, 0, NP);
                acc32_sub_from_lds64<LD>(acc, sC, ta * kT, tb * kT);
                tile64_store_global_acc32<LD>(sC, P.Ld + (size_t)pr * nn, n, ta * kT, tb * kT);
            }
        }
    }
    if (has_r && has_l) {
        const int64_t lft = i - s, rgt = i + s;
        float* dst = (((lft >> (lvl + 1)) & 1) != 0) ? P.R32 + (size_t)perm_pos(N, lvl + 1, lft) * nn
                                                     : P.T32 + (size_t)perm_pos(N, lvl + 1, rgt) * nn;
#pragma unroll
        for (int t = 0; t < W; ++t) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            mma_prod<BF16, LD, LD, false, false, true>(acc, fB, w * kT, 0, fD, t * kT, 0, NP);
            acc32_store_global(acc, dst, n, w * kT, t * kT);
        }
    }
    lds_store_as<NP, float, float>(P.L32 + (size_t)pi * nn, fL, n, true, tid, NT);
    if (has_r) lds_store_as<NP, float, float>(P.R32 + (size_t)pi * nn, fB, n, false, tid, NT);
    if (has_l) lds_store_as<NP, float, float>(P.T32 + (size_t)pi * nn, fD, n, false, tid, NT);
}

}  // namespace

// Padded tile of the mixed kernels: at least one 16 x 16 matrix-core tile.
int padded_block_mixed(int n) {
    const int np = padded_block(n);
    return (np != 0 && np < 16) ? 16 : np;
}

hipError_t launch_factor_mixed(const Launch<FactorDesc>& p, int np, bool bf16, int64_t items, hipStream_t st) {
    const dim3 g((unsigned)items);
    switch (np) {
        case 16:
            if (bf16) hipLaunchKernelGGL((k_factor_level_mixed<16, true>), g, dim3(MixCfg<16>::NT), 0, st, p);
            else hipLaunchKernelGGL((k_factor_level_mixed<16, false>), g, dim3(MixCfg<16>::NT), 0, st, p);
            break;
        case 32:
            if (bf16) hipLaunchKernelGGL((k_factor_level_mixed<32, true>), g, dim3(MixCfg<32>::NT), 0, st, p);
            else hipLaunchKernelGGL((k_factor_level_mixed<32, false>), g, dim3(MixCfg<32>::NT), 0, st, p);
            break;
        case 64:
            if (bf16) hipLaunchKernelGGL((k_factor_level_mixed<64, true>), g, dim3(MixCfg<64>::NT), 0, st, p);
            else hipLaunchKernelGGL((k_factor_level_mixed<64, false>), g, dim3(MixCfg<64>::NT), 0, st, p);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace btc
