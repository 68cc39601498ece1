// FP64 factorization level kernel on the vector ALUs (block sizes n <= 8,
// and n <= 32 where the autotuner prefers it to the matrix-core kernel): one
// workgroup per block (node) of one level of the multi-stage elimination
// tree.
//
// Factorization (section "Multi-Stage Permutation", Algorithm 4, the hybrid
// left/right-looking form): at level l (stride s) node i
//   1. applies the Schur update deferred from level l-1 by its right child:
//        S_i     -= T_{i+s/2}^T T_{i+s/2}            (if l > 0, i+s/2 <= N)
//   2. L_ii = chol(S_i)                               (potrf)
//   3. R_i = C_{i+s,i} L_ii^{-T}, T_i = L_ii^{-1} C_{i,i-s}   (two trsm)
//   4. updates the separator it owns (its right neighbour), first with the
//      update deferred from level l-1, then with its own right-looking one:
//        S_{i+s} -= T_{i+3s/2}^T T_{i+3s/2}  (if l > 0, i+3s/2 <= N)
//        S_{i+s} -= R_i R_i^T
//   5. writes the fill-in coupling of level l+1:  C_{i+s,i-s} = -R_i T_i.
// Every separator has exactly one owner per level, so no two workgroups of a
// launch write the same block and the result is deterministic (no atomics).
//
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {

static constexpr unsigned long long kInfoOk = ~0ull;

// Threads per workgroup: one wavefront for NP <= 16; for larger blocks extra
// wavefronts stage the couplings while wavefront 0 factors the pivot block.
template <int NP>
struct F64Cfg {
    static constexpr int NT = (NP >= 64) ? 256 : (NP >= 32 ? 128 : 64);
};

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_factor_level_f64(Launch<FactorDesc> L) {
    constexpr int LD = NP + 1;
    static_assert(NT >= 2 * NP, "one thread per trsm vector");
    __shared__ double sA[NP * LD];  // S_i -> L_ii
    __shared__ double sB[NP * LD];  // deferred T' -> C_{i+s,i} -> R_i
    __shared__ double sC[NP * LD];  // S_{i+s}
    __shared__ double sD[NP * LD];  // deferred T'' -> C_{i,i-s} -> T_i
    __shared__ double invd[NP];
    __shared__ double colbuf[kWave];
    __shared__ int fail;

    FactorDesc P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (*P.info != kInfoOk) return;  // an earlier level broke down

    const int tid = threadIdx.x;
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

    // 1. stage S_i, S_{i+s} and the two deferred T blocks (all loads in flight)
    {
        Stage<NP, NT> a, b, c, d;
        a.fetch(lvl == 0 ? P.A_diag + (size_t)(i - 1) * nn : P.Ld + (size_t)pi * nn, n, true, 1.0, tid);
        if (def_self) b.fetch(P.Tb + (size_t)perm_pos(N, lvl - 1, i + h) * nn, n, false, 0.0, tid);
        if (has_r)
            c.fetch(lvl == 0 ? P.A_diag + (size_t)(i + s - 1) * nn : P.Ld + (size_t)pr * nn, n, true, 1.0, tid);
        if (def_sep) d.fetch(P.Tb + (size_t)perm_pos(N, lvl - 1, i + 3 * h) * nn, n, false, 0.0, tid);
        a.put(sA, tid);
        if (def_self) b.put(sB, tid);
        if (has_r) c.put(sC, tid);
        if (def_sep) d.put(sD, tid);
    }
    if (tid == 0) fail = 0;
    __syncthreads();

    // deferred (left-looking) syrk updates
    using GridT = Grid<NP, NT>;
    if (def_self) {
        Acc<NP, NT> acc;
        tile_load<NP, NT>(acc, sA);
        Acc<NP, NT> t = {};
        mm_acc<NP, NT, true, false>(t, sB, sB);
#pragma unroll
        for (int x = 0; x < GridT::TM; ++x)
#pragma unroll
            for (int y = 0; y < GridT::TN; ++y) acc[x][y] -= t[x][y];
        tile_store_lds<NP, NT>(acc, sA);
    }
    if (def_sep) {
        Acc<NP, NT> acc;
        tile_load<NP, NT>(acc, sC);
        Acc<NP, NT> t = {};
        mm_acc<NP, NT, true, false>(t, sD, sD);
#pragma unroll
        for (int x = 0; x < GridT::TM; ++x)
#pragma unroll
            for (int y = 0; y < GridT::TN; ++y) acc[x][y] -= t[x][y];
        tile_store_lds<NP, NT>(acc, sC);
    }
    __syncthreads();

    // 2. potrf on wave 0 while the other waves stage the couplings
    const double* Cr = (lvl == 0) ? P.A_off + (size_t)(i - 1) * nn : P.Rb + (size_t)pi * nn;
    const double* Cl = (lvl == 0) ? P.A_off + (size_t)(i - 2) * nn : P.Tb + (size_t)pi * nn;
    if constexpr (NT > kWave) {
        if (tid < kWave) {
            const bool ok = potrf_wave<NP>(sA, invd, colbuf);
            if (!ok && tid == 0) fail = 1;
        } else {
            Stage<NP, NT - kWave> cr, cl;
            if (has_r) cr.fetch(Cr, n, false, 0.0, tid - kWave);
            if (has_l) cl.fetch(Cl, n, false, 0.0, tid - kWave);
            if (has_r) cr.put(sB, tid - kWave);
            if (has_l) cl.put(sD, tid - kWave);
        }
        __syncthreads();
    } else {
        // a single wavefront: issue the coupling loads first, factor while they fly
        Stage<NP, NT> cr, cl;
        if (has_r) cr.fetch(Cr, n, false, 0.0, tid);
        if (has_l) cl.fetch(Cl, n, false, 0.0, tid);
        const bool ok = potrf_wave<NP>(sA, invd, colbuf);
        if (!ok && tid == 0) fail = 1;
        if (has_r) cr.put(sB, tid);
        if (has_l) cl.put(sD, tid);
        __syncthreads();
    }
    if (fail) {
        if (tid == 0) atomicMin(P.info, (unsigned long long)i);
        return;
    }

    // 3. two trsm: thread v < NP solves row v of R (R^T = L^{-1} C_r^T),
    //    NP <= v < 2NP column v-NP of T (T = L^{-1} C_l); same recurrence.
    {
        const bool do_r = tid < NP && has_r;
        const bool do_l = tid >= NP && tid < 2 * NP && has_l;
        if (do_r || do_l) {
            double* base = do_r ? sB + tid * LD : sD + (tid - NP);
            const int stride = do_r ? 1 : LD;
            double x[NP];
#pragma unroll
            for (int c = 0; c < NP; ++c) x[c] = base[c * stride];
            trsv_lower_reg<NP>(sA, invd, x);
#pragma unroll
            for (int c = 0; c < NP; ++c) base[c * stride] = x[c];
        }
    }
    __syncthreads();

    // 4./5. separator update and fill-in, straight from registers to HBM
    if (has_r) {
        Acc<NP, NT> acc;
        tile_load<NP, NT>(acc, sC);
        Acc<NP, NT> t = {};
        mm_acc<NP, NT, false, true>(t, sB, sB);
#pragma unroll
        for (int x = 0; x < GridT::TM; ++x)
#pragma unroll
            for (int y = 0; y < GridT::TN; ++y) acc[x][y] -= t[x][y];
        tile_store_global<NP, NT>(acc, P.Ld + (size_t)pr * nn, n, 1.0);
    }
    if (has_r && has_l) {
        Acc<NP, NT> t = {};
        mm_acc<NP, NT, false, false>(t, sB, sD);
        const int64_t lft = i - s, rgt = i + s;
        double* dst = (((lft >> (lvl + 1)) & 1) != 0) ? P.Rb + (size_t)perm_pos(N, lvl + 1, lft) * nn
                                                      : P.Tb + (size_t)perm_pos(N, lvl + 1, rgt) * nn;
        tile_store_global<NP, NT>(t, dst, n, -1.0);
    }
    lds_store<NP>(P.Ld + (size_t)pi * nn, sA, n, true, tid, NT);
    if (has_r) lds_store<NP>(P.Rb + (size_t)pi * nn, sB, n, false, tid, NT);
    if (has_l) lds_store<NP>(P.Tb + (size_t)pi * nn, sD, n, false, tid, NT);
}

// ---------------------------------------------------------------------------
// Host-side launchers (one per level).

int padded_block(int n) {
    if (n <= 8) return 8;
    if (n <= 16) return 16;
    if (n <= 32) return 32;
    if (n <= 64) return 64;
    if (n <= 96) return 96;
    if (n <= 128) return 128;
    return 0;
}

hipError_t launch_factor_valu(const Launch<FactorDesc>& p, int np, int64_t items, hipStream_t st) {
    const dim3 g((unsigned)items);
    switch (np) {
        case 8: hipLaunchKernelGGL((k_factor_level_f64<8, F64Cfg<8>::NT>), g, dim3(F64Cfg<8>::NT), 0, st, p); break;
        case 16: hipLaunchKernelGGL((k_factor_level_f64<16, F64Cfg<16>::NT>), g, dim3(F64Cfg<16>::NT), 0, st, p); break;
        case 32: hipLaunchKernelGGL((k_factor_level_f64<32, F64Cfg<32>::NT>), g, dim3(F64Cfg<32>::NT), 0, st, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace btc
