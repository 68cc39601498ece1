// Tile-parallel factorization level step for large blocks (padded sizes 96
// and 128), FP64 or mixed precision.
//
// A node whose four n x n blocks no longer fit in LDS together is split over
// three launches per level (the same per-node algebra as the single-kernel
// paths, Algorithm 4):
//   K1  deferred syrk: S_i -= T'^T T' and S_{i+s} -= T''^T T'', one 256-thread
//       workgroup per 32 x 32 lower tile (panels of T' staged in LDS)
//   K2  one workgroup (8 wavefronts; 4 at padded size 128) per node: the
//       whole pivot block in LDS (FP64), blocked
//       Cholesky in 16-column panels (diagonal tiles factored and inverted by
//       one wavefront, panel and trailing updates on the matrix cores), then
//       R_i = C_{i+s,i} L_ii^{-T} and T_i = L_ii^{-1} C_{i,i-s} strip by strip
//       (one 16-row or 16-column strip per wavefront at a time, blocked
//       substitution with the inverted diagonal tiles, all products MFMA,
//       the solved tiles kept in registers as the products' B operand)
//   K4  one 256-thread workgroup per 32 x 32 tile of S_{i+s} -= R_i R_i^T
//       (lower tiles) and of the fill -R_i T_i
// In mixed precision the Schur complements and K2 stay FP64 (its solves too;
// R_i and T_i are rounded to FP32 when stored) and the products of K1 and K4
// run on FP32 matrix cores (FP32 factor storage); the BF16
// variant rounds the operands of the K1 and K4 products to BF16 (FP32
// accumulation).
#pragma once

#include "btc_device.h"
#include "btc_kernels.h"
#include "btc_tiles.h"

namespace btc {
namespace {

using namespace tiles;
constexpr unsigned long long kInfoOk = ~0ull;

template <bool MIXED>
struct Prec;

template <>
struct Prec<false> {
    using F = double;
    using Acc = d4;
    __device__ static int row(int v, int lane) { return 4 * v + (lane >> 4); }
    __device__ static Acc mma(F a, F b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static F* Lf(const FactorDesc& d) { return d.Ld; }
    __device__ static F* Rf(const FactorDesc& d) { return d.Rb; }
    __device__ static F* Tf(const FactorDesc& d) { return d.Tb; }
};

template <>
struct Prec<true> {
    using F = float;
    using Acc = f4;
    __device__ static int row(int v, int lane) { return 4 * (lane >> 4) + v; }
    __device__ static Acc mma(F a, F b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static F* Lf(const FactorDesc& d) { return d.L32; }
    __device__ static F* Rf(const FactorDesc& d) { return d.R32; }
    __device__ static F* Tf(const FactorDesc& d) { return d.T32; }
};

template <int NP>
struct TiledCfg {
    static constexpr int W32 = NP / 32;               // 32-wide tile rows
    static constexpr int NTRI32 = W32 * (W32 + 1) / 2;  // lower 32 x 32 tiles
    static constexpr int NT16 = NP / 16;              // 16-wide tiles per side
};

struct Node {
    int lvl;
    int64_t i, s, h, pi, pr, N;
    int n;
    size_t nn;
    bool has_r, has_l, def_self, def_sep;
};

__device__ __forceinline__ Node node_of(const FactorDesc& P, int lvl, int64_t kk) {
    Node d;
    d.lvl = lvl;
    d.N = P.N;
    d.n = P.n;
    d.nn = (size_t)P.n * P.n;
    d.s = (int64_t)1 << lvl;
    d.h = d.s >> 1;
    d.i = (kk * 2 + 1) << lvl;
    d.has_r = d.i + d.s <= d.N;
    d.has_l = d.i > d.s;
    d.def_self = lvl > 0 && d.i + d.h <= d.N;
    d.def_sep = lvl > 0 && d.has_r && d.i + 3 * d.h <= d.N;
    d.pi = perm_pos(d.N, lvl, d.i);
    d.pr = d.has_r ? perm_pos(d.N, level_of(d.i + d.s), d.i + d.s) : 0;
    return d;
}

// Rows [r0, r0+R) (all NP columns) of an n x n block, or when cols its
// columns [r0, r0+R) (all NP rows), zero padded: the share of thread t of
// NT in registers (buffer loads masked by offset, all issued together), then
// written to LDS as dst[r][k] or, for columns, dst[k][c] (row stride ldd).
template <int NP, int R, int NT, class F>
struct PanelRegs {
    static constexpr int TOTAL = NP * R, CNT = TOTAL / NT;
    static_assert(CNT * NT == TOTAL, "threads divide the panel");
    F v[CNT];

    // k0: first index along the panel's long side (NP of them are taken)
    template <class S>
    __device__ __forceinline__ void load(const S* __restrict__ src, int n, int r0, bool cols, int t, int k0 = 0) {
        const __amdgpu_buffer_rsrc_t rs = nn_rsrc(src, n);
#pragma unroll
        for (int u = 0; u < CNT; ++u) {
            const int e = t + NT * u;
            const int rr = cols ? k0 + e / R : r0 + e / NP, cc = cols ? r0 + e % R : k0 + e % NP;
            S x;
            buf_ld(x, rs, elem_off<S>(rr, cc, n, rr < n && cc < n));
            v[u] = (F)x;
        }
    }

    __device__ __forceinline__ void put(F* __restrict__ dst, int ldd, bool cols, int t) const {
#pragma unroll
        for (int u = 0; u < CNT; ++u) {
            const int e = t + NT * u;
            if (cols)
                dst[(e / R) * ldd + e % R] = v[u];
            else
                dst[(e / NP) * ldd + e % NP] = v[u];
        }
    }
};

template <int NP, int R, int LDD, bool COLS, int NT, class S, class F>
__device__ __forceinline__ void stage_panel(F* __restrict__ dst, const S* __restrict__ src, int n, int r0, int t) {
    PanelRegs<NP, R, NT, F> g;
    g.load(src, n, r0, COLS, t);
    g.put(dst, LDD, COLS, t);
}

// Loads in flight per thread and round when staging PER elements: the
// largest divisor of PER not above 24.
constexpr int load_chunk(int per, int c = 24) { return per % c == 0 ? c : load_chunk(per, c - 1); }

// Whole lower triangle of an n x n FP64 block into the packed lower-tile
// LDS layout (whole diagonal tiles: their strict upper part 0; identity
// padding beyond n); loads by buffer resource, masked by offset.
template <int NP, int NT>
__device__ __forceinline__ void stage_lower_packed(double* __restrict__ dst, const double* __restrict__ src, int n,
                                                   int t) {
    constexpr int TOTAL = NP * NP, PER = TOTAL / NT, CH = load_chunk(PER);
    static_assert(PER * NT == TOTAL && PER % CH == 0, "threads divide the block");
    const __amdgpu_buffer_rsrc_t rs = nn_rsrc(src, n);
#pragma unroll 1
    for (int base = 0; base < TOTAL; base += NT * CH) {
        double v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = base + t + NT * u, r = e / NP, c = e % NP;
            double x;
            buf_ld(x, rs, elem_off<double>(r, c, n, r < n && c <= r));
            v[u] = (r == c && r >= n) ? 1.0 : x;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = base + t + NT * u, r = e / NP, c = e % NP;
            if (c / kT <= r / kT) PackedLds::tile(dst, r / kT, c / kT)[(r % kT) * kLDI + c % kT] = v[u];
        }
    }
}

// Leading n x n part of a packed lower-tile LDS block to global memory as
// type D (strict upper triangle written as 0); buffer stores, the part
// beyond n dropped by offset.
template <int NP, class D>
__device__ __forceinline__ void store_lower_packed(D* __restrict__ dst, const double* __restrict__ src, int n, int t,
                                                   int nt) {
    const __amdgpu_buffer_rsrc_t rs = nn_rsrc(dst, n);
    for (int idx = t; idx < NP * NP; idx += nt) {
        const int r = idx / NP, c = idx % NP;
        const double x = c <= r ? PackedLds::tile(src, r / kT, c / kT)[(r % kT) * kLDI + c % kT] : 0.0;
        buf_st((D)x, rs, elem_off<D>(r, c, n, r < n && c < n));
    }
}

// ---------------------------------------------------------------------------
// K1: deferred syrk.  Tile number ty < NTRI32 of a node: tile of S_i; else
// tile of S_{i+s}.
template <int NP, bool MIXED, bool BF16>
__global__ __launch_bounds__(256) void k_tiled_syrk_deferred(Launch<FactorDesc> L) {
    using Pr = Prec<MIXED>;
    using F = typename Pr::F;
    using Cfg = TiledCfg<NP>;
    constexpr int LDP = 33;
    __shared__ F pa[NP * LDP];
    __shared__ F pb[NP * LDP];
    FactorDesc P;
    int lvl;
    int64_t kk;
    // the tiles of one node take consecutive numbers on one XCD (shared panels)
    const unsigned blk = xcd_local_block(), ty = blk % (2 * Cfg::NTRI32);
    fetch_item_at(L, blk / (2 * Cfg::NTRI32), P, lvl, kk);
    if (*P.info != kInfoOk || (P.flags & kFactorDeferredDone)) return;
    const Node d = node_of(P, lvl, kk);
    const bool self = (int)ty < Cfg::NTRI32;
    if (self ? !d.def_self : !d.def_sep) return;
    int a, b;
    tri_tile(self ? ty : ty - Cfg::NTRI32, a, b);
    const int64_t src_node = self ? d.i + d.h : d.i + 3 * d.h;
    const F* Tsrc = Pr::Tf(P) + (size_t)perm_pos(d.N, lvl - 1, src_node) * d.nn;
    double* S = P.Ld + (size_t)(self ? d.pi : d.pr) * d.nn;
    const int tid = threadIdx.x, w = wave_id(), lane = tid & 63;
    {
        PanelRegs<NP, 32, 256, F> ga, gb;
        ga.load(Tsrc, d.n, 32 * a, true, tid);
        gb.load(Tsrc, d.n, 32 * b, true, tid);
        ga.put(pa, LDP, true, tid);
        gb.put(pb, LDP, true, tid);
    }
    __syncthreads();
    const int sr = w >> 1, sc = w & 1;
    if (a == b && sr < sc) return;  // strictly upper sub-tile
    typename Pr::Acc acc = {};
    const int i = lane & 15, q = lane >> 4;
    if constexpr (BF16) {
        // (T^T T) tile with BF16 operands: A[r][k] = T[k][r], B[k][c] = T[k][c]
        mma_tile_bf16<LDP, LDP, true, false, false>(acc, pa, 16 * sr, 0, pb, 16 * sc, 0, NP);
    } else {
        typename Pr::Acc acc1 = {};
#pragma unroll 4
        for (int k = 0; k < NP; k += 8) {
            acc = Pr::mma(pa[(k + q) * LDP + 16 * sr + i], pb[(k + q) * LDP + 16 * sc + i], acc);
            acc1 = Pr::mma(pa[(k + 4 + q) * LDP + 16 * sr + i], pb[(k + 4 + q) * LDP + 16 * sc + i], acc1);
        }
        acc += acc1;
    }
    const __amdgpu_buffer_rsrc_t rs = nn_rsrc(S, d.n);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 32 * a + 16 * sr + Pr::row(v, lane), c = 32 * b + 16 * sc + (lane & 15);
        const int off = elem_off<double>(r, c, d.n, r < d.n && c < d.n);
        double x;
        buf_ld(x, rs, off);
        buf_st(x - (double)acc[v], rs, off);
    }
}

// ---------------------------------------------------------------------------
// K2: pivot block factorization and the two triangular solves, one
// workgroup per node (k2_waves wavefronts; twelve for launches of at most
// one node per compute unit at padded size 96).  S_i is staged in LDS and factored
// by the blocked Cholesky (which also leaves the inverted 16 x 16 diagonal
// tiles in LDS); L_ii is stored; then every wavefront solves 16-row strips
// of R_i = C_{i+s,i} L_ii^{-T} and 16-column strips of T_i = L_ii^{-1} C_{i,i-s}
// tile by tile: X_p = (C_p - sum_{q<p} X_q L_pq^T) Dinv_p^T for R (the
// transposed products for T), the solved tiles held in registers and passed
// to the matrix cores through a one-tile LDS scratch per wavefront, the
// coupling tiles read straight from HBM into the accumulator layout, two
// tiles ahead of their use.
// Wavefronts of K2 and workgroups per compute unit (measured: at padded size
// 64 four nodes of four wavefronts per CU beat five (whose register budget
// of 96 spills) and three of eight; at 96 two of eight beat three of four,
// whose strips take three rounds; at 128, one node per CU, eight wavefronts
// beat four: 16 strips in two rounds instead of four, N = 4096 level 0
// 1 492 -> 1 376 us FP64, 1 148 -> 964 us mixed).
template <int NP>
constexpr int k2_waves() { return NP >= 96 ? 8 : 4; }
// The register budget is held to the workgroups per CU (the second launch
// bound counts wavefronts per SIMD).
template <int NP>
constexpr int k2_blocks() { return NP <= 64 ? 4 : NP <= 96 ? 2 : 1; }

// A launch of at most one node per compute unit is bound by one node's
// latency, not by the throughput of nodes sharing a unit: it takes one
// wavefront per strip, so that all strips are solved in one round (padded
// size 96: twelve wavefronts, measured at N = 4096: 38 against 43 us per
// launch of the upper levels, FP64; 44 against 53 mixed; padded size 64:
// eight).
constexpr int kK2LatencyWaves = 12;
constexpr int64_t kK2LatencyItems = 256;
template <int NP>
constexpr int k2_latency_waves() { return NP == 128 ? 16 : NP == 96 ? kK2LatencyWaves : NP == 64 ? 8 : 0; }

template <int NP, bool MIXED, int NW = k2_waves<NP>(), int NB = k2_blocks<NP>()>
__global__ __launch_bounds__(NW * kWave, (NB * NW + 3) / 4) void k_tiled_potrf_trsm(Launch<FactorDesc> L) {
    using Pr = Prec<MIXED>;  // storage of the factor blocks
    using Pm = Prec<false>;  // the solves run in FP64 (latency bound: no gain from FP32)
    using F = typename Pr::F;
    using Acc = typename Pm::Acc;
    using Cfg = TiledCfg<NP>;
    constexpr int NT16 = Cfg::NT16;
    // lower tiles of S_i, then of L_ii, the strict upper part of each
    // diagonal tile holding its inverse (transposed)
    __shared__ double sS[packed_lds_elems<NP>()];
    __shared__ double invd[NP];
    // one 16 x 16 tile per wavefront: R strip tiles pass through it between
    // the row-major layout of R_i in HBM and the transposed register layout
    __shared__ double xbuf[NW][kT * kLDI];
    __shared__ int fail;
    FactorDesc P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (*P.info != kInfoOk) return;
    const Node d = node_of(P, lvl, kk);
    const int tid = threadIdx.x, w = wave_id(), lane = tid & 63;
    const int n = d.n;
    const double* src = (lvl == 0) ? P.A_diag + (size_t)(d.i - 1) * d.nn : P.Ld + (size_t)d.pi * d.nn;
    const int i = lane & 15, q4 = lane >> 4;
    // Every strip is solved as X = L^{-1} C': T strips (16 columns of T_i)
    // with C' = C_{i,i-s}, R strips transposed (R_i^T = L_ii^{-1}
    // C_{i+s,i}^T, 16 rows of R_i).  Tile p of strip t in the accumulator
    // layout: lane (c, q), register v, holds element (16p + 4v+q, 16t + c) of
    // C' or X, i.e. entry (gr, gc) below of the coupling or of R_i / T_i.
    // That layout is also the B operand of the next products, so the solved
    // tiles feed the matrix cores straight from registers.
    auto gpos = [&](bool isR, int t, int p, int v, int& gr, int& gc) {
        const int rr = Pm::row(v, lane);
        gr = isR ? kT * t + i : kT * p + rr;
        gc = isR ? kT * p + rr : kT * t + i;
    };
    // R strip tile elements in row order: lane (c, q), register v holds
    // element (16t + 4v + q, 16p + c) of R_i, so that each load or store
    // covers 16 consecutive columns of four rows
    auto rpos = [&](int t, int p, int v, int& gr, int& gc) {
        gr = kT * t + Pm::row(v, lane);
        gc = kT * p + i;
    };
    // an R strip tile from that row order into the accumulator layout (and
    // back), through the wavefront's LDS tile: element (r, c) of the R tile
    // at xb[r][c]
    double* xb = xbuf[w];
    auto rows_to_acc = [&](const Acc& raw) {
        Acc out;
#pragma unroll
        for (int v = 0; v < 4; ++v) xb[Pm::row(v, lane) * kLDI + i] = raw[v];
        wave_lds_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = xb[i * kLDI + Pm::row(v, lane)];
        wave_lds_sync();
        return out;
    };
    auto acc_to_rows = [&](const Acc& x) {
        Acc out;
#pragma unroll
        for (int v = 0; v < 4; ++v) xb[i * kLDI + Pm::row(v, lane)] = x[v];
        wave_lds_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = xb[Pm::row(v, lane) * kLDI + i];
        wave_lds_sync();
        return out;
    };
    // the coupling tile (R strips: in row order): level 0 reads the input
    // couplings (FP64), higher levels the coupling left in the output slot by
    // the previous level
    auto load_coupling = [&](bool isR, int t, int p, bool live) {
        Acc acc;
        const int64_t cblk = isR ? d.i - 1 : d.i - 2;
        const __amdgpu_buffer_rsrc_t r64 = nn_rsrc(P.A_off + (size_t)(lvl == 0 && live ? cblk : 0) * d.nn, n);
        const __amdgpu_buffer_rsrc_t rf = nn_rsrc((isR ? Pr::Rf(P) : Pr::Tf(P)) + (size_t)d.pi * d.nn, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int gr, gc;
            if (isR)
                rpos(t, p, v, gr, gc);
            else
                gpos(false, t, p, v, gr, gc);
            const bool ok = live && gr < n && gc < n;
            if (lvl == 0) {
                double x;
                buf_ld(x, r64, elem_off<double>(gr, gc, n, ok));
                acc[v] = x;
            } else {
                F x;
                buf_ld(x, rf, elem_off<F>(gr, gc, n, ok));
                acc[v] = x;
            }
        }
        return acc;
    };
    constexpr int NS = (2 * NT16 + NW - 1) / NW;  // strips per wavefront (w, w + NW, ...)
    stage_lower_packed<NP, NW * kWave>(sS, src, n, tid);
    if (tid == 0) fail = 0;
    __syncthreads();
    const bool ok = potrf_blocked<NP, kLDI, NW, PackedLds, 2>(sS, invd, nullptr, &fail, xbuf);
    if (!ok) {
        if (tid == 0) atomicMin(P.info, (unsigned long long)d.i);
        return;
    }
    store_lower_packed<NP, F>(Pr::Lf(P) + (size_t)d.pi * d.nn, sS, n, tid, NW * kWave);

#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int sidx = w + j * NW;
        if (sidx >= 2 * NT16) break;
        const bool isR = sidx < NT16;
        const int t = isR ? sidx : sidx - NT16;
        if (isR ? !d.has_r : !d.has_l) continue;
        const __amdgpu_buffer_rsrc_t rdst = nn_rsrc((isR ? Pr::Rf(P) : Pr::Tf(P)) + (size_t)d.pi * d.nn, n);
        Acc X[NT16];
        // the couplings of the next two tiles are in flight while this one
        // is solved (the solved tiles are stored after the strip, so no
        // store sits between a load and its wait)
        Acc nx0 = load_coupling(isR, t, 0, true), nx1 = {};
        if (NT16 > 1) nx1 = load_coupling(isR, t, 1, true);
#pragma unroll
        for (int p = 0; p < NT16; ++p) {
            Acc acc = isR ? rows_to_acc(nx0) : nx0;
            nx0 = nx1;
            if (p + 2 < NT16) nx1 = load_coupling(isR, t, p + 2, true);
            // acc -= L_p,qq X_qq (A from LDS, B = X_qq's registers)
#pragma unroll
            for (int qq = 0; qq < p; ++qq) {
                const double* Lt = PackedLds::tile(sS, p, qq);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc = Pm::mma(-Lt[i * kLDI + 4 * v + q4], X[qq][v], acc);
            }
            // X_p = Dinv_p acc
            Acc out = {};
            // Dinv_p[i][k]: k < i in the diagonal tile's upper part (transposed), k = i in invd
            const double* Dt = PackedLds::tile(sS, p, p);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = 4 * v + q4;
                const double dv = k < i ? Dt[k * kLDI + i] : (k == i ? invd[kT * p + i] : 0.0);
                out = Pm::mma(dv, acc[v], out);
            }
            X[p] = out;
        }
#pragma unroll
        for (int p = 0; p < NT16; ++p) {
            const Acc y = isR ? acc_to_rows(X[p]) : X[p];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int gr, gc;
                if (isR)
                    rpos(t, p, v, gr, gc);
                else
                    gpos(false, t, p, v, gr, gc);
                buf_st((F)y[v], rdst, elem_off<F>(gr, gc, n, gr < n && gc < n));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K4: tile number ty < NTRI32 of a node: lower tile of S_{i+s} -= R R^T (eagerly also
// - T'^T T' with T' = T_{i+2s}, the separator's other contribution); else
// fill tile -R T (row-major over the W32 x W32 tiles).  The panels of a
// product pass through LDS in ranges of 32 along the k index (staged
// panels then hold few registers and little LDS, so more workgroups share
// a compute unit: at padded size 128, five FP64 or seven FP32 wavefronts
// per SIMD against three and four with halves or whole panels), the next range's loads
// in flight while the current one is on the matrix cores; the accumulation
// order over k is the same for any number of ranges.
template <int NP, bool MIXED, bool BF16>
__global__ __launch_bounds__(256) void k_tiled_update(Launch<FactorDesc> L) {
    using Pr = Prec<MIXED>;
    using F = typename Pr::F;
    using Cfg = TiledCfg<NP>;
    constexpr int KS = NP / 32;
    constexpr int KH = NP / KS;
    static_assert(KH % 8 == 0, "whole k steps per range");
    constexpr int LDR = KH + 1;  // row panel [32][KH]
    constexpr int LDP = 33;      // column panel [KH][32]
    constexpr int PSZ = KH * LDP > 32 * LDR ? KH * LDP : 32 * LDR;
    __shared__ F pa[PSZ];
    __shared__ F pb[PSZ];
    FactorDesc P;
    int lvl;
    int64_t kk;
    // the tiles of one node take consecutive numbers on one XCD (shared panels)
    constexpr int NTILE = Cfg::NTRI32 + Cfg::W32 * Cfg::W32;
    const unsigned blk = xcd_local_block(), ty = blk % NTILE;
    fetch_item_at(L, blk / NTILE, P, lvl, kk);
    if (*P.info != kInfoOk) return;
    const Node d = node_of(P, lvl, kk);
    const bool sep = (int)ty < Cfg::NTRI32;
    if (sep ? !d.has_r : !(d.has_r && d.has_l)) return;
    int a, b;
    if (sep) {
        tri_tile(ty, a, b);
    } else {
        a = (ty - Cfg::NTRI32) / Cfg::W32;
        b = (ty - Cfg::NTRI32) % Cfg::W32;
    }
    const int tid = threadIdx.x, w = wave_id(), lane = tid & 63;
    const int n = d.n;
    const F* R = Pr::Rf(P) + (size_t)d.pi * d.nn;
    const F* T = Pr::Tf(P) + (size_t)d.pi * d.nn;
    const int sr = w >> 1, sc = w & 1;
    const bool idle = sep && a == b && sr < sc;  // strictly upper sub-tile
    const bool eager = sep && (P.flags & kFactorEagerT) && d.i + 2 * d.s <= d.N;
    const F* T2 = Pr::Tf(P) + (size_t)(eager ? perm_pos(d.N, lvl, d.i + 2 * d.s) : d.pi) * d.nn;
    // phase ph: k range ph % KS of product ph / KS (0: R R^T or R T; 1: the
    // right neighbour's T'^T T')
    const int nph = KS * (eager ? 2 : 1);
    using Pan = PanelRegs<KH, 32, 256, F>;
    auto load_phase = [&](int ph, Pan& x, Pan& y) {
        const int k0 = KH * (ph % KS);
        if (ph < KS) {
            x.load(R, n, 32 * a, false, tid, k0);
            y.load(sep ? R : T, n, 32 * b, !sep, tid, k0);
        } else {
            x.load(T2, n, 32 * a, true, tid, k0);
            y.load(T2, n, 32 * b, true, tid, k0);
        }
    };
    typename Pr::Acc acc = {}, acc1 = {};
    const int i = lane & 15, q = lane >> 4;
    // a phase's panels into LDS
    auto stage = [&](int ph, const Pan& ca, const Pan& cb) {
        const bool second = ph >= KS;  // the T'^T T' product
        ca.put(pa, second ? LDP : LDR, second, tid);
        cb.put(pb, (second || !sep) ? LDP : LDR, second || !sep, tid);
    };
    // a phase's products from LDS
    auto products = [&](int ph) {
        if (idle) return;
        const bool second = ph >= KS;
        if constexpr (BF16) {
            if (second)
                mma_tile_bf16<LDP, LDP, true, false, false>(acc, pa, 16 * sr, 0, pb, 16 * sc, 0, KH);
            else if (sep)
                // R R^T (B[k][c] = R[c][k]) with BF16 operands
                mma_tile_bf16<LDR, LDR, false, true, false>(acc, pa, 16 * sr, 0, pb, 16 * sc, 0, KH);
            else
                // R T (B[k][c] = T[k][c])
                mma_tile_bf16<LDR, LDP, false, false, false>(acc, pa, 16 * sr, 0, pb, 16 * sc, 0, KH);
        } else {
            // two independent accumulation chains (hide the matrix-core latency)
#pragma unroll 4
            for (int k = 0; k < KH; k += 8) {
                F a0, a1, b0, b1;
                if (second) {
                    a0 = pa[(k + q) * LDP + 16 * sr + i];
                    a1 = pa[(k + 4 + q) * LDP + 16 * sr + i];
                    b0 = pb[(k + q) * LDP + 16 * sc + i];
                    b1 = pb[(k + 4 + q) * LDP + 16 * sc + i];
                } else {
                    a0 = pa[(16 * sr + i) * LDR + k + q];
                    a1 = pa[(16 * sr + i) * LDR + k + 4 + q];
                    b0 = sep ? pb[(16 * sc + i) * LDR + k + q] : pb[(k + q) * LDP + 16 * sc + i];
                    b1 = sep ? pb[(16 * sc + i) * LDR + k + 4 + q] : pb[(k + 4 + q) * LDP + 16 * sc + i];
                }
                acc = Pr::mma(a0, b0, acc);
                acc1 = Pr::mma(a1, b1, acc1);
            }
            if (ph % KS == KS - 1) {
                // end of a product: fold its second chain
                acc += acc1;
                acc1 = {};
            }
        }
    };
    // phase 0's panels first, then the Schur complement entries this thread
    // updates and the next phase's panels load while phase 0 computes; each
    // later phase stages its panels once the previous one has read them, and
    // one register set carries every phase (a set is free again once staged)
    Pan ga, gb;
    load_phase(0, ga, gb);
    stage(0, ga, gb);
    double sv[4] = {0.0, 0.0, 0.0, 0.0};
    if (sep) {
        const double* src = (lvl == 0) ? P.A_diag + (size_t)(d.i + d.s - 1) * d.nn : P.Ld + (size_t)d.pr * d.nn;
        const __amdgpu_buffer_rsrc_t rsrc = nn_rsrc(src, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * a + 16 * sr + Pr::row(v, lane), c = 32 * b + 16 * sc + (lane & 15);
            buf_ld(sv[v], rsrc, elem_off<double>(r, c, n, !idle && r < n && c < n));
        }
    }
    if (nph > 1) load_phase(1, ga, gb);
    __syncthreads();
    products(0);
#pragma unroll
    for (int ph = 1; ph < 2 * KS; ++ph) {
        if (ph >= nph) break;
        __syncthreads();  // the previous phase's products have read the panels
        stage(ph, ga, gb);
        if (ph + 1 < nph) load_phase(ph + 1, ga, gb);
        __syncthreads();
        products(ph);
    }
    if (idle) return;
    if (sep) {
        const __amdgpu_buffer_rsrc_t rs = nn_rsrc(P.Ld + (size_t)d.pr * d.nn, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * a + 16 * sr + Pr::row(v, lane), c = 32 * b + 16 * sc + (lane & 15);
            buf_st(sv[v] - (double)acc[v], rs, elem_off<double>(r, c, n, r < n && c < n));
        }
    } else {
        const int64_t lft = d.i - d.s, rgt = d.i + d.s;
        F* dst = (((lft >> (lvl + 1)) & 1) != 0) ? Pr::Rf(P) + (size_t)perm_pos(d.N, lvl + 1, lft) * d.nn
                                                 : Pr::Tf(P) + (size_t)perm_pos(d.N, lvl + 1, rgt) * d.nn;
        const __amdgpu_buffer_rsrc_t rd = nn_rsrc(dst, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * a + 16 * sr + Pr::row(v, lane), c = 32 * b + 16 * sc + (lane & 15);
            buf_st(-acc[v], rd, elem_off<F>(r, c, n, r < n && c < n));
        }
    }
}

// part 0: the whole level step; 1, 2, 3: only K1, K2, K4 (for per-kernel
// timing; launched in that order they make up the step)
template <int NP, bool MIXED, bool BF16>
hipError_t launch_tiled_np(const Launch<FactorDesc>& p, int part, bool deferred, int64_t items, hipStream_t st) {
    using Cfg = TiledCfg<NP>;
    const unsigned g = (unsigned)items;
    if ((part == 0 || part == 1) && deferred)
        hipLaunchKernelGGL((k_tiled_syrk_deferred<NP, MIXED, BF16>), dim3(g * 2 * Cfg::NTRI32), dim3(256), 0, st, p);
    if (part == 0 || part == 2) {
        bool done = false;
        constexpr int LW = k2_latency_waves<NP>();
        if constexpr (LW > 0) {
            if (items <= kK2LatencyItems) {
                hipLaunchKernelGGL((k_tiled_potrf_trsm<NP, MIXED, LW, 1>), dim3(g), dim3(LW * kWave), 0, st, p);
                done = true;
            }
        }
        if (!done)
            hipLaunchKernelGGL((k_tiled_potrf_trsm<NP, MIXED>), dim3(g), dim3(k2_waves<NP>() * kWave), 0, st, p);
    }
    if (part == 0 || part == 3)
        hipLaunchKernelGGL((k_tiled_update<NP, MIXED, BF16>), dim3(g * (Cfg::NTRI32 + Cfg::W32 * Cfg::W32)), dim3(256),
                           0, st, p);
    return hipGetLastError();
}

}  // namespace

// Per padded size launchers (one translation unit each).
// mode: 0 FP64, 1 mixed (FP32 products), 2 mixed with BF16 Schur / fill products
hipError_t launch_factor_tiled32(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                 hipStream_t st);
hipError_t launch_factor_tiled64(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                 hipStream_t st);
hipError_t launch_factor_tiled96(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                 hipStream_t st);
hipError_t launch_factor_tiled128(const Launch<FactorDesc>& p, int mode, int part, bool deferred, int64_t items,
                                  hipStream_t st);

}  // namespace btc
