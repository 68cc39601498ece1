// Device-side helpers shared by the libbtc kernels (gfx950, wave64).
//
// Storage conventions of the library (all blocks row-major, unpadded n x n
// in HBM):
//   * the factor lives in three arrays Ld, Rb, Tb of N blocks each, indexed
//     by the PERMUTED position p of a block in the multi-stage order (all odd
//     blocks, then odd multiples of 2, ...; section "Multi-Stage
//     Permutation").  Level l (stride s = 2^l) occupies the contiguous range
//     [N - (N >> l), N - (N >> (l+1))), and block i = s(2k+1) of that level
//     sits at p = N - (N >> l) + k.
//   * Ld[p] first holds the running Schur complement S_i of the block and is
//     overwritten by L_ii when block i is eliminated; Rb[p] / Tb[p] first hold
//     the right / left coupling of block i at its level and are overwritten by
//     R_i = C_{i+s,i} L_ii^{-T} and T_i = L_ii^{-1} C_{i,i-s}.
//   * inside a kernel, blocks are staged in LDS padded to NP x NP (NP >= n,
//     a multiple of 8) with row stride NP+1 doubles, so that a wavefront
//     reading one column hits 32 distinct banks.  Padding is the identity on
//     diagonal blocks and zero on couplings, which decouples the padded
//     coordinates from the real ones.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btc {

constexpr int kWave = 64;

// Permuted position of 1-based block i (level lvl = ctz(i)) in an instance of
// N blocks.
__host__ __device__ __forceinline__ int64_t perm_pos(int64_t N, int lvl, int64_t i) {
    return N - (N >> lvl) + (i >> (lvl + 1));
}

__host__ __device__ __forceinline__ int level_of(int64_t i) {
    return __builtin_ctzll((unsigned long long)i);
}

// Buffer-resource access to one block of at most 1 GiB: every offset is
// range checked against the block's size, so a load at or past the end reads
// 0 and a store there is dropped, without touching memory.  Masking by
// offset (kOob) keeps masked loads and stores free of branches and out of
// the flat address space (whose waits also cover LDS traffic).
constexpr int kOob = 0x40000000;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ void buf_ld(double& x, __amdgpu_buffer_rsrc_t r, int off) {
    x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_ld(float& x, __amdgpu_buffer_rsrc_t r, int off) {
    x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(double x, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(float x, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, off, 0, 0);
}
// Element (r, c) of an n x n row-major block of S: byte offset, or kOob
// when not `ok`.
template <class S>
__device__ __forceinline__ int elem_off(int r, int c, int n, bool ok) {
    return ok ? (r * n + c) * (int)sizeof(S) : kOob;
}
template <class S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t nn_rsrc(const S* p, int n) {
    return block_rsrc(p, n * n * (int)sizeof(S));
}

// Index of the calling wavefront in its workgroup, as a wave-uniform
// (scalar) value: work selected by it then keeps its addresses and buffer
// resources in scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave); }

// Broadcast a double from lane `lane` (wave-uniform) to the whole wavefront.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Order LDS traffic of one wavefront (LDS executes a wave's operations in
// issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage an n x n row-major block from global memory into an NP x NP LDS tile
// (row stride NP+1).  lower_only: read only c <= r (the upper part becomes 0).
// Padding: pad_diag on the diagonal, 0 elsewhere.  Threads [t0, t0+nt) take
// part; consecutive threads read consecutive columns of a row.
template <int NP>
__device__ __forceinline__ void lds_load(double* __restrict__ dst, const double* __restrict__ src,
                                         int n, bool lower_only, double pad_diag, int t, int nt) {
    for (int idx = t; idx < NP * NP; idx += nt) {
        const int r = idx / NP, c = idx % NP;
        double v;
        if (r < n && c < n)
            v = (!lower_only || c <= r) ? src[(size_t)r * n + c] : 0.0;
        else
            v = (r == c) ? pad_diag : 0.0;
        dst[r * (NP + 1) + c] = v;
    }
}

// Batched staging of one n x n row-major block by a fixed group of NTH
// threads: fetch() issues all of the thread's global loads into registers (so
// that every load of several blocks is in flight at once), put() writes them
// to the padded LDS tile.  Same element mapping and padding as lds_load.
template <int NP, int NTH, class V = double>
struct Stage {
    static constexpr int PER = (NP * NP + NTH - 1) / NTH;
    V v[PER];

    template <class S>
    __device__ __forceinline__ void fetch(const S* __restrict__ src, int n, bool lower_only, double pad_diag, int t) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + NTH * k;
            const int r = e / NP, c = e % NP;
            V x = (V)((r == c) ? pad_diag : 0.0);
            if (e < NP * NP && r < n && c < n && (!lower_only || c <= r)) x = (V)src[(size_t)r * n + c];
            v[k] = x;
        }
    }

    __device__ __forceinline__ void put(V* __restrict__ dst, int t) const {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + NTH * k;
            if (e < NP * NP) dst[(e / NP) * (NP + 1) + e % NP] = v[k];
        }
    }
};

// Store the leading n x n part of an LDS tile of type S as type D.
template <int NP, class D, class S>
__device__ __forceinline__ void lds_store_as(D* __restrict__ dst, const S* __restrict__ src, int n, bool lower_only,
                                             int t, int nt) {
    for (int idx = t; idx < NP * NP; idx += nt) {
        const int r = idx / NP, c = idx % NP;
        if (r < n && c < n) dst[(size_t)r * n + c] = (D)((!lower_only || c <= r) ? src[r * (NP + 1) + c] : S(0));
    }
}

// Write the leading n x n part of an LDS tile to global memory
// (lower_only: the strict upper triangle is written as 0).
template <int NP>
__device__ __forceinline__ void lds_store(double* __restrict__ dst, const double* __restrict__ src,
                                          int n, bool lower_only, int t, int nt) {
    for (int idx = t; idx < NP * NP; idx += nt) {
        const int r = idx / NP, c = idx % NP;
        if (r < n && c < n) dst[(size_t)r * n + c] = (!lower_only || c <= r) ? src[r * (NP + 1) + c] : 0.0;
    }
}

// Register tiling of an NP x NP result over NT threads: a GR x GC thread
// grid, each thread owning the TM x TN elements (tr + GR*a, tc + GC*b)
// (cyclic, so that neighbouring lanes touch neighbouring LDS words and global
// addresses).
template <int NP, int NT>
struct Grid {
    static constexpr int GR = (NT >= 256) ? 16 : 8;
    static constexpr int GC = NT / GR;
    static constexpr int TM = NP / GR;
    static constexpr int TN = NP / GC;
    static_assert(GR * GC == NT, "thread grid must cover the workgroup");
    static_assert(TM * GR == NP && TN * GC == NP && TN > 0, "tile must divide the block");
};

template <int NP, int NT>
using Acc = double[Grid<NP, NT>::TM][Grid<NP, NT>::TN];

// acc[a][b] += sum_k opA(A)[r][k] * opB(B)[k][c] over LDS tiles, with
// opA(A)[r][k] = TA ? A[k][r] : A[r][k] and opB(B)[k][c] = TB ? B[c][k] : B[k][c].
template <int NP, int NT, bool TA, bool TB>
__device__ __forceinline__ void mm_acc(Acc<NP, NT>& acc,
                                       const double* __restrict__ A, const double* __restrict__ B) {
    using Gd = Grid<NP, NT>;
    constexpr int LD = NP + 1;
    const int tr = threadIdx.x / Gd::GC, tc = threadIdx.x % Gd::GC;
#pragma unroll 4
    for (int k = 0; k < NP; ++k) {
        double a[Gd::TM], b[Gd::TN];
#pragma unroll
        for (int x = 0; x < Gd::TM; ++x) {
            const int r = tr + Gd::GR * x;
            a[x] = TA ? A[k * LD + r] : A[r * LD + k];
        }
#pragma unroll
        for (int y = 0; y < Gd::TN; ++y) {
            const int c = tc + Gd::GC * y;
            b[y] = TB ? B[c * LD + k] : B[k * LD + c];
        }
#pragma unroll
        for (int x = 0; x < Gd::TM; ++x)
#pragma unroll
            for (int y = 0; y < Gd::TN; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
}

template <int NP, int NT>
__device__ __forceinline__ void tile_load(Acc<NP, NT>& acc, const double* __restrict__ S) {
    using Gd = Grid<NP, NT>;
    constexpr int LD = NP + 1;
    const int tr = threadIdx.x / Gd::GC, tc = threadIdx.x % Gd::GC;
#pragma unroll
    for (int x = 0; x < Gd::TM; ++x)
#pragma unroll
        for (int y = 0; y < Gd::TN; ++y) acc[x][y] = S[(tr + Gd::GR * x) * LD + tc + Gd::GC * y];
}

template <int NP, int NT>
__device__ __forceinline__ void tile_store_lds(const Acc<NP, NT>& acc, double* __restrict__ S) {
    using Gd = Grid<NP, NT>;
    constexpr int LD = NP + 1;
    const int tr = threadIdx.x / Gd::GC, tc = threadIdx.x % Gd::GC;
#pragma unroll
    for (int x = 0; x < Gd::TM; ++x)
#pragma unroll
        for (int y = 0; y < Gd::TN; ++y) S[(tr + Gd::GR * x) * LD + tc + Gd::GC * y] = acc[x][y];
}

// Store the leading n x n part of a register tile to a row-major global block,
// multiplied by `scale`.
template <int NP, int NT>
__device__ __forceinline__ void tile_store_global(const Acc<NP, NT>& acc, double* __restrict__ dst, int n,
                                                  double scale) {
    using Gd = Grid<NP, NT>;
    const int tr = threadIdx.x / Gd::GC, tc = threadIdx.x % Gd::GC;
#pragma unroll
    for (int x = 0; x < Gd::TM; ++x) {
        const int r = tr + Gd::GR * x;
#pragma unroll
        for (int y = 0; y < Gd::TN; ++y) {
            const int c = tc + Gd::GC * y;
            if (r < n && c < n) dst[(size_t)r * n + c] = scale * acc[x][y];
        }
    }
}

// Cholesky factorization of the lower triangle of an NP x NP LDS tile by ONE
// wavefront (NP <= 64): lane r keeps row r in registers; at step j the pivot
// is broadcast with readlane and the new column j through a wave-private LDS
// buffer, then every lane applies the rank-1 update to its row.  Writes L
// (zero strict upper part) back to the tile and 1/L_jj to invd.  Returns true
// when every pivot was positive (uniform across the wave).
template <int NP>
__device__ __forceinline__ bool potrf_wave(double* __restrict__ A, double* __restrict__ invd,
                                           double* __restrict__ colbuf) {
    static_assert(NP <= kWave, "one lane per row");
    constexpr int LD = NP + 1;
    const int lane = threadIdx.x & (kWave - 1);
    double a[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) a[c] = (lane < NP && c <= lane) ? A[lane * LD + c] : 0.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const double ajj = readlane_d(a[j], j);
        ok = ok && (ajj > 0.0);
        const double d = sqrt(ajj);
        const double inv = 1.0 / d;
        double l = (lane == j) ? d : a[j] * inv;
        if (lane < j) l = 0.0;
        a[j] = l;
        if (lane < NP) colbuf[lane] = l;
        wave_lds_sync();
#pragma unroll
        for (int c = j + 1; c < NP; ++c) a[c] = fma(-l, colbuf[c], a[c]);
        if (lane == 0) invd[j] = inv;
        wave_lds_sync();
    }
    if (lane < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) A[lane * LD + c] = (c <= lane) ? a[c] : 0.0;
    }
    return ok;
}

// x <- L^{-1} x for a vector held in registers by one thread (L lower
// triangular in LDS, invd = 1/diag): column-oriented forward substitution,
// so the updates of one step are independent FMAs.
template <int NP>
__device__ __forceinline__ void trsv_lower_reg(const double* __restrict__ L, const double* __restrict__ invd,
                                               double (&x)[NP]) {
    constexpr int LD = NP + 1;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        x[j] *= invd[j];
#pragma unroll
        for (int k = j + 1; k < NP; ++k) x[k] = fma(-L[k * LD + j], x[j], x[k]);
    }
}

}  // namespace btc
