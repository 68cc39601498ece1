// Level sweeps of the solve (section "Cholesky Solve", Algorithm 6) and the
// FP64 residual b - Psi x, streaming form: one wavefront per node (per block
// row for the residual), every n x n block read from HBM once and coalesced.
//
// Lane r owns rows r and r + 64 of the node's vectors (columns of the
// right-hand side are processed MC at a time, MC independent chains).  Every
// block goes through LDS in slabs of 16 columns (each row contributes one
// contiguous 16-element segment, written transposed) or 16 rows (contiguous),
// laid out so that lane r reads slab[k][r] conflict-free whichever of
// M[r][c] or M[c][r] the product needs.  The global loads of slab p+1 (NP/4
// per lane, held in registers) are in flight while slab p is consumed from
// LDS, so the triangular solves' dependency chains overlap the block
// traffic; with one wavefront per workgroup and one slab buffer (at most
// 16.5 KB), many nodes share each compute unit.
//
//   forward, node i of level l (stride s), levels ascending:
//     y_i = L_ii^{-1} (b_i - sum of the u / v its descendants left for it)
//         [column slabs of L_ii, column sweep, pivots broadcast by readlane]
//     u_i = R_i y_i   [column slabs of R_i]   (pulled by node i+s)
//     v_i = T_i^T y_i [row slabs of T_i]      (pulled by node i-s)
//   backward, levels descending:
//     x_i = L_ii^{-T} (y_i - R_i^T x_{i+s} - T_i x_{i-s})
//         [R_i row slabs; T_i column slabs; L_ii row slabs consumed from the
//          last row up]
//   residual, block row i: r_i = b_i - D_i x_i - E_{i-1} x_{i-1} - E_i^T x_{i+1}
//     [row slabs of the lower triangle of D_i and of E_i, each element used
//      for its own row and, through a wavefront sum, for its transpose's;
//      E_i x_i is left for row i+1]; then per-column partial squared norms
//     of r_i and b_i.
// Instead of two nodes subtracting into the same y concurrently, each node
// pulls its contributions in a fixed order: results are deterministic.
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc {
namespace {

constexpr unsigned long long kInfoOk = ~0ull;
constexpr int kS = 16;  // slab width

__device__ __forceinline__ double bcast(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }

template <int NP>
struct Geo {
    static_assert(NP % kS == 0, "padded size is a multiple of the slab width");
    static constexpr int RPL = (NP + kWave - 1) / kWave;  // rows per lane
    static constexpr int LDB = NP + 1;                    // slab stride (elements)
    // lanes past the last row (r >= NP) read past the end of the last slab
    // row: the buffer is long enough for them (their values are never used)
    static constexpr int BUF = kS * LDB + kWave * RPL - NP;
    static constexpr int PER = NP * kS / kWave;           // slab elements per lane
    // row slab element u of a lane: pattern u % RP (row, column) of the first
    // RP elements, moved down by (u / RP) * RK rows
    static constexpr int RP = NP / gcd_i(NP, kWave);
    static constexpr int RK = kWave / gcd_i(NP, kWave);
};

// Slab loads go through buffer resources (block_rsrc): rows and columns
// beyond n and the skipped parts are masked by offset.

// Where the next slab comes from: column slab (elements M[r][c0+k], rows
// r >= rmin) or row slab (elements M[r0+k][r], only r <= r0+k when tri).
template <class S>
struct SlabSrc {
    const S* M;
    int off;
    int rmin;
    bool rows;
    bool tri;
};

template <int NP, class T>
struct SlabRegs {
    T v[Geo<NP>::PER];

    // Column slab: lane (q, k) = (lane / 16, lane % 16) reads rows q + 4u
    // of column off + k, every offset a lane constant plus 4un.  Row slab:
    // lanes read along the rows (pattern offsets of Geo).  Both skip what the
    // triangular blocks do not use (column slab: the rows above rmin, a
    // whole element index at a time; row slab: columns past the slab's last
    // row).
    template <class S>
    __device__ __forceinline__ void fetch(const SlabSrc<S>& s, int n, int lane) {
        using G = Geo<NP>;
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(s.M, n * n * (int)sizeof(S));
        if (!s.rows) {
            const int k = lane & (kS - 1), q = lane >> 4;
            const int c = s.off + k;
            const int base = c < n ? (q * n + c) * (int)sizeof(S) : kOob;
            const int step = 4 * n * (int)sizeof(S);
#pragma unroll
            for (int u = 0; u < G::PER; ++u) {
                if (4 * u < s.rmin)
                    v[u] = T(0);
                else
                    buf_ld(v[u], rs, base + u * step);
            }
        } else {
            int base[G::RP];
#pragma unroll
            for (int j = 0; j < G::RP; ++j) {
                const int e = lane + kWave * j, r = e % NP, k = e / NP;
                const bool ok = r < n && (!s.tri || r < s.off + kS);
                base[j] = ok ? ((s.off + k) * n + r) * (int)sizeof(S) : kOob;
            }
            const int step = G::RK * n * (int)sizeof(S);
#pragma unroll
            for (int u = 0; u < G::PER; ++u) buf_ld(v[u], rs, base[u % G::RP] + (u / G::RP) * step);
        }
    }

    __device__ __forceinline__ void put(T* __restrict__ buf, bool rows, int lane) const {
        if (!rows) {
#pragma unroll
            for (int u = 0; u < Geo<NP>::PER; ++u) {
                const int e = lane + kWave * u;
                buf[(e % kS) * Geo<NP>::LDB + e / kS] = v[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < Geo<NP>::PER; ++u) {
                const int e = lane + kWave * u;
                buf[(e / NP) * Geo<NP>::LDB + e % NP] = v[u];
            }
        }
    }
};

// Value of vector row j (wave-uniform) of column c, held by lane j % 64.
template <int RPL, int MC, class T>
__device__ __forceinline__ T row_value(const T (&a)[RPL][MC], int j, int c) {
    T x = a[0][c];
#pragma unroll
    for (int rr = 1; rr < RPL; ++rr)
        if (j >= kWave * rr) x = a[rr][c];
    return bcast(x, j & (kWave - 1));
}

template <class T>
__device__ __forceinline__ bool skip_item(const SweepDesc<T>& P) {
    if (*P.info != kInfoOk) return true;
    if (P.skip && *P.skip) return true;
    return false;
}

// A kernel's block traffic as a list of up to four segments of slabs, each
// segment the slabs of one block in one orientation.  Kept as separate
// scalars (selected by wave-uniform indices) so the plan lives in registers.
template <class S>
struct Seg {
    const S* M;
    int count;   // slabs (0: segment absent)
    bool rows;   // row slabs (else column slabs)
    bool desc;   // slabs from the last one to the first
    bool tri;    // column slab p: rows >= 16p only; row slab: r <= row only
};

template <class S>
struct Plan {
    const S *m0, *m1, *m2, *m3;
    int c0, c1, c2, c3;
    unsigned rows, desc, tri;  // bit g: property of segment g
    int total;
    int slabs;                 // slabs per block (the same for every present segment)

    __device__ __forceinline__ void set(int g, const Seg<S>& sg) {
        if (g == 0) { m0 = sg.M; c0 = sg.count; }
        if (g == 1) { m1 = sg.M; c1 = sg.count; }
        if (g == 2) { m2 = sg.M; c2 = sg.count; }
        if (g == 3) { m3 = sg.M; c3 = sg.count; }
        const unsigned bit = 1u << g;
        rows = sg.rows ? (rows | bit) : (rows & ~bit);
        desc = sg.desc ? (desc | bit) : (desc & ~bit);
        tri = sg.tri ? (tri | bit) : (tri & ~bit);
        total = c0 + c1 + c2 + c3;
        if (sg.count) slabs = sg.count;
    }

    __device__ __forceinline__ void clear() {
        m0 = m1 = m2 = m3 = nullptr;
        c0 = c1 = c2 = c3 = 0;
        rows = desc = tri = 0u;
        total = 0;
        slabs = 0;
    }

    __device__ __forceinline__ bool is_rows(int g) const { return (rows >> g) & 1u; }

    // segment index and slab index within it of global slab p
    __device__ __forceinline__ int locate(int p, int& q) const {
        q = p;
        if (q < c0) return 0;
        q -= c0;
        if (q < c1) return 1;
        q -= c1;
        if (q < c2) return 2;
        q -= c2;
        return 3;
    }

    __device__ __forceinline__ SlabSrc<S> src(int p) const {
        int q;
        const int g = locate(p, q);
        const S* M = g == 0 ? m0 : g == 1 ? m1 : g == 2 ? m2 : m3;
        const bool r = (rows >> g) & 1u, d = (desc >> g) & 1u, t = (tri >> g) & 1u;
        const int sl = d ? slabs - 1 - q : q;  // every present segment has `slabs` slabs
        return {M, kS * sl, (!r && t) ? kS * sl : 0, r, r && t};
    }
};

// target[r] += sgn * slab[k][r] * vec[off + k] over the 16 slab columns
// (column slab: vec indexed by the block's column; row slab: by its row).
// mask: 0 none, 1 only off+k <= r, 2 only r < off+k.
template <int NP, int MC, class T>
__device__ __forceinline__ void slab_axpy(T (&target)[Geo<NP>::RPL][MC], const T* __restrict__ b,
                                          const T (&vec)[Geo<NP>::RPL][MC], int off, int n, T sgn, int mask,
                                          int lane) {
    constexpr int RPL = Geo<NP>::RPL, LDB = Geo<NP>::LDB;
    for (int k = 0; k < kS; ++k) {
        const int cc = off + k;
        if (cc >= n) break;
        T xc[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) xc[c] = sgn * row_value<RPL, MC, T>(vec, cc, c);
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
            T a = b[k * LDB + r];
            if (mask == 1 && cc > r) a = T(0);
            if (mask == 2 && r >= cc) a = T(0);
#pragma unroll
            for (int c = 0; c < MC; ++c) target[rr][c] = fma(a, xc[c], target[rr][c]);
        }
    }
}

// Slabs in flight beyond the one being consumed.  Measured on MI355X: a
// second one buys little per-node latency and costs occupancy (registers),
// so one.
template <int NP, class T>
constexpr int slab_depth() { return 1; }

// Walk the slabs of a plan through the LDS buffer: slab p is consumed by
// body(p, segment, slab index in segment, buffer) while the loads of the next
// DEPTH slabs are in flight (register buffers indexed by unrolled constants).
template <int NP, class T, int DEPTH, class S, class Body>
__device__ __forceinline__ void run_slabs(const Plan<S>& pl, int n, int lane, T* __restrict__ buf, Body&& body) {
    SlabRegs<NP, T> r[DEPTH];
#pragma unroll
    for (int u = 0; u < DEPTH; ++u)
        if (u < pl.total) r[u].fetch(pl.src(u), n, lane);
    for (int p = 0; p < pl.total; p += DEPTH) {
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            const int q = p + u;
            if (q < pl.total) {
                int qs;
                const int g = pl.locate(q, qs);
                r[u].put(buf, pl.is_rows(g), lane);
                wave_lds_sync();
                if (q + DEPTH < pl.total) r[u].fetch(pl.src(q + DEPTH), n, lane);
                body(g, qs, buf);
                wave_lds_sync();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// a minus the contributions left for node i of level lvl by its descendants:
// u from node i - 2^l2 and v from node i + 2^l2 for every l2 < lvl,
// subtracted in level order.  The loads go out in groups of eight before any
// subtraction, so their latencies overlap (a top-level node pulls from up to
// twice its level count of places); a contribution that does not exist reads
// slot 0 and subtracts +0, which leaves every value unchanged bit for bit.
template <class T>
__device__ __forceinline__ T pull(const SweepDesc<T>& P, T a, int64_t i, int lvl, size_t off, size_t nm) {
    const int64_t N = P.N;
    for (int g = 0; g < lvl; g += 8) {
        T cu[8], cv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int l2 = g + u;
            const bool okl = l2 < lvl;
            const int64_t s2 = (int64_t)1 << (okl ? l2 : 0);
            const bool okr = okl && i + s2 <= N;
            const size_t iu = okl ? (size_t)perm_pos(N, l2, i - s2) * nm + off : 0;
            const size_t iv = okr ? (size_t)perm_pos(N, l2, i + s2) * nm + off : 0;
            const T x = P.U[iu], y = P.V[iv];
            cu[u] = okl ? x : T(0);
            cv[u] = okr ? y : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a -= cu[u];
            a -= cv[u];
        }
    }
    return a;
}

// ---------------------------------------------------------------------------
// Forward step of node kk of level lvl by one wavefront (buf: its slab buffer).
template <int NP, int MC, class T>
__device__ __forceinline__ void fwd_node(const SweepDesc<T>& P, int lvl, int64_t kk, T* __restrict__ buf) {
    using G = Geo<NP>;
    constexpr int RPL = G::RPL, LDB = G::LDB;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);
    const int ns = (n + kS - 1) / kS;
    // L_ii column slabs (lower part), R_i column slabs, T_i row slabs
    Plan<T> pl;
    pl.clear();
    pl.set(0, {P.Ld + pi * nn, ns, false, false, true});
    pl.set(1, {P.Rb + pi * nn, has_r ? ns : 0, false, false, false});
    pl.set(2, {P.Tb + pi * nn, has_l ? ns : 0, true, false, false});

    for (int q0 = 0; q0 < m; q0 += MC) {
        T acc[RPL][MC], u[RPL][MC], v[RPL][MC];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                T a = T(0);
                if (r < n && q < m) {
                    const size_t bidx = ((size_t)(i - 1) * n + r) * m + q;
                    a = P.B64 ? (T)P.B64[bidx] : P.B[bidx];
                    a = pull(P, a, i, lvl, (size_t)r * m + q, nm);
                }
                acc[rr][c] = a;
                u[rr][c] = T(0);
                v[rr][c] = T(0);
            }
        }
        run_slabs<NP, T, slab_depth<NP, T>()>(pl, n, lane, buf, [&](int g, int q, const T* b) {
            if (g == 0) {
                // y = L^{-1} acc over columns j of this slab
                for (int k = 0; k < kS; ++k) {
                    const int j = kS * q + k;
                    if (j >= n) break;
                    const T inv = T(1) / b[k * LDB + j];
                    T yj[MC];
#pragma unroll
                    for (int c = 0; c < MC; ++c) yj[c] = row_value<RPL, MC, T>(acc, j, c) * inv;
#pragma unroll
                    for (int rr = 0; rr < RPL; ++rr) {
                        const int r = lane + kWave * rr;
                        const T l = b[k * LDB + r];
#pragma unroll
                        for (int c = 0; c < MC; ++c) {
                            if (r == j) acc[rr][c] = yj[c];
                            else if (r > j) acc[rr][c] = fma(-l, yj[c], acc[rr][c]);
                        }
                    }
                }
            } else if (g == 1) {
                slab_axpy<NP, MC, T>(u, b, acc, kS * q, n, T(1), 0, lane);  // u += R y
            } else {
                slab_axpy<NP, MC, T>(v, b, acc, kS * q, n, T(1), 0, lane);  // v += T^T y
            }
        });
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
            if (r >= n) continue;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                if (q >= m) continue;
                const size_t o = (size_t)pi * nm + (size_t)r * m + q;
                P.Y[o] = acc[rr][c];
                if (has_r) P.U[o] = u[rr][c];
                if (has_l) P.V[o] = v[rr][c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Backward step of node kk of level lvl by one wavefront.
template <int NP, int MC, class T>
__device__ __forceinline__ void bwd_node(const SweepDesc<T>& P, int lvl, int64_t kk, T* __restrict__ buf) {
    using G = Geo<NP>;
    constexpr int RPL = G::RPL, LDB = G::LDB;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m;
    const int64_t s = (int64_t)1 << lvl;
    const int64_t i = (kk * 2 + 1) << lvl;
    const bool has_r = i + s <= N, has_l = i > s;
    const int64_t pi = perm_pos(N, lvl, i);
    const int ns = (n + kS - 1) / kS;
    // R_i row slabs, T_i column slabs, L_ii row slabs from the last one up
    Plan<T> pl;
    pl.clear();
    pl.set(0, {P.Rb + pi * nn, has_r ? ns : 0, true, false, false});
    pl.set(1, {P.Tb + pi * nn, has_l ? ns : 0, false, false, false});
    pl.set(2, {P.Ld + pi * nn, ns, true, true, true});

    for (int q0 = 0; q0 < m; q0 += MC) {
        T acc[RPL][MC], xr[RPL][MC], xl[RPL][MC];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                const bool ok = r < n && q < m;
                acc[rr][c] = ok ? P.Y[(size_t)pi * nm + (size_t)r * m + q] : T(0);
                xr[rr][c] = (ok && has_r) ? P.X[((size_t)(i + s - 1) * n + r) * m + q] : T(0);
                xl[rr][c] = (ok && has_l) ? P.X[((size_t)(i - s - 1) * n + r) * m + q] : T(0);
            }
        }
        run_slabs<NP, T, slab_depth<NP, T>()>(pl, n, lane, buf, [&](int g, int q, const T* b) {
            if (g < 2) {
                // acc -= R^T x_{i+s} (g = 0) or T x_{i-s} (g = 1); the vector is
                // selected element by element so that both stay in registers
                T xv[RPL][MC];
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
                    for (int c = 0; c < MC; ++c) xv[rr][c] = g == 0 ? xr[rr][c] : xl[rr][c];
                slab_axpy<NP, MC, T>(acc, b, xv, kS * q, n, T(-1), 0, lane);
            } else {
                // x = L^{-T} acc over rows j of this slab, last row first
                const int sl = ns - 1 - q;
                for (int k = kS - 1; k >= 0; --k) {
                    const int j = kS * sl + k;
                    if (j >= n) continue;
                    const T inv = T(1) / b[k * LDB + j];
                    T xj[MC];
#pragma unroll
                    for (int c = 0; c < MC; ++c) xj[c] = row_value<RPL, MC, T>(acc, j, c) * inv;
#pragma unroll
                    for (int rr = 0; rr < RPL; ++rr) {
                        const int r = lane + kWave * rr;
                        const T l = b[k * LDB + r];
#pragma unroll
                        for (int c = 0; c < MC; ++c) {
                            if (r == j) acc[rr][c] = xj[c];
                            else if (r < j) acc[rr][c] = fma(-l, xj[c], acc[rr][c]);
                        }
                    }
                }
            }
        });
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
            if (r >= n) continue;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                if (q >= m) continue;
                const size_t idx = ((size_t)(i - 1) * n + r) * m + q;
                P.X[idx] = acc[rr][c];
                if (P.X64) P.X64[idx] = P.first ? (double)acc[rr][c] : P.X64[idx] + (double)acc[rr][c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One level of one or many instances: one wavefront per node.
template <int NP, int MC, class T>
__global__ __launch_bounds__(kWave) void k_fwd(Launch<SweepDesc<T>> L) {
    __shared__ T buf[Geo<NP>::BUF];
    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_item(P)) return;
    fwd_node<NP, MC, T>(P, lvl, kk, buf);
}

template <int NP, int MC, class T>
__global__ __launch_bounds__(kWave) void k_bwd(Launch<SweepDesc<T>> L) {
    __shared__ T buf[Geo<NP>::BUF];
    SweepDesc<T> P;
    int lvl;
    int64_t kk;
    fetch_item(L, P, lvl, kk);
    if (skip_item(P)) return;
    bwd_node<NP, MC, T>(P, lvl, kk, buf);
}

// Several levels in one launch.  The nodes of levels l0 .. l1-1 that lie
// strictly between the blocks j 2^l1 and (j+1) 2^l1 form a subtree of the
// elimination tree whose forward steps read only each other's results and
// those of levels below l0 (a level-l node pulls from the blocks within s of
// it), and whose backward steps read only each other's results and those of
// levels l1 and above (the two blocks at the subtree's ends).  Item (inst, l0
// | l1 << 8, j) is that subtree; its KW wavefronts take the nodes of one level
// at a time (forward: levels ascending, backward: descending), with a
// workgroup barrier between levels: the wavefronts of a workgroup share one
// compute unit and its vector L1, so the barrier's workgroup-scope release
// and acquire make one level's global stores visible to the next level's
// loads (an agent-scope fence would write back and invalidate the L2 at
// every level).
template <int NP, int MC, class T, int KW, bool BWD>
__global__ __launch_bounds__(KW * kWave) void k_sweep_chunk(Launch<SweepDesc<T>> L) {
    __shared__ T buf[KW][Geo<NP>::BUF];
    SweepDesc<T> P;
    int code;
    int64_t j;
    fetch_item(L, P, code, j);
    if (skip_item(P)) return;  // uniform over the workgroup
    const int l0 = code & 0xff, l1 = code >> 8;
    const int w = wave_id();
    const int64_t N = P.N;
    for (int t = 0; t < l1 - l0; ++t) {
        const int l = BWD ? l1 - 1 - t : l0 + t;
        const int64_t per = (int64_t)1 << (l1 - l - 1);  // nodes of a full subtree at level l
        const int64_t s = (int64_t)1 << l;
        const int64_t k0 = j * per, nodes = (N + s) / (2 * s);
        const int64_t k1 = k0 + per < nodes ? k0 + per : nodes;
        for (int64_t k = k0 + w; k < k1; k += KW) {
            if (BWD)
                bwd_node<NP, MC, T>(P, l, k, buf[w]);
            else
                fwd_node<NP, MC, T>(P, l, k, buf[w]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Residual in two kernels, every block read from HBM once.  The wavefront of
// block row i streams the lower triangle of D_i and the coupling E_i (block
// (i+1, i)) as row slabs and uses each element M[c][r] twice: as M^T[r][c]
// (lane r, the vector's row c broadcast) and as M[c][r] (lane r's product
// with the lane's own vector row, summed over the wavefront into row c):
//   P_i     = b_i - D_i x_i - E_i^T x_{i+1}
//   Q_{i+1} = E_i x_i
// The second kernel forms r_i = P_i - Q_i, its FP32 copy and the per-column
// partial squared norms of r_i and b_i.  Work items of consecutive block rows
// share an XCD (xcd_local_block).

// Value of the exchange partner across lane bit H: DPP within rows of 16
// lanes (the row mirror for bit 3, the half-row mirror for bit 2, quad
// permutations for bits 1 and 0), LDS permute across rows.  Each pairing is
// an involution whose pairs differ in bit H and otherwise only in lower bits.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long w = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)w, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(w >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int H>
__device__ __forceinline__ double partner(double v) {
    if constexpr (H == 8) return dpp_d<0x140>(v);       // row_mirror
    else if constexpr (H == 4) return dpp_d<0x141>(v);  // row_half_mirror
    else if constexpr (H == 2) return dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    else if constexpr (H == 1) return dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    else return __shfl_xor(v, H);
}
// Lane bit of exchange step T: bits 3, 2, 1, 0 first (a mirror also flips
// the bits below its own, so those must not be bound to a value yet), then
// 4 and 5.
constexpr int step_bit(int t) { return t < 4 ? 8 >> t : 16 << (t - 4); }

// Halving exchanges from step T on, W values per lane in play: the lane
// keeps the half its step bit selects and adds its partner's copy of it.
template <int W, int T>
__device__ __forceinline__ void halve(double* v, int lane) {
    if constexpr (W >= 1) {
        constexpr int H = step_bit(T);
        const bool up = (lane & H) != 0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const double send = up ? v[j] : v[j + W];
            const double keep = up ? v[j + W] : v[j];
            v[j] = keep + partner<H>(send);
        }
        halve<W / 2, T + 1>(v, lane);
    }
}
template <int T>
__device__ __forceinline__ double all_sum(double s) {
    if constexpr (T < 6) return all_sum<T + 1>(s + partner<step_bit(T)>(s));
    else return s;
}
constexpr int ilog2_c(int v) { return v <= 1 ? 0 : 1 + ilog2_c(v / 2); }

// Sum over the wavefront of KB values per lane (KB a power of two <= 16).
// Afterwards the lanes given by row_source hold the totals.  Every total is
// formed by the same tree of additions whatever KB is, so chunking rows
// differently does not change a bit of the result.
template <int KB>
__device__ __forceinline__ double wave_sum_rows(double (&v)[KB], int lane) {
    static_assert(KB >= 1 && KB <= 16 && (KB & (KB - 1)) == 0, "power of two up to 16");
    halve<KB / 2, 0>(v, lane);
    return all_sum<ilog2_c(KB)>(v[0]);
}
// A lane that holds the total of value k after wave_sum_rows<KB>: step t of
// the halving bound the value's bit KB / 2^(t+1) to lane bit step_bit(t).
template <int KB>
__device__ __forceinline__ int row_source(int k) {
    int l = 0;
#pragma unroll
    for (int t = 0, w = KB / 2; w >= 1; ++t, w /= 2)
        if (k & w) l |= step_bit(t);
    return l;
}

template <int NP, int MC>
__global__ __launch_bounds__(kWave) void k_res(Launch<ResidualDesc> L) {
    using G = Geo<NP>;
    constexpr int RPL = G::RPL, LDB = G::LDB;
    constexpr int KB = 4 / MC;              // slab rows per wavefront sum (4 sums live)
    static_assert(KB >= 1 && kS % KB == 0, "chunks divide the slab");
    __shared__ double buf[G::BUF];
    ResidualDesc P;
    int64_t row0;
    {
        const unsigned b = xcd_local_block();
        if (L.items) {
            const WorkItem it = L.items[b];
            P = L.descs[it.inst];
            row0 = it.k;
        } else {
            P = L.single;
            row0 = b;
        }
    }
    if (P.state && P.state->done) return;
    const int lane = threadIdx.x;
    const int64_t N = P.N;
    const int n = P.n, m = P.m;
    const size_t nn = (size_t)n * n;
    const int64_t i = row0 + 1;
    const bool rgt = i < N;
    const int ns = (n + kS - 1) / kS;
    // D_i row slabs (the lower triangle: slab rows c, columns r <= last row
    // of the slab), E_i row slabs
    Plan<double> pl;
    pl.clear();
    pl.set(0, {P.A_diag + (size_t)(i - 1) * nn, ns, true, false, true});
    pl.set(1, {rgt ? P.A_off + (size_t)(i - 1) * nn : nullptr, rgt ? ns : 0, true, false, false});

    for (int q0 = 0; q0 < m; q0 += MC) {
        // acc: b_i minus the broadcast products; dl: (D_i x_i) over the lower
        // triangle; qa: E_i x_i.  dl and qa take one wavefront sum per row,
        // so the result does not depend on how rows are chunked (MC).
        double acc[RPL][MC], dl[RPL][MC], qa[RPL][MC], x1[RPL][MC], x2[RPL][MC];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                const bool ok = r < n && q < m;
                acc[rr][c] = ok ? P.B[((size_t)(i - 1) * n + r) * m + q] : 0.0;
                dl[rr][c] = 0.0;
                qa[rr][c] = 0.0;
                x1[rr][c] = ok ? P.X[((size_t)(i - 1) * n + r) * m + q] : 0.0;
                x2[rr][c] = (ok && rgt) ? P.X[((size_t)i * n + r) * m + q] : 0.0;
            }
        }
        run_slabs<NP, double, slab_depth<NP, double>()>(pl, n, lane, buf, [&](int g, int q, const double* b) {
            // g = 0: slab row c of D_i (elements with r <= c valid); g = 1:
            // row c of E_i.  Rows past n are zero.
            const int off = kS * q, dslot = off / kWave;
#pragma unroll 1
            for (int k0 = 0; k0 < kS; k0 += KB) {
                double ps[MC][KB];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int cc = off + k0 + k;
                    double xb[MC];
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        double t = g == 0 ? x1[0][c] : x2[0][c];
#pragma unroll
                        for (int rr = 1; rr < RPL; ++rr)
                            if (cc >= kWave * rr) t = g == 0 ? x1[rr][c] : x2[rr][c];
                        xb[c] = -bcast(t, cc & (kWave - 1));
                        ps[c][k] = 0.0;
                    }
#pragma unroll
                    for (int rr = 0; rr < RPL; ++rr) {
                        const int r = lane + kWave * rr;
                        // columns r in [n, NP) of the slab are zero; lanes r >= NP
                        // would read the next slab row (perhaps the unread
                        // upper triangle of D_i) and feed the wavefront sums
                        const double a = (NP % kWave == 0 || rr < RPL - 1 || r < NP) ? b[(k0 + k) * LDB + r] : 0.0;
                        if (g == 0 && rr == dslot) {
                            // the diagonal tile of D_i: as element (r, c) above
                            // the diagonal (r < c), as element (c, r) on and
                            // below it
                            const double au = r >= cc ? 0.0 : a;
                            const double al = r > cc ? 0.0 : a;
#pragma unroll
                            for (int c = 0; c < MC; ++c) {
                                acc[rr][c] = fma(au, xb[c], acc[rr][c]);
                                ps[c][k] = fma(al, x1[rr][c], ps[c][k]);
                            }
                        } else {
                            // D_i left of the diagonal tile (the rest of the
                            // slab row is zero), E_i: both uses
#pragma unroll
                            for (int c = 0; c < MC; ++c) {
                                acc[rr][c] = fma(a, xb[c], acc[rr][c]);
                                ps[c][k] = fma(a, x1[rr][c], ps[c][k]);
                            }
                        }
                    }
                }
                // row c = off + k0 + k gets its sum from lane row_source(k);
                // its owner is lane c % 64 in slot c / 64
                const int base = off + k0, slot = base / kWave;
                const int k = lane - (base & (kWave - 1));
                const int src = row_source<KB>(k & (KB - 1));
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const double s = wave_sum_rows<KB>(ps[c], lane);
                    const double t = __shfl(s, src);
                    if (k >= 0 && k < KB) {
#pragma unroll
                        for (int rr = 0; rr < RPL; ++rr) {
                            if (rr == slot) {
                                if (g == 0)
                                    dl[rr][c] += t;
                                else
                                    qa[rr][c] += t;
                            }
                        }
                    }
                }
            }
        });
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int r = lane + kWave * rr;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int q = q0 + c;
                if (r < n && q < m) {
                    P.P[((size_t)(i - 1) * n + r) * m + q] = acc[rr][c] - dl[rr][c];
                    if (rgt) P.Q[((size_t)i * n + r) * m + q] = qa[rr][c];
                }
            }
        }
    }
}

// r_i = P_i - Q_i (Q_1 = 0), its FP32 copy and the partial norms; one
// wavefront per block row.
__global__ __launch_bounds__(kWave) void k_res_fin(Launch<ResidualDesc> L) {
    ResidualDesc P;
    int level;
    int64_t row0;
    fetch_item(L, P, level, row0);
    if (P.state && P.state->done) return;
    const int lane = threadIdx.x;
    const int n = P.n, m = P.m;
    const int64_t i = row0 + 1;
    for (int q = 0; q < m; ++q) {
        double r2 = 0.0, b2 = 0.0;
        for (int r = lane; r < n; r += kWave) {
            const size_t e = ((size_t)(i - 1) * n + r) * m + q;
            const double v = i > 1 ? P.P[e] - P.Q[e] : P.P[e];
            if (P.R32) P.R32[e] = (float)v;
            if (P.R64) P.R64[e] = P.neg ? -v : v;
            const double bv = P.B[e];
            r2 = fma(v, v, r2);
            b2 = fma(bv, bv, b2);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            r2 += __shfl_xor(r2, off);
            b2 += __shfl_xor(b2, off);
        }
        if (lane == 0) {
            P.part[((size_t)(i - 1) * m + q) * 2 + 0] = r2;
            P.part[((size_t)(i - 1) * m + q) * 2 + 1] = b2;
        }
    }
}

template <int NP, class T>
hipError_t launch_sweep_np(const Launch<SweepDesc<T>>& p, int64_t items, bool backward, int mc, hipStream_t st) {
    const dim3 g((unsigned)items), b(kWave);
    if (mc <= 1) {
        if (backward)
            hipLaunchKernelGGL((k_bwd<NP, 1, T>), g, b, 0, st, p);
        else
            hipLaunchKernelGGL((k_fwd<NP, 1, T>), g, b, 0, st, p);
    } else {
        if (backward)
            hipLaunchKernelGGL((k_bwd<NP, 4, T>), g, b, 0, st, p);
        else
            hipLaunchKernelGGL((k_fwd<NP, 4, T>), g, b, 0, st, p);
    }
    return hipGetLastError();
}

template <int NP, class T, int KW>
hipError_t launch_chunk_kw(const Launch<SweepDesc<T>>& p, int64_t items, bool backward, int mc, hipStream_t st) {
    const dim3 g((unsigned)items), b(KW * kWave);
    if (mc <= 1) {
        if (backward)
            hipLaunchKernelGGL((k_sweep_chunk<NP, 1, T, KW, true>), g, b, 0, st, p);
        else
            hipLaunchKernelGGL((k_sweep_chunk<NP, 1, T, KW, false>), g, b, 0, st, p);
    } else {
        if (backward)
            hipLaunchKernelGGL((k_sweep_chunk<NP, 4, T, KW, true>), g, b, 0, st, p);
        else
            hipLaunchKernelGGL((k_sweep_chunk<NP, 4, T, KW, false>), g, b, 0, st, p);
    }
    return hipGetLastError();
}

template <int NP, class T>
hipError_t launch_chunk_np(const Launch<SweepDesc<T>>& p, int64_t items, bool backward, int mc, hipStream_t st,
                           int kw) {
    return kw == 8 ? launch_chunk_kw<NP, T, 8>(p, items, backward, mc, st)
                   : launch_chunk_kw<NP, T, 4>(p, items, backward, mc, st);
}

template <class T>
hipError_t launch_sweep_t(const Launch<SweepDesc<T>>& p, int np, int64_t items, bool backward, int mc,
                          hipStream_t st, bool chunk, int kw) {
    switch (np) {
        case 8:
        case 16: return chunk ? launch_chunk_np<16, T>(p, items, backward, mc, st, kw) : launch_sweep_np<16, T>(p, items, backward, mc, st);
        case 32: return chunk ? launch_chunk_np<32, T>(p, items, backward, mc, st, kw) : launch_sweep_np<32, T>(p, items, backward, mc, st);
        case 64: return chunk ? launch_chunk_np<64, T>(p, items, backward, mc, st, kw) : launch_sweep_np<64, T>(p, items, backward, mc, st);
        case 96: return chunk ? launch_chunk_np<96, T>(p, items, backward, mc, st, kw) : launch_sweep_np<96, T>(p, items, backward, mc, st);
        case 128: return chunk ? launch_chunk_np<128, T>(p, items, backward, mc, st, kw) : launch_sweep_np<128, T>(p, items, backward, mc, st);
        default: return hipErrorInvalidValue;
    }
}

template <int NP>
hipError_t launch_res_np(const Launch<ResidualDesc>& p, int64_t items, int mc, hipStream_t st) {
    const dim3 g((unsigned)items), b(kWave);
    if (mc <= 1)
        hipLaunchKernelGGL((k_res<NP, 1>), g, b, 0, st, p);
    else
        hipLaunchKernelGGL((k_res<NP, 4>), g, b, 0, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_res_fin, g, b, 0, st, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const Launch<SweepDesc<double>>& p, int np, int64_t items, bool backward, int mc,
                        hipStream_t st, bool chunk, int kw) {
    return launch_sweep_t<double>(p, np, items, backward, mc, st, chunk, kw);
}

hipError_t launch_sweep(const Launch<SweepDesc<float>>& p, int np, int64_t items, bool backward, int mc,
                        hipStream_t st, bool chunk, int kw) {
    return launch_sweep_t<float>(p, np, items, backward, mc, st, chunk, kw);
}

hipError_t launch_residual(const Launch<ResidualDesc>& p, int np, int64_t items, int mc, hipStream_t st) {
    switch (np) {
        case 8:
        case 16: return launch_res_np<16>(p, items, mc, st);
        case 32: return launch_res_np<32>(p, items, mc, st);
        case 64: return launch_res_np<64>(p, items, mc, st);
        case 96: return launch_res_np<96>(p, items, mc, st);
        case 128: return launch_res_np<128>(p, items, mc, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace btc
