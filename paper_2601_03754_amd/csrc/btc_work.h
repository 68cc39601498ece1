// Algorithmic work of one level step (host side; used by the launch
// profiler and exported as btc_level_work).
//
// Factor, per node i of level l (stride s, h = s/2), the block traffic of the
// level step of Algorithm 4, every n x n block counted once:
//   reads  S_i, S_{i+s} (if right), the couplings C_{i+s,i} (if right) and
//          C_{i,i-s} (if left), T_{i+h} and T_{i+3h} (the deferred updates,
//          levels above 0)
//   writes L_ii, R_i (if right), T_i (if left), S_{i+s} (if right), the fill
//          C_{i+s,i-s} (if both)
//   flops  potrf n^3/3; trsm n^3 per coupling; syrk n^3 per coupling (the
//          deferred one of T counted where it is applied); fill gemm 2n^3
//          (operation counts of section "Computational Complexity"; summed
//          over the levels: n^3 (N/3 + 2 M_off + 2 F) with M_off couplings and
//          F fills).
// Word sizes: FP64 8 bytes; mixed precision keeps S and the inputs in FP64
// and the factor and fill blocks in FP32 (4 bytes).
// Sweeps (Algorithm 6), per node and sweep: read L_ii, R_i, T_i; vectors of
// n x m words: forward reads b_i, the pulled products of lower levels (at
// most two per lower level), writes y_i and the products R_i y_i, T_i^T y_i;
// backward reads y_i and x_{i+-s}, writes x_i.  Flops n^2 m per triangular
// solve plus 2 n^2 m per coupling product.
// Residual (FP64), per block row: D_i and E_i once each over the matrix
// (8 n^2 (2N - 1) bytes in total), x_i, b_i read and r_i written
// (24 n m per row); flops 2 n^2 m per block of the row.
#pragma once

#include <stdint.h>

namespace btc_host {

struct Work {
    double bytes = 0.0;
    double flops = 0.0;
    int64_t items = 0;
};

inline Work level_work(int op, bool mixed, int64_t N, int64_t n, int64_t m, int level) {
    Work w;
    const double nn = (double)n * (double)n, n3 = nn * (double)n;
    const double wS = 8.0, wF = mixed ? 4.0 : 8.0;
    if (op == 3) {  // residual: all block rows
        w.items = N;
        w.bytes = 8.0 * nn * (double)(2 * N - 1) + 24.0 * (double)(N * n * m);
        w.flops = 2.0 * nn * (double)m * (double)(3 * N - 2);
        return w;
    }
    if (op == 4 || op == 5) {  // refinement set-up / test: per-column norms
        w.items = 1;
        w.bytes = 16.0 * (double)(N * m);
        return w;
    }
    if (level < 0 || level > 62) return w;
    const int64_t s = (int64_t)1 << level, h = s >> 1;
    if (s > N) return w;
    int64_t nodes = 0, r = 0, l = 0, ds = 0, dp = 0, both = 0;
    for (int64_t i = s; i <= N; i += 2 * s) {
        const bool hr = i + s <= N, hl = i > s;
        ++nodes;
        r += hr;
        l += hl;
        both += hr && hl;
        ds += level > 0 && i + h <= N;
        dp += level > 0 && hr && i + 3 * h <= N;
    }
    w.items = nodes;
    if (op == 0) {
        const double wC = level == 0 ? 8.0 : wF;
        const double rd = nn * (wS * (double)(nodes + r) + wC * (double)(r + l) + wF * (double)(ds + dp));
        const double wr = nn * (wS * (double)r + wF * (double)(nodes + r + l + both));
        w.bytes = rd + wr;
        w.flops = n3 * ((double)nodes / 3.0 + 2.0 * (double)r + (double)l + (double)(ds + dp) + 2.0 * (double)both);
        return w;
    }
    const double vec = wF * (double)(n * m);
    const double blocks = (double)(nodes + r + l);
    if (op == 1) {
        const double pulls = (double)nodes * 2.0 * level;
        w.bytes = blocks * nn * wF + vec * ((double)nodes + pulls) + vec * (double)(nodes + r + l);
    } else {
        w.bytes = blocks * nn * wF + vec * (double)(nodes + r + l) + vec * (double)nodes;
    }
    w.flops = nn * (double)m * (double)(nodes + 2 * r + 2 * l);
    return w;
}

// Work of one launch of the tile-parallel factorization (padded sizes 64 and
// above) split by kernel: part 1 the deferred syrk (reads T_{i+h}, T_{i+3h},
// reads and writes the S blocks it updates; nothing when the previous level
// ran eagerly), part 2 the pivot factorization with both triangular solves
// (reads S_i and the couplings, writes L_ii, R_i, T_i), part 3 the separator
// and fill products (reads R_i, T_i and S_{i+s}, writes S_{i+s} and the fill;
// eagerly also reads the right neighbour's T_{i+2s} and applies its syrk).
// The parts pass S and the factor blocks through HBM between them, so their
// sum exceeds the level step's count.  flags: the FactorDesc flags.
inline Work tiled_part_work(int part, bool mixed, int64_t N, int64_t n, int level, int flags) {
    Work w;
    const double nn = (double)n * (double)n, n3 = nn * (double)n;
    const double wS = 8.0, wF = mixed ? 4.0 : 8.0, wC = level == 0 ? 8.0 : wF;
    const int64_t s = (int64_t)1 << level, h = s >> 1;
    if (level < 0 || level > 62 || s > N) return w;
    const bool eager = (flags & 1) != 0, done = (flags & 2) != 0;
    for (int64_t i = s; i <= N; i += 2 * s) {
        const bool hr = i + s <= N, hl = i > s, both = hr && hl;
        const int def = done ? 0 : (level > 0 && i + h <= N) + (level > 0 && hr && i + 3 * h <= N);
        const int nb = eager && hr && i + 2 * s <= N;  // right neighbour's T^T T
        ++w.items;
        if (part == 1) {
            w.bytes += nn * (wF + 2.0 * wS) * def;
            w.flops += n3 * def;
        } else if (part == 2) {
            w.bytes += nn * (wS + wC * (hr + hl) + wF * (1 + hr + hl));
            w.flops += n3 * (1.0 / 3.0 + hr + hl);
        } else {
            w.bytes += nn * (wF * (hr + both + nb) + 2.0 * wS * hr + wF * both);
            w.flops += n3 * (hr + 2.0 * both + nb);
        }
    }
    return w;
}

}  // namespace btc_host
