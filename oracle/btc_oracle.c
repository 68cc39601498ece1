/*
 * btc_oracle.c -- plain, slow, FP64 CPU oracle for the Cholesky factorization
 * and solve of a symmetric positive-definite block-tridiagonal matrix in
 * nested-dissection order (Schwan, Kuhn, Jones: "GPU-Accelerated Cholesky
 * Factorization of Block Tridiagonal Matrices", arXiv 2601.03754).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may link, load or call
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * Everything here is FP64, plain loops, no BLAS, no blocking beyond the block
 * structure the paper defines, no reordering beyond the permutation the paper
 * defines.  Each routine names the passage of the paper it writes out.
 *
 * Conventions (1-based block indices as in the paper, section "Sequential
 * Cholesky Factorization"):
 *   Psi has diagonal blocks D_1..D_N (n x n, symmetric; only the LOWER triangle
 *   of each stored D_i is read, the upper one is ignored) and sub-diagonal
 *   blocks E_1..E_{N-1}, E_i sitting at block position (i+1, i); E_i^T sits at
 *   (i, i+1).
 *   D is stored [N][n][n] row-major, E is stored [N-1][n][n] row-major with
 *   E[(i-1)] = E_i.  Right-hand sides and solutions are [N][n][m] row-major
 *   (global row (i-1)*n + r, column q).
 *
 * Factor output of the nested-dissection routines, indexed by ORIGINAL block
 * index i (1-based, stored at slot i-1):
 *   Ld[i] = L_ii       lower-triangular diagonal block of the factor of
 *                      P Psi P^T (strict upper triangle written as 0)
 *   Rb[i] = R_i        the factor block at (row i+s, column i), present when
 *                      node i has a right neighbour i+s <= N, else zero
 *   Tb[i] = T_i        the TRANSPOSE of the factor block at (row i-s,
 *                      column i), present when node i has a left neighbour
 *                      i-s >= 1, else zero.  T_i = L_ii^{-1} C where C is the
 *                      coupling block at (row i, column i-s).
 * where s = 2^ctz(i) is the stride of the level that node i belongs to.
 *
 * Parity: the nested-dissection factor is pinned against a textbook dense
 * Cholesky of the explicitly permuted matrix (orc_dense_chol, and LAPACK via
 * numpy in the tests), the solve against dense solves, closed forms and the
 * natural-order algorithm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Op counters: number of calls to each elementary block operation of the
 * cost table in section "Computational Complexity" (potrf, trsm, syrk,
 * gemm), so that tests can compare operation counts with the paper's cost
 * formulas.  counts[0]=potrf, [1]=trsm, [2]=syrk, [3]=gemm. */
static void bump(int64_t *counts, int which)
{
    if (counts) counts[which] += 1;
}

/* number of trailing zero bits of i > 0: the level a block belongs to in the
 * multi-stage (nested-dissection) permutation, section "Multi-Stage
 * Permutation": level-l blocks are the odd multiples of 2^l. */
int64_t orc_level_of(int64_t i)
{
    int64_t l = 0;
    while ((i & 1) == 0) {
        i >>= 1;
        ++l;
    }
    return l;
}

/* Number of levels floor(log2 N) + 1 (section "Multi-Stage Permutation": the
 * multi-stage factorization needs floor(log2 N)+1 parallel iterations). */
int64_t orc_num_levels(int64_t N)
{
    int64_t L = 0;
    while ((((int64_t)1) << (L + 1)) <= N) ++L;
    return L + 1;
}

/* The multi-stage permutation P_inf (section "Multi-Stage Permutation", the
 * display of Phi_inf): all odd blocks first, then the odd blocks of the
 * remaining (even) sequence, and so on recursively.  order[p] is the 1-based
 * original block index placed at permuted position p. */
void orc_nd_order(int64_t N, int64_t *order)
{
    int64_t p = 0;
    for (int64_t s = 1; s <= N; s *= 2)
        for (int64_t i = s; i <= N; i += 2 * s) order[p++] = i;
}

/* ------------------------------------------------------------------------ */
/* Dense helpers on row-major n x n blocks with leading dimension n. */

#define AT(M, r, c) ((M)[(size_t)(r) * (size_t)n + (size_t)(c)])

/* Copy the symmetric matrix whose lower triangle is stored in src. */
static void sym_from_lower(int64_t n, const double *src, double *dst)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c)
            AT(dst, r, c) = (c <= r) ? AT(src, r, c) : AT(src, c, r);
}

/* Textbook column-by-column (Cholesky-Crout) factorization of a dense
 * symmetric positive-definite matrix of order dim, lower triangle in place:
 * L_jj = sqrt(A_jj - sum_k L_jk^2), L_ij = (A_ij - sum_k L_ik L_jk)/L_jj.
 * Reads the lower triangle only; writes 0 to the strict upper triangle.
 * Returns 0 on success, j+1 (1-based column) when the pivot of column j is not
 * positive (or not finite).  Used on single blocks and, in tests, on the whole
 * permuted matrix as the brute-force definition. */
int64_t orc_dense_chol(int64_t dim, double *A)
{
    const int64_t n = dim;
    for (int64_t j = 0; j < n; ++j) {
        double d = AT(A, j, j);
        for (int64_t k = 0; k < j; ++k) d -= AT(A, j, k) * AT(A, j, k);
        if (!(d > 0.0) || !isfinite(d)) return j + 1;
        d = sqrt(d);
        AT(A, j, j) = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = AT(A, i, j);
            for (int64_t k = 0; k < j; ++k) v -= AT(A, i, k) * AT(A, j, k);
            AT(A, i, j) = v / d;
        }
        for (int64_t c = j + 1; c < n; ++c) AT(A, j, c) = 0.0;
    }
    return 0;
}

/* C <- C * L^{-T}   (trsm, right side, L lower triangular): row r of the
 * result solves X L^T = C by forward substitution over the columns. */
static void trsm_right_lower_t(int64_t n, const double *L, double *C)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t j = 0; j < n; ++j) {
            double v = AT(C, r, j);
            for (int64_t k = 0; k < j; ++k) v -= AT(C, r, k) * AT(L, j, k);
            AT(C, r, j) = v / AT(L, j, j);
        }
}

/* C <- L^{-1} * C   (trsm, left side, L lower triangular): forward
 * substitution down every column of C. */
static void trsm_left_lower(int64_t n, const double *L, double *C, int64_t m)
{
    for (int64_t q = 0; q < m; ++q)
        for (int64_t j = 0; j < n; ++j) {
            double v = C[(size_t)j * m + q];
            for (int64_t k = 0; k < j; ++k) v -= AT(L, j, k) * C[(size_t)k * m + q];
            C[(size_t)j * m + q] = v / AT(L, j, j);
        }
}

/* C <- L^{-T} * C   (backward substitution with the transpose of L). */
static void trsm_left_lower_t(int64_t n, const double *L, double *C, int64_t m)
{
    for (int64_t q = 0; q < m; ++q)
        for (int64_t j = n - 1; j >= 0; --j) {
            double v = C[(size_t)j * m + q];
            for (int64_t k = j + 1; k < n; ++k) v -= AT(L, k, j) * C[(size_t)k * m + q];
            C[(size_t)j * m + q] = v / AT(L, j, j);
        }
}

/* S <- S - A A^T (syrk; the full symmetric result is formed). */
static void sub_aat(int64_t n, double *S, const double *A)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += AT(A, r, k) * AT(A, c, k);
            AT(S, r, c) -= v;
        }
}

/* S <- S - A^T A (syrk with the transpose on the left). */
static void sub_ata(int64_t n, double *S, const double *A)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += AT(A, k, r) * AT(A, k, c);
            AT(S, r, c) -= v;
        }
}

/* F <- -A B (gemm producing a fill-in block). */
static void neg_ab(int64_t n, const double *A, const double *B, double *F)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += AT(A, r, k) * AT(B, k, c);
            AT(F, r, c) = -v;
        }
}

/* y <- y - A x for an n x n block A and n x m panels x, y. */
static void sub_ax(int64_t n, int64_t m, const double *A, const double *x, double *y)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t q = 0; q < m; ++q) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += AT(A, r, k) * x[(size_t)k * m + q];
            y[(size_t)r * m + q] -= v;
        }
}

/* y <- y - A^T x. */
static void sub_atx(int64_t n, int64_t m, const double *A, const double *x, double *y)
{
    for (int64_t r = 0; r < n; ++r)
        for (int64_t q = 0; q < m; ++q) {
            double v = 0.0;
            for (int64_t k = 0; k < n; ++k) v += AT(A, k, r) * x[(size_t)k * m + q];
            y[(size_t)r * m + q] -= v;
        }
}

#define BLK(P, i) ((P) + (size_t)((i) - 1) * (size_t)n * (size_t)n)
#define VEC(P, i) ((P) + (size_t)((i) - 1) * (size_t)n * (size_t)m)

/* ------------------------------------------------------------------------ */
/* Nested-dissection factorization, written as the textbook right-looking
 * (submatrix) block Cholesky of section "Block Cholesky Factorization" applied
 * to the permuted matrix Phi_inf = P_inf Psi P_inf^T of section "Multi-Stage
 * Permutation", visiting columns in permuted order and skipping the blocks
 * that are structurally zero.
 *
 * In permuted order the column of node i (level l, stride s = 2^l) has at
 * most two nonzero blocks below its diagonal: the rows of its current
 * neighbours i+s and i-s, which belong to higher levels.  Eliminating the
 * column therefore takes (cf. the per-level body of Algorithm 4 and of
 * Algorithm 5, which reach the same factor up to rounding order):
 *   L_ii       = chol(S_i)                                   potrf
 *   R_i        = C_{i+s,i} L_ii^{-T},  S_{i+s} -= R_i R_i^T  trsm, syrk
 *   T_i        = L_ii^{-1} C_{i,i-s},  S_{i-s} -= T_i^T T_i  trsm, syrk
 *   C_{i+s,i-s} = -R_i T_i   (fill-in coupling of the next level)  gemm
 * with S_j initialised to D_j and the couplings of level 0 to E_j.
 *
 * Returns 0 on success, or the 1-based original index of the first block (in
 * elimination order) whose pivot block is not positive definite; the factor is
 * then incomplete.  counts (nullable) receives the number of potrf/trsm/syrk/
 * gemm block operations. */
int64_t orc_factor_nd(int64_t N, int64_t n, const double *D, const double *E,
                      double *Ld, double *Rb, double *Tb, int64_t *counts)
{
    const size_t bs = (size_t)n * (size_t)n;
    /* S: working diagonal blocks (Schur complements), by original index. */
    double *S = (double *)malloc(bs * (size_t)N * sizeof(double));
    /* C[j]: coupling between j and j+s at the current level, stored as the
     * block at (row j+s, column j), indexed by its lower endpoint j. */
    double *C = (double *)calloc(bs * (size_t)N, sizeof(double));
    double *Cn = (double *)calloc(bs * (size_t)N, sizeof(double));
    int64_t info = 0;
    if (!S || !C || !Cn) {
        free(S); free(C); free(Cn);
        return -1;
    }
    for (int64_t i = 1; i <= N; ++i) sym_from_lower(n, BLK(D, i), BLK(S, i));
    for (int64_t i = 1; i < N; ++i) memcpy(BLK(C, i), BLK(E, i), bs * sizeof(double));
    memset(Ld, 0, bs * (size_t)N * sizeof(double));
    memset(Rb, 0, bs * (size_t)N * sizeof(double));
    memset(Tb, 0, bs * (size_t)N * sizeof(double));

    for (int64_t s = 1; s <= N && info == 0; s *= 2) {
        memset(Cn, 0, bs * (size_t)N * sizeof(double));
        for (int64_t i = s; i <= N; i += 2 * s) {
            double *L = BLK(Ld, i);
            memcpy(L, BLK(S, i), bs * sizeof(double));
            bump(counts, 0);
            if (orc_dense_chol(n, L) != 0) {
                info = i;
                break;
            }
            const int has_r = (i + s <= N);
            const int has_l = (i > s);
            if (has_r) {
                double *R = BLK(Rb, i);
                memcpy(R, BLK(C, i), bs * sizeof(double));
                trsm_right_lower_t(n, L, R);
                bump(counts, 1);
                sub_aat(n, BLK(S, i + s), R);
                bump(counts, 2);
            }
            if (has_l) {
                double *T = BLK(Tb, i);
                memcpy(T, BLK(C, i - s), bs * sizeof(double));
                trsm_left_lower(n, L, T, n);
                bump(counts, 1);
                sub_ata(n, BLK(S, i - s), T);
                bump(counts, 2);
            }
            if (has_r && has_l) {
                neg_ab(n, BLK(Rb, i), BLK(Tb, i), BLK(Cn, i - s));
                bump(counts, 3);
            }
        }
        double *t = C;
        C = Cn;
        Cn = t;
    }
    free(S);
    free(C);
    free(Cn);
    return info;
}

/* Nested-dissection solve Psi X = B with the factor of orc_factor_nd, written
 * as the plain block forward substitution P^T L Y = B followed by the block
 * backward substitution L^T P X = Y (section "Cholesky Solve", Algorithm 6):
 *   forward, levels ascending:  y_i = L_ii^{-1} y_i; y_{i+s} -= R_i y_i;
 *                               y_{i-s} -= T_i^T y_i
 *   backward, levels descending: x_i -= R_i^T x_{i+s}; x_i -= T_i x_{i-s};
 *                               x_i = L_ii^{-T} x_i
 * B and X are [N][n][m]; X may alias B. */
void orc_solve_nd(int64_t N, int64_t n, int64_t m, const double *Ld, const double *Rb,
                  const double *Tb, const double *B, double *X)
{
    const size_t vs = (size_t)n * (size_t)m;
    if (X != B) memmove(X, B, vs * (size_t)N * sizeof(double));
    int64_t smax = 1;
    while (smax * 2 <= N) smax *= 2;
    for (int64_t s = 1; s <= N; s *= 2)
        for (int64_t i = s; i <= N; i += 2 * s) {
            trsm_left_lower(n, BLK(Ld, i), VEC(X, i), m);
            if (i + s <= N) sub_ax(n, m, BLK(Rb, i), VEC(X, i), VEC(X, i + s));
            if (i > s) sub_atx(n, m, BLK(Tb, i), VEC(X, i), VEC(X, i - s));
        }
    for (int64_t s = smax; s >= 1; s /= 2)
        for (int64_t i = s; i <= N; i += 2 * s) {
            if (i + s <= N) sub_atx(n, m, BLK(Rb, i), VEC(X, i + s), VEC(X, i));
            if (i > s) sub_ax(n, m, BLK(Tb, i), VEC(X, i - s), VEC(X, i));
            trsm_left_lower_t(n, BLK(Ld, i), VEC(X, i), m);
        }
}

/* ------------------------------------------------------------------------ */
/* Natural-order sequential factorization, Algorithm 1 (section "Sequential
 * Cholesky Factorization"):
 *   Dh_1 = chol(D_1);  for i = 2..N:  Eh_{i-1} = E_{i-1} Dh_{i-1}^{-T};
 *   Dh_i = chol(D_i - Eh_{i-1} Eh_{i-1}^T).
 * Dh is [N][n][n] (lower), Eh is [N-1][n][n].  Returns 0 or the 1-based index
 * of the first failing block.  An independent second route to the solution. */
int64_t orc_factor_seq(int64_t N, int64_t n, const double *D, const double *E,
                       double *Dh, double *Eh, int64_t *counts)
{
    const size_t bs = (size_t)n * (size_t)n;
    sym_from_lower(n, BLK(D, 1), BLK(Dh, 1));
    bump(counts, 0);
    if (orc_dense_chol(n, BLK(Dh, 1)) != 0) return 1;
    for (int64_t i = 2; i <= N; ++i) {
        memcpy(BLK(Eh, i - 1), BLK(E, i - 1), bs * sizeof(double));
        trsm_right_lower_t(n, BLK(Dh, i - 1), BLK(Eh, i - 1));
        bump(counts, 1);
        sym_from_lower(n, BLK(D, i), BLK(Dh, i));
        sub_aat(n, BLK(Dh, i), BLK(Eh, i - 1));
        bump(counts, 2);
        bump(counts, 0);
        if (orc_dense_chol(n, BLK(Dh, i)) != 0) return i;
    }
    return 0;
}

/* Solve with the block-bidiagonal factor of Algorithm 1:
 * forward  y_1 = Dh_1^{-1} b_1,  y_i = Dh_i^{-1}(b_i - Eh_{i-1} y_{i-1});
 * backward x_N = Dh_N^{-T} y_N,  x_i = Dh_i^{-T}(y_i - Eh_i^T x_{i+1}). */
void orc_solve_seq(int64_t N, int64_t n, int64_t m, const double *Dh, const double *Eh,
                   const double *B, double *X)
{
    const size_t vs = (size_t)n * (size_t)m;
    if (X != B) memmove(X, B, vs * (size_t)N * sizeof(double));
    for (int64_t i = 1; i <= N; ++i) {
        if (i > 1) sub_ax(n, m, BLK(Eh, i - 1), VEC(X, i - 1), VEC(X, i));
        trsm_left_lower(n, BLK(Dh, i), VEC(X, i), m);
    }
    for (int64_t i = N; i >= 1; --i) {
        if (i < N) sub_atx(n, m, BLK(Eh, i), VEC(X, i + 1), VEC(X, i));
        trsm_left_lower_t(n, BLK(Dh, i), VEC(X, i), m);
    }
}

/* Residual Rr = B - Psi X in FP64 (block-tridiagonal product with the matrix
 * of section "Sequential Cholesky Factorization": row block i is
 * E_{i-1} x_{i-1} + D_i x_i + E_i^T x_{i+1}; D_i symmetric from its lower
 * triangle). */
void orc_residual(int64_t N, int64_t n, int64_t m, const double *D, const double *E,
                  const double *X, const double *B, double *Rr)
{
    const size_t vs = (size_t)n * (size_t)m;
    memcpy(Rr, B, vs * (size_t)N * sizeof(double));
    for (int64_t i = 1; i <= N; ++i) {
        double *r = VEC(Rr, i);
        const double *Di = BLK(D, i);
        for (int64_t a = 0; a < n; ++a)
            for (int64_t q = 0; q < m; ++q) {
                double v = 0.0;
                for (int64_t b = 0; b < n; ++b) {
                    const double dab = (b <= a) ? AT(Di, a, b) : AT(Di, b, a);
                    v += dab * VEC(X, i)[(size_t)b * m + q];
                }
                r[(size_t)a * m + q] -= v;
            }
        if (i > 1) sub_ax(n, m, BLK(E, i - 1), VEC(X, i - 1), r);
        if (i < N) sub_atx(n, m, BLK(E, i), VEC(X, i + 1), r);
    }
}

/* ------------------------------------------------------------------------ */
/* Other elimination orders of the same chain (section "Parallel Cholesky
 * Factorization": the partition permutation of Algorithm 2, the single-stage
 * permutation, and the two-stage variant of the strategy comparison; the
 * multi-stage order is orc_nd_order).  Each is the Cholesky factorization of
 * P Psi P^T for another block permutation P, written as the same right-looking
 * block elimination as orc_factor_nd: in every one of these orders a block,
 * when it is eliminated, is coupled to at most one not-yet-eliminated block on
 * each side (its left and right neighbours at that time), so the column of
 * block i holds L_ii and at most two blocks below it:
 *   Ro[i] = the factor block at (row rn[i], column i)   (rn[i] > i, or 0: none)
 *   To[i] = the TRANSPOSE of the factor block at (row ln[i], column i)
 *                                                        (ln[i] < i, or 0: none)
 * with the same convention as Rb / Tb of orc_factor_nd (T_i = L_ii^{-1} C where C
 * is the coupling block at (row i, column ln[i])).  Eliminating i:
 *   L_ii = chol(S_i); R_i = C_{rn,i} L_ii^{-T}; S_rn -= R_i R_i^T;
 *   T_i = L_ii^{-1} C_{i,ln}; S_ln -= T_i^T T_i; C_{rn,ln} = -R_i T_i (fill),
 * after which rn and ln are each other's neighbours.
 *
 * order: the 1-based original block indices in elimination order (a
 * permutation of 1..N).  Returns 0, or the 1-based index of the first block
 * whose pivot is not positive definite.  counts as in orc_factor_nd; when
 * phase is not NULL, counts are kept per phase[i] (counts + 4*phase[i]). */
int64_t orc_factor_order(int64_t N, int64_t n, const int64_t *order, const double *D, const double *E,
                         double *Ld, double *Ro, double *To, int64_t *rn, int64_t *ln,
                         const int64_t *phase, int64_t *counts)
{
    const size_t bs = (size_t)n * (size_t)n;
    double *S = (double *)malloc(bs * (size_t)N * sizeof(double));
    /* CR[j]: coupling between j and its current right neighbour R[j], stored
     * as the block at (row R[j], column j); indexed by the lower endpoint. */
    double *CR = (double *)calloc(bs * (size_t)N, sizeof(double));
    double *F = (double *)malloc(bs * sizeof(double));
    int64_t *Rn = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 2));
    int64_t *Lnb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 2));
    int64_t info = 0;
    if (!S || !CR || !F || !Rn || !Lnb) {
        free(S); free(CR); free(F); free(Rn); free(Lnb);
        return -1;
    }
    for (int64_t i = 1; i <= N; ++i) {
        sym_from_lower(n, BLK(D, i), BLK(S, i));
        Rn[i] = i < N ? i + 1 : 0;
        Lnb[i] = i > 1 ? i - 1 : 0;
    }
    for (int64_t i = 1; i < N; ++i) memcpy(BLK(CR, i), BLK(E, i), bs * sizeof(double));
    memset(Ld, 0, bs * (size_t)N * sizeof(double));
    memset(Ro, 0, bs * (size_t)N * sizeof(double));
    memset(To, 0, bs * (size_t)N * sizeof(double));
    for (int64_t p = 0; p < N && info == 0; ++p) {
        const int64_t i = order[p];
        int64_t *cnt = counts ? counts + (phase ? 4 * phase[i - 1] : 0) : NULL;
        const int64_t r = Rn[i], l = Lnb[i];
        rn[i - 1] = r;
        ln[i - 1] = l;
        double *L = BLK(Ld, i);
        memcpy(L, BLK(S, i), bs * sizeof(double));
        bump(cnt, 0);
        if (orc_dense_chol(n, L) != 0) {
            info = i;
            break;
        }
        if (r) {
            double *Rm = BLK(Ro, i);
            memcpy(Rm, BLK(CR, i), bs * sizeof(double));
            trsm_right_lower_t(n, L, Rm);
            bump(cnt, 1);
            sub_aat(n, BLK(S, r), Rm);
            bump(cnt, 2);
        }
        if (l) {
            double *Tm = BLK(To, i);
            memcpy(Tm, BLK(CR, l), bs * sizeof(double));  /* block (i, l): C_{i,l} */
            trsm_left_lower(n, L, Tm, n);
            bump(cnt, 1);
            sub_ata(n, BLK(S, l), Tm);
            bump(cnt, 2);
        }
        if (r && l) {
            /* the fill couples l and r: block (r, l) = -R_i T_i */
            neg_ab(n, BLK(Ro, i), BLK(To, i), F);
            bump(cnt, 3);
            memcpy(BLK(CR, l), F, bs * sizeof(double));
        }
        /* i leaves the graph: its neighbours become each other's */
        if (l) Rn[l] = r;
        if (r) Lnb[r] = l;
    }
    free(S); free(CR); free(F); free(Rn); free(Lnb);
    return info;
}

/* Solve with the factor of orc_factor_order: forward substitution in
 * elimination order (y_i = L_ii^{-1} y_i; y_rn -= R_i y_i; y_ln -= T_i^T y_i),
 * then backward substitution in reverse order (x_i -= R_i^T x_rn;
 * x_i -= T_i x_ln; x_i = L_ii^{-T} x_i). */
void orc_solve_order(int64_t N, int64_t n, int64_t m, const int64_t *order, const double *Ld,
                     const double *Ro, const double *To, const int64_t *rn, const int64_t *ln,
                     const double *B, double *X)
{
    const size_t vs = (size_t)n * (size_t)m;
    if (X != B) memmove(X, B, vs * (size_t)N * sizeof(double));
    for (int64_t p = 0; p < N; ++p) {
        const int64_t i = order[p];
        trsm_left_lower(n, BLK(Ld, i), VEC(X, i), m);
        if (rn[i - 1]) sub_ax(n, m, BLK(Ro, i), VEC(X, i), VEC(X, rn[i - 1]));
        if (ln[i - 1]) sub_atx(n, m, BLK(To, i), VEC(X, i), VEC(X, ln[i - 1]));
    }
    for (int64_t p = N - 1; p >= 0; --p) {
        const int64_t i = order[p];
        if (rn[i - 1]) sub_atx(n, m, BLK(Ro, i), VEC(X, rn[i - 1]), VEC(X, i));
        if (ln[i - 1]) sub_ax(n, m, BLK(To, i), VEC(X, ln[i - 1]), VEC(X, i));
        trsm_left_lower_t(n, BLK(Ld, i), VEC(X, i), m);
    }
}

/* k-stage order: the first k levels of the multi-stage permutation (odd
 * blocks, odd multiples of 2, ..., of 2^(k-1)), then the remaining blocks (the
 * multiples of 2^k) in natural order, eliminated one after the other as in
 * Algorithm 1.  k = 0: natural order (Algorithm 1); k = 1: the single-stage
 * permutation Phi_1; k = 2: the two-stage variant; k >= floor(log2 N)+1: the
 * multi-stage order. */
void orc_kstage_order(int64_t N, int64_t k, int64_t *order)
{
    int64_t p = 0, s = 1;
    for (int64_t l = 0; l < k && s <= N; ++l, s *= 2)
        for (int64_t i = s; i <= N; i += 2 * s) order[p++] = i;
    for (int64_t i = s; i <= N; i += s) order[p++] = i;
}

/* Chunk sizes of the partition permutation with p chunks (section "Partition
 * Permutation", Proposition 1): the first chunk costs (7/3 N_1 - 1) n^3 and
 * every other (19/3 N_k - 1) n^3, so the balanced sizes are N_k* =
 * (7N - 7p + 7)/(7p + 12) for k > 1 and N_1 = N - (p-1) - (p-1) N_k (p-1
 * blocks are pivots).  N_k* is rounded down and up; of the two the one with
 * the smaller larger phase cost is kept (ties: rounded down).  sizes[0..p-1]
 * receives N_1..N_p; returns 0, or -1 when no chunk sizes >= 1 exist. */
int64_t orc_partition_sizes(int64_t N, int64_t p, int64_t *sizes)
{
    if (p < 1) return -1;
    if (p == 1) {
        sizes[0] = N;
        return N >= 1 ? 0 : -1;
    }
    const double nk = (7.0 * (double)N - 7.0 * (double)p + 7.0) / (7.0 * (double)p + 12.0);
    int64_t best = -1;
    double best_cost = 0.0;
    for (int64_t c = (int64_t)floor(nk); c <= (int64_t)ceil(nk); ++c) {
        if (c < 1) continue;
        const int64_t n1 = N - (p - 1) - (p - 1) * c;
        if (n1 < 1) continue;
        const double c1 = 7.0 / 3.0 * (double)n1 - 1.0, ck = 19.0 / 3.0 * (double)c - 1.0;
        const double cost = c1 > ck ? c1 : ck;
        if (best < 0 || cost < best_cost) {
            best = c;
            best_cost = cost;
        }
    }
    if (best < 0) return -1;
    sizes[0] = N - (p - 1) - (p - 1) * best;
    for (int64_t k = 1; k < p; ++k) sizes[k] = best;
    return 0;
}

/* Partition order (Algorithm 2): chunk 1 = blocks 1..N_1, pivot A_2 = block
 * N_1+1, chunk 2 = the next N_2 blocks, pivot A_3, ..., chunk p; the blocks of
 * every chunk in natural order, chunk after chunk, then the p-1 pivots in
 * natural order.  phase[i-1] (nullable) receives k-1 for the blocks of chunk
 * k and p for the pivots (for per-chunk operation counts, cf. the cost table
 * of section "Partition Permutation"). */
void orc_partition_order(int64_t N, int64_t p, const int64_t *sizes, int64_t *order, int64_t *phase)
{
    int64_t q = 0, b = 1;
    int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p > 1 ? p : 1));
    for (int64_t k = 0; k < p; ++k) {
        for (int64_t t = 0; t < sizes[k]; ++t, ++b) {
            order[q++] = b;
            if (phase) phase[b - 1] = k;
        }
        if (k + 1 < p) {
            piv[k] = b;
            if (phase) phase[b - 1] = p;
            ++b;
        }
    }
    for (int64_t k = 0; k + 1 < p; ++k) order[q++] = piv[k];
    free(piv);
}
