// Extensions of the method to two neighbouring sparsity structures (the
// paper names both without an algorithm: arrow structures in the section
// "Multi-Stage Permutation", after the cyclic-reduction remark; block-banded
// matrices of larger bandwidth in the section "Conclusion").
//
// Block-banded, block bandwidth b: b consecutive block rows and columns form
// one super-block of order b*n, which makes the matrix block tridiagonal
// with ceil(N/b) super-blocks; a pack kernel writes those super-blocks and
// the multi-stage factor and sweeps run on them unchanged.  A missing part of
// the last super-block is completed with identity rows and columns (zero
// right-hand side, zero solution).
//
// Arrow [[Psi, F], [F^T, C]] (Psi block tridiagonal, F its dense border of m
// columns, C the m x m tip): Psi is eliminated first by the multi-stage
// method, then the tip:
//     Z = Psi^{-1} F   (one solve with m right-hand sides)
//     S = C - F^T Z    (tall-skinny product on the FP64 matrix cores:
//                       per-chunk partial tiles, summed in chunk order)
//     S = L_S L_S^T    (one workgroup, the packed lower triangle in LDS)
// and a solve is y = Psi^{-1} b1, x2 = L_S^{-T} L_S^{-1} (b2 - F^T y),
// x1 = y - Z x2.  The Psi solves refine to the handle's target in the
// mixed-precision modes, so Z, y and the tip are FP64-accurate in every mode.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "btc.h"
#include "btc_device.h"
#include "btc_handle.h"

using namespace btc;
using namespace btc_host;

namespace {

constexpr int kTipMax = 128;      // largest tip (m) of an arrow
constexpr int kT = 256;           // threads of the elementwise kernels
constexpr int kChunksMax = 256;   // partial tiles of a tall-skinny product
typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Super-blocks of a block-banded matrix.  One thread per element of D2
// (N2 blocks of order n2 = b n) and of E2 (N2 - 1 blocks, E2[I-1] the block
// at super-row I, super-column I-1).  Element (R, C) of super-block (I, J)
// is element (R % n, C % n) of block (b I + R / n, b J + C / n).
__global__ __launch_bounds__(kT) void k_band_pack(const double* __restrict__ A, int64_t N, int n, int b,
                                                  int64_t N2, double* __restrict__ D2, double* __restrict__ E2) {
    const int n2 = b * n;
    const int64_t per = (int64_t)n2 * n2;
    const int64_t total = (2 * N2 - 1) * per;
    const size_t nn = (size_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kT) {
        const bool diag = e < N2 * per;
        const int64_t sb = diag ? e / per : (e - N2 * per) / per;  // super-block (I, or I-1 for E2)
        const int64_t rc = diag ? e % per : (e - N2 * per) % per;
        const int R = (int)(rc / n2), C = (int)(rc % n2);
        const int r = R / n, rr = R % n, c = C / n, cc = C % n;
        double v = 0.0;
        if (diag) {
            const int64_t i = b * sb + r, j = b * sb + c;
            if (i >= N || j >= N) {
                v = (R == C) ? 1.0 : 0.0;  // completion, decoupled from the band
            } else if (r >= c) {
                const double* blk = A + ((size_t)i * (b + 1) + (r - c)) * nn;
                v = (r > c || rr >= cc) ? blk[(size_t)rr * n + cc] : blk[(size_t)cc * n + rr];
            } else {
                // above the diagonal: the transpose of block (j, i)
                const double* blk = A + ((size_t)j * (b + 1) + (c - r)) * nn;
                v = blk[(size_t)cc * n + rr];
            }
            D2[e] = v;
        } else {
            const int64_t I = sb + 1;
            const int64_t i = b * I + r;
            const int k = b + r - c;  // block distance i - j
            if (i < N && k <= b) v = A[((size_t)i * (b + 1) + k) * nn + (size_t)rr * n + cc];
            E2[e - N2 * per] = v;
        }
    }
}

// dst = src for the first `rows` rows, 0 for the rest (rows of q values).
__global__ __launch_bounds__(kT) void k_pad_rows(const double* __restrict__ src, int64_t rows, int64_t rows_pad,
                                                 int64_t q, double* __restrict__ dst) {
    const int64_t total = rows_pad * q;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kT)
        dst[e] = e < rows * q ? src[e] : 0.0;
}

__global__ __launch_bounds__(kT) void k_copy(const double* __restrict__ src, int64_t count, double* __restrict__ dst) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < count; e += (int64_t)gridDim.x * kT) dst[e] = src[e];
}

unsigned grid_for(int64_t elems) {
    const int64_t g = (elems + kT - 1) / kT;
    return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

// ---------------------------------------------------------------------------
// Tall-skinny product out = C0 - F^T Y with F (K x m) and Y (K x q) row-major.
// Pass 1: workgroup (chunk, tile) forms the 32 x 32 output tile `tile` over
// rows [chunk*rows, (chunk+1)*rows) of F and Y, one 16 x 16 quadrant per
// wavefront on the FP64 matrix cores (lane (i, kq) feeds F[k + kq][row0 + i]
// and Y[k + kq][col0 + i]; accumulator v of the lane holds output row
// 4 v + kq, column i).  Pass 2 sums the chunks in order.
__global__ __launch_bounds__(256) void k_tsk_part(const double* __restrict__ F, const double* __restrict__ Y,
                                                  int64_t K, int m, int q, int64_t rows, double* __restrict__ part) {
    const int tq = (q + 31) / 32;
    const int tm = (int)blockIdx.y / tq, tc = (int)blockIdx.y % tq;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
    const int r0 = 32 * tm + 16 * (w >> 1), c0 = 32 * tc + 16 * (w & 1);
    const int64_t k0 = (int64_t)blockIdx.x * rows, k1 = k0 + rows < K ? k0 + rows : K;
    const bool okr = r0 + i < m, okc = c0 + i < q;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int64_t k = k0; k < k1; k += 4) {
        const int64_t kk = k + kq;
        const bool okk = kk < k1;
        const double a = (okk && okr) ? F[kk * m + r0 + i] : 0.0;
        const double y = (okk && okc) ? Y[kk * q + c0 + i] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, y, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + 4 * v + kq, c = c0 + i;
        if (r < m && c < q) part[((size_t)blockIdx.x * m + r) * q + c] = acc[v];
    }
}

// out[r][c] = C0[r][c] - sum over chunks (in order) of part[chunk][r][c];
// sym: C0 symmetric with its lower triangle read.
__global__ __launch_bounds__(kT) void k_tsk_fin(const double* __restrict__ part, int chunks, const double* __restrict__ C0,
                                                int m, int q, bool sym, double* __restrict__ out) {
    const int64_t total = (int64_t)m * q;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kT) {
        const int r = (int)(e / q), c = (int)(e % q);
        double s = 0.0;
        for (int t = 0; t < chunks; ++t) s += part[(size_t)t * total + e];
        const double c0 = (sym && c > r) ? C0[(size_t)c * q + r] : C0[e];
        out[e] = c0 - s;
    }
}

// ---------------------------------------------------------------------------
// Cholesky of the m x m tip S (row-major, lower triangle read) in place by
// one workgroup: the packed lower triangle in LDS, column by column (pivot
// square root, column scaled, trailing triangle updated by all threads).
// Writes L_S (strict upper part 0) and *info = 0, or the 1-based column of
// the first non-positive (or NaN) pivot.
__device__ __forceinline__ int tri_at(int r, int c) { return r * (r + 1) / 2 + c; }
__device__ __forceinline__ void tri_rc(int e, int& r, int& c) {
    r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > e) --r;
    while ((r + 1) * (r + 2) / 2 <= e) ++r;
    c = e - r * (r + 1) / 2;
}

__global__ __launch_bounds__(256) void k_tip_chol(double* __restrict__ S, int m, unsigned long long* __restrict__ info) {
    __shared__ double a[kTipMax * (kTipMax + 1) / 2];
    __shared__ int fail;
    const int tid = threadIdx.x;
    const int tot = m * (m + 1) / 2;
    for (int e = tid; e < tot; e += 256) {
        int r, c;
        tri_rc(e, r, c);
        a[e] = S[(size_t)r * m + c];
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double d = a[tri_at(j, j)];
            if (!(d > 0.0))
                fail = j + 1;
            else
                a[tri_at(j, j)] = sqrt(d);
        }
        __syncthreads();
        if (fail) break;
        const double dj = a[tri_at(j, j)];
        for (int r = j + 1 + tid; r < m; r += 256) a[tri_at(r, j)] /= dj;
        __syncthreads();
        const int t = m - j - 1;
        for (int e = tid; e < t * (t + 1) / 2; e += 256) {
            int rr, cc;
            tri_rc(e, rr, cc);
            const int r = j + 1 + rr, c = j + 1 + cc;
            a[tri_at(r, c)] = fma(-a[tri_at(r, j)], a[tri_at(c, j)], a[tri_at(r, c)]);
        }
        __syncthreads();
    }
    for (int e = tid; e < m * m; e += 256) {
        const int r = e / m, c = e % m;
        S[e] = c <= r ? a[tri_at(r, c)] : 0.0;
    }
    if (tid == 0) *info = (unsigned long long)fail;
}

// X2 (m x q) <- L_S^{-T} L_S^{-1} X2, one wavefront per column: lane r holds
// rows r and r + 64; each step broadcasts the finished value by readlane.
__global__ __launch_bounds__(64) void k_tip_solve(const double* __restrict__ Ls, int m, double* __restrict__ X2,
                                                  int q) {
    const int col = blockIdx.x, lane = threadIdx.x;
    double x0 = lane < m ? X2[(size_t)lane * q + col] : 0.0;
    double x1 = lane + 64 < m ? X2[(size_t)(lane + 64) * q + col] : 0.0;
    for (int j = 0; j < m; ++j) {
        double xj = j < 64 ? readlane_d(x0, j) : readlane_d(x1, j - 64);
        xj = xj / Ls[(size_t)j * m + j];
        if (lane == j) x0 = xj;
        if (lane + 64 == j) x1 = xj;
        if (lane > j && lane < m) x0 = fma(-Ls[(size_t)lane * m + j], xj, x0);
        if (lane + 64 > j && lane + 64 < m) x1 = fma(-Ls[(size_t)(lane + 64) * m + j], xj, x1);
    }
    for (int j = m - 1; j >= 0; --j) {
        double xj = j < 64 ? readlane_d(x0, j) : readlane_d(x1, j - 64);
        xj = xj / Ls[(size_t)j * m + j];
        if (lane == j) x0 = xj;
        if (lane + 64 == j) x1 = xj;
        if (lane < j) x0 = fma(-Ls[(size_t)j * m + lane], xj, x0);
        if (lane + 64 < j) x1 = fma(-Ls[(size_t)j * m + lane + 64], xj, x1);
    }
    if (lane < m) X2[(size_t)lane * q + col] = x0;
    if (lane + 64 < m) X2[(size_t)(lane + 64) * q + col] = x1;
}

// X1 (K x q) -= Z (K x m) X2 (m x q).
__global__ __launch_bounds__(kT) void k_arrow_update(const double* __restrict__ Z, int64_t K, int m,
                                                     const double* __restrict__ X2, int q, double* __restrict__ X1) {
    const int64_t total = K * q;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total; e += (int64_t)gridDim.x * kT) {
        const int64_t r = e / q;
        const int c = (int)(e % q);
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc = fma(Z[(size_t)r * m + j], X2[(size_t)j * q + c], acc);
        X1[e] -= acc;
    }
}

// out = C0 - F^T Y through the allocator (stream-ordered partial tiles).
int tsk(const Allocator& al, const double* F, const double* Y, int64_t K, int m, int q, const double* C0, bool sym,
        double* out, hipStream_t st) {
    if (m == 0 || q == 0) return 0;
    // K >= 1: every arrow has at least one block row
    int64_t rows = (K + kChunksMax - 1) / kChunksMax;
    if (rows < 64) rows = 64;
    rows = (rows + 3) / 4 * 4;
    const int chunks = (int)((K + rows - 1) / rows);
    void* part = nullptr;
    if (dev_alloc_async(al, &part, (size_t)chunks * m * q * sizeof(double), st) != hipSuccess) return BTC_ERR_OOM;
    const int tiles = ((m + 31) / 32) * ((q + 31) / 32);
    hipLaunchKernelGGL(k_tsk_part, dim3((unsigned)chunks, (unsigned)tiles), dim3(256), 0, st, F, Y, K, m, q, rows,
                       (double*)part);
    hipLaunchKernelGGL(k_tsk_fin, dim3(grid_for((int64_t)m * q)), dim3(kT), 0, st, (const double*)part, chunks, C0, m, q,
                       sym, out);
    const hipError_t e = hipGetLastError();
    dev_free_async(al, part, st);
    return e == hipSuccess ? 0 : BTC_ERR_HIP;
}

}  // namespace

// ---------------------------------------------------------------------------
// Block-banded

struct btc_banded_s {
    btc_handle h = nullptr;
    int64_t N = 0, n = 0, b = 0, N2 = 0, n2 = 0;
    double* D2 = nullptr;
    double* E2 = nullptr;
    Allocator alloc;
};

namespace {
int band_pack(btc_banded s, const double* A_band, hipStream_t st) {
    const int64_t total = (2 * s->N2 - 1) * s->n2 * s->n2;
    hipLaunchKernelGGL(k_band_pack, dim3(grid_for(total)), dim3(kT), 0, st, A_band, s->N, (int)s->n, (int)s->b, s->N2,
                       s->D2, s->E2);
    return hipGetLastError() == hipSuccess ? 0 : BTC_ERR_HIP;
}
}  // namespace

BTC_API int btc_banded_create(const btc_options* opt, int64_t N, int64_t n, int64_t b, const double* A_band,
                              void* stream, btc_banded* out) {
    if (!out) return -7;
    *out = nullptr;
    if (N < 1) return -2;
    if (n < 1) return -3;
    if (b < 1) return -4;
    if (!A_band) return -5;
    if (b * n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    btc_banded s = new btc_banded_s;
    s->N = N;
    s->n = n;
    s->b = b;
    s->N2 = (N + b - 1) / b;
    s->n2 = b * n;
    s->alloc = current_allocator();
    const size_t blk = (size_t)s->n2 * s->n2 * sizeof(double);
    int rc = 0;
    if (dev_alloc(s->alloc, (void**)&s->D2, blk * s->N2, st) != hipSuccess ||
        dev_alloc(s->alloc, (void**)&s->E2, blk * (s->N2 > 1 ? s->N2 - 1 : 1), st) != hipSuccess)
        rc = BTC_ERR_OOM;
    if (rc == 0) rc = btc_create(s->N2, s->n2, opt, &s->h);
    if (rc == 0) rc = band_pack(s, A_band, st);
    if (rc == 0) rc = btc_refactor(s->h, s->D2, s->E2, stream);
    if (rc != 0) {
        btc_banded_destroy(s);
        return rc;
    }
    *out = s;
    return 0;
}

BTC_API int btc_banded_refactor(btc_banded s, const double* A_band, void* stream) {
    if (!s) return -1;
    if (!A_band) return -2;
    int rc = band_pack(s, A_band, (hipStream_t)stream);
    return rc ? rc : btc_refactor(s->h, s->D2, s->E2, stream);
}

BTC_API int btc_banded_solve(btc_banded s, const double* B, double* X, int64_t nrhs, void* stream,
                             btc_solve_info* info) {
    if (!s) return -1;
    if (!B) return -2;
    if (!X) return -3;
    if (nrhs < 0) return -4;
    if (nrhs == 0) return btc_solve(s->h, B, X, 0, stream, info);
    const int64_t rows = s->N * s->n, rows2 = s->N2 * s->n2;
    if (rows == rows2) return btc_solve(s->h, B, X, nrhs, stream, info);
    // completion rows: solve on padded copies
    hipStream_t st = (hipStream_t)stream;
    void* mem = nullptr;
    if (dev_alloc_async(s->alloc, &mem, 2 * (size_t)rows2 * nrhs * sizeof(double), st) != hipSuccess)
        return BTC_ERR_OOM;
    double* B2 = (double*)mem;
    double* X2 = B2 + (size_t)rows2 * nrhs;
    hipLaunchKernelGGL(k_pad_rows, dim3(grid_for(rows2 * nrhs)), dim3(kT), 0, st, B, rows, rows2, nrhs, B2);
    int rc = hipGetLastError() == hipSuccess ? 0 : BTC_ERR_HIP;
    if (rc == 0) rc = btc_solve(s->h, B2, X2, nrhs, stream, info);
    if (rc == 0) {
        hipLaunchKernelGGL(k_copy, dim3(grid_for(rows * nrhs)), dim3(kT), 0, st, (const double*)X2, rows * nrhs, X);
        rc = hipGetLastError() == hipSuccess ? 0 : BTC_ERR_HIP;
    }
    dev_free_async(s->alloc, mem, st);
    return rc;
}

BTC_API int btc_banded_status(btc_banded s, int64_t* info) {
    if (!s) return -1;
    return btc_status(s->h, info);
}

BTC_API btc_handle btc_banded_inner(btc_banded s) { return s ? s->h : nullptr; }

BTC_API void btc_banded_destroy(btc_banded s) {
    if (!s) return;
    if (s->h)
        btc_destroy(s->h);
    else
        (void)hipDeviceSynchronize();
    dev_free(s->alloc, s->D2, nullptr);
    dev_free(s->alloc, s->E2, nullptr);
    delete s;
}

// ---------------------------------------------------------------------------
// Arrow

struct btc_arrow_s {
    btc_handle h = nullptr;
    int64_t N = 0, n = 0, m = 0;
    double* F = nullptr;   // (N n) x m, the caller's border copied
    double* Z = nullptr;   // (N n) x m, Psi^{-1} F
    double* Ls = nullptr;  // m x m, Cholesky factor of the tip's Schur complement
    unsigned long long* tip_info = nullptr;
    Allocator alloc;
    hipStream_t last = nullptr;
};

namespace {
// Border copy, Z = Psi^{-1} F, S = C - F^T Z, S = L_S L_S^T.
int arrow_tip(btc_arrow s, const double* F, const double* C, hipStream_t st) {
    const int64_t K = s->N * s->n;
    const int m = (int)s->m;
    s->last = st;
    if (m == 0) return 0;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(K * m)), dim3(kT), 0, st, F, K * m, s->F);
    if (hipGetLastError() != hipSuccess) return BTC_ERR_HIP;
    int rc = btc_solve(s->h, s->F, s->Z, m, st, nullptr);
    if (rc == BTC_ERR_NOT_SPD) return 0;  // Psi broke down: btc_arrow_status reports it
    if (rc == 0) rc = tsk(s->alloc, s->F, s->Z, K, m, m, C, true, s->Ls, st);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_tip_chol, dim3(1), dim3(256), 0, st, s->Ls, m, s->tip_info);
    return hipGetLastError() == hipSuccess ? 0 : BTC_ERR_HIP;
}
}  // namespace

BTC_API int btc_arrow_create(const btc_options* opt, int64_t N, int64_t n, int64_t m, const double* A_diag,
                             const double* A_off, const double* F, const double* C, void* stream, btc_arrow* out) {
    if (!out) return -10;
    *out = nullptr;
    if (N < 1) return -2;
    if (n < 1) return -3;
    if (m < 0) return -4;
    if (!A_diag) return -5;
    if (N > 1 && !A_off) return -6;
    if (m > 0 && !F) return -7;
    if (m > 0 && !C) return -8;
    if (m > kTipMax || n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    btc_arrow s = new btc_arrow_s;
    s->N = N;
    s->n = n;
    s->m = m;
    s->alloc = current_allocator();
    s->last = st;
    int rc = btc_factor(A_diag, A_off, N, n, opt, stream, &s->h);
    const size_t km = (size_t)N * n * (m > 0 ? m : 1) * sizeof(double);
    if (rc == 0 && (dev_alloc(s->alloc, (void**)&s->F, km, st) != hipSuccess ||
                    dev_alloc(s->alloc, (void**)&s->Z, km, st) != hipSuccess ||
                    dev_alloc(s->alloc, (void**)&s->Ls, (size_t)(m > 0 ? m * m : 1) * sizeof(double), st) !=
                        hipSuccess ||
                    dev_alloc(s->alloc, (void**)&s->tip_info, 256, st) != hipSuccess))
        rc = BTC_ERR_OOM;
    if (rc == 0) {
        unsigned long long zero = 0;
        if (hipMemcpyAsync(s->tip_info, &zero, sizeof(zero), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = BTC_ERR_HIP;
    }
    if (rc == 0) rc = arrow_tip(s, F, C, st);
    if (rc != 0) {
        btc_arrow_destroy(s);
        return rc;
    }
    *out = s;
    return 0;
}

BTC_API int btc_arrow_refactor(btc_arrow s, const double* A_diag, const double* A_off, const double* F,
                               const double* C, void* stream) {
    if (!s) return -1;
    if (!A_diag) return -2;
    if (s->N > 1 && !A_off) return -3;
    if (s->m > 0 && !F) return -4;
    if (s->m > 0 && !C) return -5;
    int rc = btc_refactor(s->h, A_diag, A_off, stream);
    return rc ? rc : arrow_tip(s, F, C, (hipStream_t)stream);
}

BTC_API int btc_arrow_solve(btc_arrow s, const double* B, double* X, int64_t nrhs, void* stream,
                            btc_solve_info* info) {
    if (!s) return -1;
    if (!B) return -2;
    if (!X) return -3;
    if (nrhs < 0) return -4;
    hipStream_t st = (hipStream_t)stream;
    s->last = st;
    const int64_t K = s->N * s->n;
    const int m = (int)s->m, q = (int)nrhs;
    if (nrhs > (1 << 20)) return BTC_ERR_UNSUPPORTED;
    // y = Psi^{-1} b1 into the first K rows of X
    int rc = btc_solve(s->h, B, X, nrhs, stream, info);
    if (rc != 0 || m == 0 || q == 0) return rc;
    double* X2 = X + (size_t)K * q;
    rc = tsk(s->alloc, s->F, X, K, m, q, B + (size_t)K * q, false, X2, st);  // b2 - F^T y
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_tip_solve, dim3((unsigned)q), dim3(64), 0, st, (const double*)s->Ls, m, X2, q);
    hipLaunchKernelGGL(k_arrow_update, dim3(grid_for(K * q)), dim3(kT), 0, st, (const double*)s->Z, K, m,
                       (const double*)X2, q, X);
    return hipGetLastError() == hipSuccess ? 0 : BTC_ERR_HIP;
}

BTC_API int btc_arrow_status(btc_arrow s, int64_t* info_psi, int64_t* info_tip) {
    if (!s) return -1;
    if (!info_psi) return -2;
    if (!info_tip) return -3;
    int rc = btc_status(s->h, info_psi);
    if (rc != 0) return rc;
    unsigned long long t = 0;
    if (s->m > 0) {
        if (hipStreamSynchronize(s->last) != hipSuccess ||
            hipMemcpy(&t, s->tip_info, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess)
            return BTC_ERR_HIP;
    }
    *info_tip = (int64_t)t;
    return 0;
}

BTC_API int btc_arrow_export(btc_arrow s, double* Ls, double* Z) {
    if (!s) return -1;
    if (hipStreamSynchronize(s->last) != hipSuccess) return BTC_ERR_HIP;
    const int64_t K = s->N * s->n, m = s->m;
    if (m == 0) return 0;
    if (Ls && hipMemcpy(Ls, s->Ls, (size_t)m * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return BTC_ERR_HIP;
    if (Z && hipMemcpy(Z, s->Z, (size_t)K * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return BTC_ERR_HIP;
    return 0;
}

BTC_API btc_handle btc_arrow_inner(btc_arrow s) { return s ? s->h : nullptr; }

BTC_API void btc_arrow_destroy(btc_arrow s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->last);
    if (s->h) btc_destroy(s->h);
    dev_free(s->alloc, s->F, nullptr);
    dev_free(s->alloc, s->Z, nullptr);
    dev_free(s->alloc, s->Ls, nullptr);
    dev_free(s->alloc, s->tip_info, nullptr);
    delete s;
}
