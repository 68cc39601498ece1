// Internal interface between the libbtc host code and its kernels.
//
// Every kernel is driven by work items.  An item names one node (or one block
// row, or one instance) of one instance at one level; the instance itself is
// described by a descriptor.  A launch either processes the implicit items
// (0, level, k = blockIdx.x) of a single instance whose descriptor travels by
// value in the kernel arguments, or an explicit device array of items whose
// descriptors live in a device array.  Explicit items let one launch serve
// many instances of different sizes, at different levels, at once (batched
// factorizations and continuous batching of requests); every item of one
// launch shares the padded block size the kernel was compiled for.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btc {

struct WorkItem {
    int32_t inst;   // index into the descriptor array
    int32_t level;  // level of the node (ignored by per-row / per-instance kernels)
    int64_t k;      // node index within its level (block row for the residual)
};

template <class D>
struct Launch {
    D single;               // descriptor of the implicit-item launch
    const D* descs;         // explicit mode: descriptor array (device)
    const WorkItem* items;  // explicit mode: item array (device); nullptr = implicit
    int32_t level;          // implicit mode: level of every item
};

template <class D>
__device__ __forceinline__ void fetch_item_at(const Launch<D>& P, int64_t idx, D& d, int& level, int64_t& k) {
    if (P.items) {
        const WorkItem it = P.items[idx];
        d = P.descs[it.inst];
        level = it.level;
        k = it.k;
    } else {
        d = P.single;
        level = P.level;
        k = idx;
    }
}

template <class D>
__device__ __forceinline__ void fetch_item(const Launch<D>& P, D& d, int& level, int64_t& k) {
    fetch_item_at(P, blockIdx.x, d, level, k);
}

// Renumbering of a one-dimensional grid under which consecutive numbers
// run on the same XCD at about the same time (blocks are dispatched to the
// 8 XCDs round-robin, each XCD with its own L2): work that shares data
// should take consecutive numbers.
__device__ __forceinline__ unsigned xcd_local_block() {
    constexpr unsigned kXcd = 8;
    const unsigned g = gridDim.x, b = blockIdx.x;
    const unsigned x = b % kXcd, per = g / kXcd, rem = g % kXcd;
    return x * per + (x < rem ? x : rem) + b / kXcd;
}

// Factorization of one instance.  FP64 path: S_i then L_ii in Ld, couplings
// then R_i / T_i in Rb / Tb.  Mixed path: FP64 Schur complements in Ld, FP32
// factor in L32 / R32 / T32.  All arrays [N][n][n], permuted order.
struct FactorDesc {
    const double* A_diag;      // [N][n][n] user input (lower triangles)
    const double* A_off;       // [N-1][n][n] user input
    double* Ld;
    double* Rb;
    double* Tb;
    float* L32;
    float* R32;
    float* T32;
    unsigned long long* info;  // ~0 = ok, else smallest failing 1-based block
    int64_t N;
    int32_t n;
    int32_t flags;  // kFactorEagerT | kFactorDeferredDone
};

// Sweeps of one instance; T is the storage type of the factor and vectors.
template <class T>
struct SweepDesc {
    const T* Ld;
    const T* Rb;
    const T* Tb;
    const T* B;                // [N][n][m] right-hand side (original order)
    const double* B64;         // optional: read the right-hand side from this FP64 array instead
    T* X;                      // [N][n][m] solution (original order)
    T* Y;                      // [N][n][m] permuted: forward-sweep result y
    T* U;                      // [N][n][m] permuted: R_i y_i left for i+s
    T* V;                      // [N][n][m] permuted: T_i^T y_i left for i-s
    double* X64;               // optional: X64 = X (first) or X64 += X after the backward sweep
    const unsigned long long* info;
    const int* skip;           // optional: the item does nothing while *skip != 0
    int64_t N;
    int32_t n;
    int32_t m;
    int32_t first;
    int32_t pad;
};

// Device-side state of iterative refinement of one solve.
struct IrState {
    int done;        // no further refinement work (converged, stalled, NaN or budget spent)
    int steps;       // low-precision solves applied so far
    int converged;   // max column relative residual <= tol
    int stalled;     // last step reduced the residual by less than 2x
    double relres;   // max over columns of ||b - Psi x||_2 / ||b||_2 after the last step
    double prev;
    double tol;
    int max_steps;
    int pad;
};

// FP64 residual of one instance (items: k = 0-based block row).
struct ResidualDesc {
    const double* A_diag;
    const double* A_off;
    const double* B;           // [N][n][m] FP64 right-hand side
    const double* X;           // [N][n][m] FP64 iterate
    float* R32;                // optional: residual rounded to FP32
    double* part;              // [N][m][2] squared column norms of r_i and b_i per block row
    double* P;                 // [N][n][m] scratch: b_i - D_i x_i - E_i^T x_{i+1}
    double* Q;                 // [N][n][m] scratch: row i holds E_{i-1} x_{i-1} (i >= 2)
    const IrState* state;      // optional: skip when state->done
    double* R64;               // optional: the residual in FP64 (negated when neg: Psi x - b)
    int64_t N;
    int32_t n;
    int32_t m;
    int32_t neg;
    int32_t pad;
};

// Refinement set-up / convergence test of one instance (items: one per instance).
struct IrDesc {
    IrState* state;
    const double* part;        // [N][m][2]
    const double* B;           // FP64 right-hand side (set-up)
    float* R32;                // FP32 copy of B (set-up; may be null)
    int64_t N;
    int32_t n;
    int32_t m;
    double tol;
    int32_t max_steps;
    int32_t pad;
};

// Sequential elimination of the chain of blocks that remain after the first
// k levels of the multi-stage order (k = 0: the whole chain, Algorithm 1),
// and its solve (btc_chain.hip).  Factor arrays as FactorDesc (FP64 path);
// vectors as SweepDesc<double>.
struct ChainDesc {
    const double* A_diag;
    const double* A_off;
    double* Ld;
    double* Rb;
    double* Tb;
    unsigned long long* info;
    const double* B;   // solve: right-hand side [N][n][m] (original order)
    double* X;         // solve: solution [N][n][m]
    double* Y;         // solve: forward results, permuted
    const double* U;   // solve: contributions of the first k levels (as SweepDesc)
    const double* V;
    int64_t N;
    int32_t n;
    int32_t k;
    int32_t m;
    int32_t parts;  // partition order: number of chunks p (0: a k-stage chain)
    int64_t n1;     // partition order: blocks of the first chunk
    int64_t nk;     // partition order: blocks of every other chunk
};
hipError_t launch_chain_factor(const ChainDesc& p, int np, hipStream_t st);
hipError_t launch_chain_solve(const ChainDesc& p, int np, hipStream_t st);
// Partition order (Algorithm 2): the chunks in parallel, then the chain of
// the p - 1 separating blocks.
hipError_t launch_part_factor(const ChainDesc& p, int np, hipStream_t st);
hipError_t launch_part_solve(const ChainDesc& p, int np, hipStream_t st);

// FactorDesc.flags (tile-parallel families).  Eager: the Schur update of a
// node's right separator S_{i+s} also subtracts T'^T T' of the node's right
// neighbour at the same level (T' = T_{i+2s}, the separator's other
// contribution), so no update of a later level is deferred.  Deferred done:
// the previous level ran eagerly, this level has no deferred updates.
constexpr int32_t kFactorEagerT = 1;
constexpr int32_t kFactorDeferredDone = 2;

// Padded compute tile for block size n (0 when unsupported).
int padded_block(int n);
int padded_block_mixed(int n);

hipError_t launch_factor_valu(const Launch<FactorDesc>& p, int np, int64_t items, hipStream_t st);
hipError_t launch_factor_mfma(const Launch<FactorDesc>& p, int np, int64_t items, hipStream_t st);
// bf16: Schur / fill products with BF16 operands (FP32 accumulation)
hipError_t launch_factor_mixed(const Launch<FactorDesc>& p, int np, bool bf16, int64_t items, hipStream_t st);
// Padded sizes 64 to 128: three tile-parallel launches per level (deferred
// false skips the deferred-update launch: level 0, or every item's previous
// level ran eagerly).
// mode: 0 FP64, 1 mixed, 2 mixed with BF16 Schur / fill products; part 0 the
// whole level step, 1..3 one of its three kernels (in that order).
hipError_t launch_factor_tiled(const Launch<FactorDesc>& p, int np, int mode, int part, bool deferred,
                               int64_t items, hipStream_t st);
// mc: right-hand-side columns per dependency-chain group (1 or 4; with 4,
// instances with fewer columns mask the rest).  chunk: the items are
// subtrees of several levels (level field l0 | l1 << 8, k the subtree index
// j: the nodes of levels l0 .. l1-1 strictly between blocks j 2^l1 and
// (j+1) 2^l1), one workgroup of kw (4 or 8) wavefronts each; else single
// nodes, one wavefront each.
hipError_t launch_sweep(const Launch<SweepDesc<double>>& p, int np, int64_t items, bool backward, int mc,
                        hipStream_t st, bool chunk = false, int kw = 4);
hipError_t launch_sweep(const Launch<SweepDesc<float>>& p, int np, int64_t items, bool backward, int mc,
                        hipStream_t st, bool chunk = false, int kw = 4);
// Two launches over the same items (every block row of each instance).
hipError_t launch_residual(const Launch<ResidualDesc>& p, int np, int64_t items, int mc, hipStream_t st);
hipError_t launch_ir_init(const Launch<IrDesc>& p, int64_t items, hipStream_t st);
hipError_t launch_ir_check(const Launch<IrDesc>& p, int64_t items, hipStream_t st);

// FP64 vector kernels of the GMRES correction solve.  A vector is `rows`
// rows of m columns ([rows][m], row-major); a basis of k vectors is k such
// vectors at stride rows*m.  Reductions run in a fixed order (per-workgroup
// partial sums, then one workgroup in workgroup order), so results are
// reproducible.
//   dots: h[i*m + q] = sum_r V_i[r][q] z[r][q] for i < k, and with self,
//         h[k*m + q] = sum_r z[r][q]^2 (part: kGmresBlocks*(k+1)*m scratch)
//   update: z[r][q] -= sum_{i<k} h[i*m+q] V_i[r][q]
//   scale: dst[r][q] = src[r][q] * s[q]
//   combine: x[r][q] += sum_{j<k} y[j*m+q] V_j[r][q]
//   fill: x[e] = v for e < count
constexpr int kGmresBlocks = 256;
hipError_t launch_gmres_dots(const double* V, int k, const double* z, bool self, int64_t rows, int m, double* part,
                             double* h, hipStream_t st);
hipError_t launch_gmres_update(const double* V, int k, const double* h, double* z, int64_t rows, int m,
                               hipStream_t st);
hipError_t launch_gmres_scale(const double* src, const double* s, double* dst, int64_t rows, int m, hipStream_t st);
hipError_t launch_gmres_combine(const double* V, int k, const double* y, double* x, int64_t rows, int m,
                                hipStream_t st);
hipError_t launch_fill(double* x, double v, int64_t count, hipStream_t st);

}  // namespace btc
