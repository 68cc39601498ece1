// Internal interface between the libbtc host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btc {

// One level of the factorization of one instance.
struct FactorParams {
    const double* A_diag;      // [N][n][n] user input (lower triangles)
    const double* A_off;       // [N-1][n][n] user input
    double* Ld;                // [N][n][n] permuted: S_i, then L_ii
    double* Rb;                // [N][n][n] permuted: right coupling, then R_i
    double* Tb;                // [N][n][n] permuted: left coupling, then T_i
    unsigned long long* info;  // ~0 = ok, else smallest failing 1-based block
    int64_t N;
    int32_t n;
    int32_t level;
};

// Mixed-precision factor storage: S_i in FP64 during the elimination, the
// factor itself (L_ii, R_i, T_i and the fill couplings) in FP32.
struct FactorParamsMixed {
    const double* A_diag;      // [N][n][n] user input (lower triangles)
    const double* A_off;       // [N-1][n][n] user input
    double* S64;               // [N][n][n] permuted: running Schur complements (FP64)
    float* L32;                // [N][n][n] permuted: L_ii rounded to FP32
    float* R32;                // [N][n][n] permuted: right coupling, then R_i
    float* T32;                // [N][n][n] permuted: left coupling, then T_i
    unsigned long long* info;
    int64_t N;
    int32_t n;
    int32_t level;
};

// One level of a forward or backward sweep of one instance; T is the storage
// type of the factor and of the vectors (double or float).
template <class T>
struct SweepParams {
    const T* Ld;
    const T* Rb;
    const T* Tb;
    const T* B;                // [N][n][m] right-hand side (original order)
    T* X;                      // [N][n][m] solution (original order)
    T* Y;                      // [N][n][m] permuted: forward-sweep result y
    T* U;                      // [N][n][m] permuted: R_i y_i left for i+s
    T* V;                      // [N][n][m] permuted: T_i^T y_i left for i-s
    double* X64;               // optional: X64 = X (first) or X64 += X after the backward sweep
    const unsigned long long* info;
    const int* skip;           // optional: the launch does nothing while *skip != 0
    int64_t N;
    int32_t n;
    int32_t m;
    int32_t level;
    int32_t first;
};

// Device-side state of iterative refinement.
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

struct ResidualParams {
    const double* A_diag;
    const double* A_off;
    const double* B;           // [N][n][m] FP64 right-hand side
    const double* X;           // [N][n][m] FP64 iterate
    float* R32;                // optional: residual rounded to FP32
    double* part;              // [N][m][2] squared column norms of r_i and b_i per block row
    const IrState* state;      // optional: skip when state->done
    int64_t N;
    int32_t n;
    int32_t m;
};

// Padded compute tile for block size n (0 when unsupported).
int padded_block(int n);

hipError_t launch_factor_level_f64(const FactorParams& p, int64_t nodes, hipStream_t st);
// Matrix-core variant for padded block sizes 16, 32, 64.
hipError_t launch_factor_level_mfma(const FactorParams& p, int64_t nodes, hipStream_t st);
hipError_t launch_factor_level_mixed(const FactorParamsMixed& p, int64_t nodes, hipStream_t st);
hipError_t launch_sweep(const SweepParams<double>& p, int64_t nodes, bool backward, hipStream_t st);
hipError_t launch_sweep(const SweepParams<float>& p, int64_t nodes, bool backward, hipStream_t st);
hipError_t launch_residual(const ResidualParams& p, hipStream_t st);
hipError_t launch_ir_check(IrState* state, const double* part, int64_t N, int m, hipStream_t st);
hipError_t launch_ir_init(IrState* state, double tol, int max_steps, const double* B, float* R32, size_t count,
                          hipStream_t st);

}  // namespace btc
