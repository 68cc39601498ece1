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

// One level of a forward or backward sweep of one instance.
struct SolveParams {
    const double* Ld;
    const double* Rb;
    const double* Tb;
    const double* B;           // [N][n][m] user right-hand side (original order)
    double* X;                 // [N][n][m] user solution (original order)
    double* Y;                 // [N][n][m] permuted: forward-sweep result y
    double* U;                 // [N][n][m] permuted: R_i y_i left for i+s
    double* V;                 // [N][n][m] permuted: T_i^T y_i left for i-s
    const unsigned long long* info;
    int64_t N;
    int32_t n;
    int32_t m;
    int32_t level;
};

// Padded compute tile for block size n (0 when unsupported).
int padded_block(int n);

hipError_t launch_factor_level_f64(const FactorParams& p, int64_t nodes, hipStream_t st);
// Matrix-core variant for padded block sizes 16, 32, 64.
hipError_t launch_factor_level_mfma(const FactorParams& p, int64_t nodes, hipStream_t st);
hipError_t launch_solve_level_f64(const SolveParams& p, int64_t nodes, bool backward, hipStream_t st);

}  // namespace btc
