/*
 * btc.h -- C ABI of libbtc: nested-dissection Cholesky factorization and solve
 * of symmetric positive-definite block-tridiagonal matrices on AMD MI355X
 * (gfx950), after Schwan, Kuhn, Jones, "GPU-Accelerated Cholesky
 * Factorization of Block Tridiagonal Matrices" (arXiv 2601.03754).
 *
 * Problem (section "Sequential Cholesky Factorization"): Psi is N x N blocks
 * of size n x n, diagonal blocks D_1..D_N symmetric, sub-diagonal blocks
 * E_1..E_{N-1} with E_i at block position (i+1, i) and E_i^T at (i, i+1).
 * The library computes P Psi P^T = L L^T with the multi-stage (nested
 * dissection) permutation P of section "Multi-Stage Permutation"
 * (Algorithm 4: floor(log2 N)+1 levels of per-block potrf/trsm/syrk/gemm),
 * and solves Psi X = B with the level sweeps of section "Cholesky Solve"
 * (Algorithm 6).
 *
 * Memory: unless stated otherwise every array argument is a DEVICE pointer
 * (memory of the current HIP device), row-major, FP64, and owned by the
 * caller.  Layouts:
 *   A_diag  [N][n][n]   D_i at A_diag + (i-1)*n*n; only the LOWER triangle of
 *                       each block is read (the upper one may hold anything).
 *   A_off   [N-1][n][n] E_i at A_off + (i-1)*n*n (may be NULL when N == 1).
 *   B, X    [N][n][nrhs] block i, row r, column q at ((i-1)*n + r)*nrhs + q.
 * The library never writes A_diag, A_off or B.
 *
 * Streams: every call that launches work takes a hipStream_t (passed as
 * void*, NULL = the default stream) and returns as soon as the work is
 * enqueued; inputs must stay valid and unchanged until that work completes.
 * Calls that must read a device result (btc_status, a non-NULL
 * btc_solve_info) synchronise with the stream.
 *
 * Errors: functions return 0 on success, -k when argument k (1-based) is
 * invalid, or one of the negative BTC_ERR_* codes.  A numerical breakdown
 * (a pivot block that is not positive definite) is not an error code of
 * btc_factor, which returns before the device work completes; it is reported
 * by btc_status.
 */
#ifndef BTC_H
#define BTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef BTC_API
#define BTC_API __attribute__((visibility("default")))
#endif

#define BTC_OK 0
#define BTC_ERR_HIP (-100)          /* a HIP runtime call failed */
#define BTC_ERR_OOM (-101)          /* device memory allocation failed */
#define BTC_ERR_NOT_SPD (-102)      /* solve requested on a failed factorization */
#define BTC_ERR_UNSUPPORTED (-103)  /* block size or option not supported */

/* Largest supported block size n. */
#define BTC_MAX_BLOCK 128

typedef struct btc_handle_s *btc_handle; /* opaque; owned by the library */

/* Defaults of the refinement options (used when the field is 0). */
#define BTC_DEFAULT_MAX_REFINE 4
#define BTC_DEFAULT_MAX_REFINE_BF16 30
#define BTC_DEFAULT_TOL 1e-10

/*
 * Arithmetic of the factorization and solve.  The paper computes in one
 * precision throughout and names mixed precision as future work (section
 * "Conclusion"); BTC_FP32_IR is that extension:
 *   BTC_FP64     every step in FP64.
 *   BTC_FP32_IR  Schur complements and the Cholesky factorization of every
 *                pivot block in FP64; triangular solves, Schur/fill products
 *                and the solve sweeps in FP32 (matrix cores, FP32
 *                accumulation); the solution is refined in FP64: the residual
 *                b - Psi x is formed in FP64 from the original blocks and a
 *                correction solved in FP32 is added, until the target is met.
 *                The handle keeps pointers to A_diag and A_off for the
 *                residual, so they must stay valid and unchanged while the
 *                handle is used for solves.
 *   BTC_BF16_IR  as BTC_FP32_IR, but the Schur and fill products (syrk,
 *                gemm) take BF16 operands (round to nearest even) with FP32
 *                accumulation; more refinement steps are needed (default cap
 *                BTC_DEFAULT_MAX_REFINE_BF16).
 */
typedef enum {
    BTC_FP64 = 0,
    BTC_FP32_IR = 1,
    BTC_BF16_IR = 2
} btc_precision;

/*
 * How the mixed-precision paths compute each correction d of refinement
 * (the residual r = b - Psi x is always formed in FP64 from the original
 * blocks):
 *   BTC_REFINE_CLASSIC  d = (L L^T)^{-1} r with the low-precision factor
 *                       (one pair of sweeps per correction);
 *   BTC_REFINE_GMRES    d from GMRES in FP64 on (L L^T)^{-1} Psi d =
 *                       (L L^T)^{-1} r, the low-precision factor as the
 *                       preconditioner (Carson and Higham's GMRES-based
 *                       refinement): each iteration one FP64 product with
 *                       Psi and one pair of low-precision sweeps, the basis
 *                       orthogonalised twice (classical Gram-Schmidt) in
 *                       FP64; the correction stops when the preconditioned
 *                       residual has fallen by 1e-8 or after gmres_m
 *                       iterations.  For ill-conditioned systems, where the
 *                       classic correction contracts slowly or not at all
 *                       (BF16 products at condition numbers of 1e3 and
 *                       more).  btc_solve only (the runner and the server
 *                       refine classically); synchronises once per GMRES
 *                       iteration.
 */
#define BTC_REFINE_CLASSIC 0
#define BTC_REFINE_GMRES 1
#define BTC_DEFAULT_GMRES_M 40

/*
 * Elimination order (section "Parallel Cholesky Factorization"; the paper
 * compares the strategies and leaves choosing among them per problem to
 * future work, section "Multi-Stage Permutation"):
 *   BTC_STRATEGY_MULTISTAGE  the multi-stage (nested-dissection) order of
 *                            Algorithm 4: floor(log2 N)+1 parallel levels.
 *   BTC_STRATEGY_KSTAGE      the first `stages` levels of that order, then
 *                            the remaining chain of blocks (the multiples of
 *                            2^stages) eliminated one after the other by one
 *                            wavefront, as in Algorithm 1: stages = 0 is the
 *                            sequential Algorithm 1 (one launch for the
 *                            factor, one for the solve), 1 the single-stage
 *                            permutation, 2 the two-stage variant.  FP64, n
 *                            <= 64, btc_factor / btc_solve only.
 *   BTC_STRATEGY_AUTO        the fastest of these for (N, n) as measured by
 *                            btc_autotune_strategy (else MULTISTAGE).
 *   BTC_STRATEGY_PARTITION   the partition order of Algorithm 2 with
 *                            p = `stages` >= 2 chunks sized by Proposition 1
 *                            (the first chunk N_1 blocks, the others N_k,
 *                            one separating block between neighbours): every
 *                            chunk eliminated in natural order by its own
 *                            wavefront, all chunks at once, then the p - 1
 *                            separating blocks in order.  FP64, n <= 64,
 *                            btc_factor / btc_solve only; BTC_ERR_UNSUPPORTED
 *                            when N is too small for p chunks of at least one
 *                            block.
 * Every order computes the Cholesky factor of its own permuted matrix; the
 * solutions agree to rounding.
 */
#define BTC_STRATEGY_MULTISTAGE 0
#define BTC_STRATEGY_KSTAGE 1
#define BTC_STRATEGY_AUTO 2
#define BTC_STRATEGY_PARTITION 3

typedef struct {
    int32_t precision;   /* btc_precision */
    int32_t max_refine;  /* refinement corrections after the first solve (0: default) */
    double tol;          /* target max-column relative residual (0: default 1e-10) */
    int32_t refine;      /* BTC_REFINE_CLASSIC or BTC_REFINE_GMRES (mixed precision only) */
    int32_t gmres_m;     /* BTC_REFINE_GMRES: iterations per correction, 1..200 (0: default) */
    int32_t strategy;    /* BTC_STRATEGY_* (0: multi-stage) */
    int32_t stages;      /* BTC_STRATEGY_KSTAGE: levels of the multi-stage order before the chain;
                            BTC_STRATEGY_PARTITION: number of chunks p */
} btc_options;

typedef struct {
    int32_t steps;      /* refinement corrections applied (0 for BTC_FP64) */
    int32_t converged;  /* 1 if the residual target was met (always 1 for BTC_FP64) */
    double relres;      /* max over columns of ||b - Psi x||_2 / ||b||_2, FP64 */
    int32_t inner;      /* BTC_REFINE_GMRES: GMRES iterations over all corrections, else 0 */
    int32_t pad;
} btc_solve_info;

/*
 * btc_factor -- factor P Psi P^T = L L^T (section "Multi-Stage Permutation",
 * Algorithm 4) and return a handle that owns the factor.
 *   A_diag, A_off  device inputs as above (A_off ignored when N == 1)
 *   N >= 1, 1 <= n <= BTC_MAX_BLOCK
 *   opt            NULL for FP64 defaults
 *   stream         hipStream_t or NULL
 *   out            receives the new handle (host pointer, not NULL)
 * The handle allocates its device memory here, through the allocator set by
 * btc_set_allocator (default hipMalloc); it is freed by btc_destroy.
 * Argument errors: -1..-7 for the argument at that position (-5 for an
 * unknown precision or a negative max_refine / tol).
 */
BTC_API int btc_factor(const double *A_diag, const double *A_off, int64_t N, int64_t n,
               const btc_options *opt, void *stream, btc_handle *out);

/*
 * btc_create -- allocate a handle for systems of this shape and precision
 * without factoring anything yet (for btc_refactor, the batched entry points
 * and the step runner).  Same argument rules as btc_factor.
 */
BTC_API int btc_create(int64_t N, int64_t n, const btc_options *opt, btc_handle *out);

/*
 * btc_refactor -- factor a new matrix of the same (N, n) into an existing
 * handle, reusing its device memory (repeated factorizations, e.g. the
 * re-linearised systems of successive model-predictive-control steps).
 */
BTC_API int btc_refactor(btc_handle h, const double *A_diag, const double *A_off, void *stream);

/*
 * btc_solve -- solve Psi X = B with the handle's factor: forward sweep over
 * the levels in ascending order, backward sweep in descending order
 * (section "Cholesky Solve", Algorithm 6); with BTC_FP32_IR followed by FP64
 * iterative refinement (see btc_precision).
 *   B, X    device [N][n][nrhs]; X may alias B for BTC_FP64 only
 *   nrhs >= 1 (nrhs == 0 is a no-op)
 *   info    NULL, or a host struct; when non-NULL the call synchronises with
 *           the stream and fills it (for BTC_FP64 it also computes the FP64
 *           relative residual of the solution).
 * Refinement stops on its own on the device (no host synchronisation) once
 * the target is met, once a step reduces the residual by less than 2x, or
 * after max_refine corrections; the launches of rounds after the stop exit
 * at once.  When info is given (the call waits for the result anyway), the
 * rounds after the first correction are enqueued only while the refinement
 * has not stopped (one small device-to-host read per round).  Returns BTC_ERR_NOT_SPD (without writing X)
 * if the factorization is known to have broken down.
 * Concurrency: once the factorization has completed, the factor is only
 * read, and solves of one handle may run concurrently on different streams:
 * a solve uses the handle's workspace on the stream that last used it, or on
 * another stream when the last solve that used it has finished; otherwise it
 * takes a workspace of its own from the allocator (btc_set_allocator) for the
 * duration of the call, released in stream order.  Calls from several host
 * threads on one handle must be serialised by the caller.
 */
BTC_API int btc_solve(btc_handle h, const double *B, double *X, int64_t nrhs, void *stream,
              btc_solve_info *info);

/*
 * btc_solve_noalloc -- btc_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops or harnesses that must
 * not call hipMalloc or a framework allocator): the same kernels and results
 * as btc_solve, with the solve workspace in a fixed device array of the
 * library (BTC_NOALLOC_MAX_BYTES, one per GPU the library runs on, held until
 * the process ends) instead of allocated memory.  The workspace needs
 * 40 N n nrhs + 16 N nrhs + 1024 bytes (FP64) or 36 N n nrhs + 16 N nrhs +
 * 1024 (mixed precision), as btc_footprint_bytes counts it; larger requests
 * return BTC_ERR_UNSUPPORTED without enqueuing anything.  The current device
 * must be the handle's (-1 otherwise).  Every call on one GPU shares that
 * array: calls whose work overlaps on one GPU (other streams, other handles)
 * race and must be ordered by the caller.  Allocates nothing, also when info
 * is given.
 */
#define BTC_NOALLOC_MAX_BYTES (64u << 20)
BTC_API int btc_solve_noalloc(btc_handle h, const double *B, double *X, int64_t nrhs, void *stream,
                              btc_solve_info *info);

/*
 * btc_status -- synchronise with the handle's last stream and report the
 * numerical outcome of the last factorization: *info = 0 if every pivot block
 * was positive definite, otherwise the 1-based ORIGINAL index of the first
 * failing block in elimination order (lowest level first, then smallest
 * index).
 */
BTC_API int btc_status(btc_handle h, int64_t *info);

/* btc_destroy -- wait for the handle's work on every stream it was used
 * on, then free the handle and its device memory (NULL is a no-op). */
BTC_API void btc_destroy(btc_handle h);

/*
 * btc_footprint_bytes -- device bytes a handle of this shape holds after one
 * solve with nrhs right-hand sides (for admission control).  0 on invalid
 * arguments.
 */
BTC_API size_t btc_footprint_bytes(int64_t N, int64_t n, int32_t precision, int64_t nrhs);

/*
 * btc_export_factor -- copy the factor to HOST arrays, indexed by ORIGINAL
 * block index (slot i-1 holds block i), each [N][n][n]:
 *   Ld[i] = L_ii (lower; strict upper triangle returned as 0)
 *   Rb[i] = R_i = factor block at (row i+s, column i), zero if i+s > N
 *   Tb[i] = T_i = transpose of the factor block at (row i-s, column i),
 *           zero if i <= s
 * where s = 2^(number of trailing zero bits of i).  For a k-stage order the
 * blocks of its chain (the multiples of 2^k) have Rb[i] = the factor block
 * at (row i + 2^k, column i) (zero for the last) and Tb[i] = 0.  Synchronises.
 * Any of the three pointers may be NULL.  For BTC_FP32_IR the FP32 factor
 * blocks are returned (widened to FP64).
 */
BTC_API int btc_export_factor(btc_handle h, double *Ld, double *Rb, double *Tb);

/*
 * btc_permutation -- the multi-stage permutation as a HOST array:
 * order[p] = 1-based original index of the block at permuted position p
 * (all odd blocks, then the odd multiples of 2, of 4, ...).
 */
BTC_API int btc_permutation(int64_t N, int64_t *order);

/*
 * btc_profile -- switch per-launch kernel timing of a handle on (1) or off
 * (0).  While on, every kernel the handle launches is bracketed by two HIP
 * events recorded on its launch stream; switching on clears the totals.
 */
BTC_API int btc_profile(btc_handle h, int enable);

/*
 * btc_profile_read -- synchronise with the handle's stream and report the
 * accumulated kernel time since profiling was switched on, per level, for
 * one phase: 0 = factorization, 1 = forward sweep, 2 = backward sweep,
 * 3 = refinement (entry 0: set-up, 1: residual, 2: convergence test).
 *   ms[l], counts[l] (host arrays of max_levels entries, either may be NULL):
 *   total milliseconds and number of launches of that phase at level l.
 * Returns the number of levels of the handle (>= 0) or an error code.
 */
BTC_API int btc_profile_read(btc_handle h, int phase, double *ms, int64_t *counts, int max_levels);

/* ------------------------------------------------------------------------
 * Many instances per launch.
 *
 * The elimination of section "Multi-Stage Permutation" is a sequence of
 * level steps; steps of different instances are independent.  A runner
 * executes a list of level steps of many handles (of any sizes, at any
 * levels) with one kernel launch per operation and block-size class, each
 * launch carrying the work items (nodes, block rows) of all its steps.
 * Batched factorization / solve of independent instances and continuous
 * batching of requests (new requests joining while others are mid-tree) are
 * built on it.  All runner work is enqueued on the runner's stream; handles
 * used with a runner adopt that stream.
 */
typedef struct btc_runner_s *btc_runner;

typedef enum {
    BTC_OP_FACTOR = 0,       /* one level of the factorization (level 0 also resets the status) */
    BTC_OP_FORWARD = 1,      /* one level of the forward sweep */
    BTC_OP_BACKWARD = 2,     /* one level of the backward sweep */
    BTC_OP_RESIDUAL = 3,     /* FP64 residual b - Psi x and its column norms */
    BTC_OP_REFINE_INIT = 4,  /* reset the refinement state of a solve */
    BTC_OP_REFINE_TEST = 5   /* convergence test of the refinement */
} btc_op;

typedef struct {
    btc_handle h;
    int32_t op;             /* btc_op */
    int32_t level;          /* FACTOR / FORWARD / BACKWARD: level 0 .. floor(log2 N) (the first
                               level of a range, see level_end) */
    const double *A_diag;   /* FACTOR at level 0: the matrix (device; kept for RESIDUAL) */
    const double *A_off;
    const double *B;        /* sweeps / RESIDUAL: right-hand side [N][n][nrhs] (device) */
    double *X;              /* sweeps / RESIDUAL: solution / iterate (device) */
    int64_t nrhs;           /* >= 1 for every op but FACTOR */
    int32_t first;          /* BTC_FP32_IR sweeps: 1 for the first solve (reads B, sets X) */
    int32_t level_end;      /* FORWARD / BACKWARD: 0 for the single level `level`; else the
                               levels level .. level_end-1 in one step (level < level_end <=
                               floor(log2 N)+1): the elimination subtrees of those levels, one
                               workgroup each (btc_sweep_ranges gives the library's ranges) */
    int32_t stage;          /* 0..7: order of dependent steps within one call */
    int32_t pad;
} btc_step;

/* btc_runner_create -- a runner enqueuing on `stream` (hipStream_t or NULL). */
BTC_API int btc_runner_create(void *stream, btc_runner *out);

/*
 * btc_runner_run -- enqueue `count` steps (host array).  The steps of one
 * call run stage by stage (all steps of stage 0, then of stage 1, ...);
 * steps of one stage must not depend on each other: at most one step per
 * handle per stage, except that FACTOR level l and a FORWARD range ending at
 * level l (level_end, or level + 1) of one handle may share a stage (the
 * sweep reads only factor blocks below level l, the factor step writes only
 * blocks of level l and above), and so may a RESIDUAL and the REFINE_TEST
 * that reads it (REFINE_TEST steps run after every other step of their
 * stage).  A step that depends on another step of the same call (a sweep
 * after REFINE_INIT or after the test that may stop it, a residual after the
 * backward sweep) goes in a later stage.  Calls are executed in order.
 * Returns once the work is enqueued; -3 for an invalid step (unknown op,
 * level or range out of range, stage outside 0..7, missing pointers, a sweep
 * or residual on a handle never factored).
 */
BTC_API int btc_runner_run(btc_runner r, int32_t count, const btc_step *steps);

/*
 * btc_sweep_ranges -- the level ranges in which the library runs a sweep of
 * an instance with N blocks (host computation): bounds[0] = 0 < bounds[1] <
 * ... < bounds[r] = floor(log2 N)+1, r returned (bounds needs r+1 <= max
 * entries; -2 if it is too short).  A range of one level runs one wavefront
 * per node; a longer range runs each elimination subtree of its levels in
 * one workgroup (section "Cholesky Solve": the forward step of a node reads
 * only results of its descendants, the backward step only those of its
 * ancestors), so it costs one launch and one dependency step instead of one
 * per level.
 */
BTC_API int btc_sweep_ranges(int64_t N, int32_t *bounds, int32_t max);

/* btc_runner_query -- 1 if all enqueued work has finished, 0 if not. */
BTC_API int btc_runner_query(btc_runner r);

/* btc_runner_sync -- wait for all enqueued work. */
BTC_API int btc_runner_sync(btc_runner r);

/* btc_runner_host_stats -- host time spent in btc_runner_run since the
 * runner was created (or last reset): *run_s in total, *wait_s of it blocked
 * until the device released a descriptor staging slot (the runner keeps two;
 * a call waits when the call two before it has not finished on the device),
 * *calls the number of calls (any pointer may be NULL).  reset != 0 clears
 * the counters after reading them. */
BTC_API int btc_runner_host_stats(btc_runner r, double *run_s, double *wait_s, int64_t *calls, int reset);

/* btc_runner_destroy -- wait for the runner's work and free it (NULL: no-op). */
BTC_API void btc_runner_destroy(btc_runner r);

/*
 * Level schedules as HIP graphs.  btc_graph_begin(r) makes the runner record
 * instead of run: every following btc_runner_run, btc_factor_batched and
 * btc_solve_batched call on r is validated, its workspaces are allocated and
 * its launches are planned, but nothing is enqueued.  btc_graph_end(r, &g)
 * uploads the planned descriptors once (synchronising r's stream first) and
 * captures all recorded launches (each call's independent groups on several
 * streams) into an instantiated HIP graph; btc_graph_launch(g, stream)
 * replays it with no host work per level.  A replay reads whatever the
 * recorded A_diag / A_off / B arrays hold at that time and writes the recorded
 * X arrays and factors: the repeated factor+solve of an MPC loop with new
 * values in the same buffers.  The recorded handles must stay alive and keep
 * their workspaces (a handle may not be given more right-hand sides than at
 * recording while a graph of it exists; growing one inside a recording is
 * refused with BTC_ERR_UNSUPPORTED).  Replays on one stream are ordered;
 * replays of one graph must not run concurrently.
 */
typedef struct btc_graph_s *btc_graph;

BTC_API int btc_graph_begin(btc_runner r);
BTC_API int btc_graph_end(btc_runner r, btc_graph *out);
BTC_API int btc_graph_launch(btc_graph g, void *stream);
BTC_API void btc_graph_destroy(btc_graph g);

/*
 * Autotuned kernel variants (a process-wide table; until set, variant 1 for
 * the factor at n 33..64 and 0 everywhere else),
 * keyed by operation, precision, block size n (through its padded size) and
 * level (bucket: level 0, levels >= 1):
 *   BTC_OP_FACTOR, BTC_FP64, n 9..32: 0 matrix-core kernel, 1 vector-ALU
 *     kernel, and for n 17..32 also 2 the tile-parallel level step; mixed
 *     precisions, n 17..32, and any precision, n 33..64: 0 one workgroup per
 *     node, 1 the tile-parallel level step (different rounding orders:
 *     results change at round-off level when the choice changes)
 *   BTC_OP_FORWARD / BACKWARD / RESIDUAL (nrhs > 1; level ignored): 0 four
 *     right-hand-side columns per dependency-chain group, 1 one (identical
 *     results)
 *   BTC_TUNE_SWEEP_SHAPE, any precision, any n (level ignored): the launch
 *     shape of both sweeps: 0 level ranges (btc_sweep_ranges) with
 *     workgroups of 4 wavefronts, 1 one launch per level, 2 level ranges
 *     with workgroups of 8 wavefronts (ranges one level deeper); identical
 *     results
 * With the environment variable BTC_TUNE_CACHE naming a file, the table
 * (kernel variants and the strategy choices of btc_autotune_strategy) is
 * read from that file when the library first consults it, and written back
 * after every btc_tune_set / btc_autotune / btc_autotune_strategy (text, one
 * entry per line).
 * Other keys have the single variant 0 (btc_tune_set accepts only 0 there).
 * btc_autotune times every variant of the handle's tunable families on the
 * caller's matrix (reps timed repetitions after one warm-up each, per-level
 * HIP events; the sweep shape by the time of whole solves) and stores the
 * fastest per key; it refactors the handle and overwrites X.  B and X are device arrays [N][n][nrhs], B != X.  Call it
 * once at start-up: results computed before and after may differ at
 * round-off level.  Returns 0 or -k for argument k.
 */
#define BTC_TUNE_SWEEP_SHAPE 6 /* tune key: launch shape of the sweeps (op field; level ignored) */
/*
 * btc_autotune_batched -- tune the table for a batch of instances as
 * btc_factor_batched / btc_solve_batched run it (one launch per level
 * carrying the nodes of every instance favours other variants than one
 * instance alone): every key the batch touches (factor per level bucket,
 * sweep shape, and with more than one right-hand side the sweeps and the
 * residual) is tried variant by variant on the whole batched factor + solve,
 * the other keys at their current choice, and the fastest kept (median of
 * reps timed calls after one warm-up; one pass of coordinate descent).
 * Arguments as btc_factor_batched and btc_solve_batched (B[k] != X[k]);
 * leaves every instance factored and solved with the final choices and
 * writes the BTC_TUNE_CACHE file if set.  Returns 0, -k for argument k, or
 * an error of the batched calls.
 */
BTC_API int btc_autotune_batched(btc_runner r, int32_t count, const btc_handle *h, const double *const *A_diag,
                                 const double *const *A_off, const double *const *B, double *const *X,
                                 const int64_t *nrhs, int32_t reps);
BTC_API int btc_tune_get(int32_t op, int32_t precision, int64_t n, int32_t level, int32_t *variant);
BTC_API int btc_tune_set(int32_t op, int32_t precision, int64_t n, int32_t level, int32_t variant);
BTC_API int btc_autotune(btc_handle h, const double *A_diag, const double *A_off, const double *B, double *X,
                         int64_t nrhs, int32_t reps, void *stream);

/*
 * Launch profiler of a runner.  While on, the algorithmic work of every
 * launch (btc_level_work summed over the steps of the launch) is added to the
 * totals of its (op, kernel family, padded block size), and every launch of a
 * selected group is also bracketed by two HIP events recorded on the stream
 * it runs on (ms stays 0 for groups not selected).  The independent groups of
 * one btc_runner_run call run concurrently on the runner's stream and up to
 * three side streams (created with the runner on the current device, default
 * priority), so a timed launch may share the GPU with others.
 *   btc_runner_profile(r, op, kind): op -2 switches off, -1 selects every
 *   group, >= 0 one btc_op; kind -1 any kernel family, else that family
 *   (FACTOR: 0 FP64 VALU, 1 FP64 MFMA, 2 mixed, 3 FP64 tile-parallel,
 *   4 mixed tile-parallel; sweeps: 0 FP64, 1 FP32).  Synchronises and
 *   clears the totals.
 *   btc_runner_profile_read(r, out, max, count): synchronises and writes up
 *   to max totals (host array), largest time first, then clears them.
 * A timed tile-parallel factor group is timed kernel by kernel (part 1..3,
 * each with its own algorithmic work: the kernels pass S and the factor
 * blocks through HBM between them).
 */
typedef struct {
    int32_t op;        /* btc_op */
    int32_t kind;      /* kernel family, as above */
    int32_t np;        /* padded block size of the kernel */
    int32_t part;      /* tile-parallel factor, timed: 1 deferred syrk, 2 pivot factorization and
                          triangular solves, 3 separator / fill products; else 0 (whole launch) */
    int64_t launches;
    int64_t items;     /* nodes (sweeps, factor), block rows (residual) */
    double ms;         /* summed event time (0 for groups not timed) */
    double bytes;      /* algorithmic bytes (btc_level_work) */
    double flops;      /* algorithmic flops (btc_level_work) */
} btc_kernel_stat;

BTC_API int btc_runner_profile(btc_runner r, int32_t op, int32_t kind);
BTC_API int btc_runner_profile_read(btc_runner r, btc_kernel_stat *out, int32_t max, int32_t *count);

/*
 * btc_level_work -- algorithmic work of one step (host computation, no
 * device access): HBM bytes and flops of level `level` of op FACTOR /
 * FORWARD / BACKWARD, or of a whole RESIDUAL / REFINE_* step (level
 * ignored), for a (N, n, nrhs) instance at the given precision.
 *   Factor, per node i of level l (stride s): every n x n block the level
 *   step of Algorithm 4 reads (S_i, S_{i+s}, the couplings, the deferred
 *   T blocks of level l-1) or writes (L_ii, R_i, T_i, S_{i+s}, the fill)
 *   counted once; flops n^3/3 (potrf) + n^3 per triangular solve and per
 *   syrk + 2n^3 per fill (section "Computational Complexity").
 *   Sweeps (Algorithm 6): the node's factor blocks once, its n x nrhs
 *   vectors; flops n^2 nrhs per triangular solve, 2 n^2 nrhs per product.
 *   Residual: 8 n^2 (2N-1) + 24 N n nrhs bytes, 2 n^2 nrhs (3N-2) flops.
 * Word size 8 (FP64); BTC_FP32_IR: 4 for factor blocks, fills and sweep
 * vectors, 8 for Schur complements, inputs and the residual.
 * Returns 0, or -k for argument k out of range.
 */
BTC_API int btc_level_work(int32_t op, int32_t precision, int64_t N, int64_t n, int64_t nrhs, int32_t level,
                           double *bytes, double *flops);

/*
 * btc_factor_batched -- factor `count` independent instances (handles from
 * btc_create, of any shapes and precisions; host arrays of device pointers),
 * walking their levels together: one group of launches per level, each
 * launch carrying the nodes of every instance at that level.  The batched
 * calls take a runner rather than a stream: the runner is the stream plus
 * the side streams and staging buffers its launches use, and it is what a
 * HIP graph of the level schedule is recorded from (btc_graph_begin).
 *   info   NULL, or a host array of count entries: synchronises with the
 *          runner and writes each instance's status as btc_status does.
 */
BTC_API int btc_factor_batched(btc_runner r, int32_t count, const btc_handle *h, const double *const *A_diag,
                               const double *const *A_off, int64_t *info);

/*
 * btc_solve_batched -- solve `count` independent instances, instance k with
 * nrhs[k] >= 1 columns (host array); BTC_FP32_IR / BTC_BF16_IR handles are
 * refined in FP64 as in btc_solve (X must not alias B for them).
 *   info   NULL, or a host array of count entries: synchronises with the
 *          runner and fills each as btc_solve_info (an instance whose factor
 *          broke down gets steps = 0, converged = 0, relres = -1).
 * Without info: status per handle btc_status, refinement outcome
 * btc_refine_info.  Inside a graph recording (btc_graph_begin) info must be
 * NULL.
 */
BTC_API int btc_solve_batched(btc_runner r, int32_t count, const btc_handle *h, const double *const *B,
                              double *const *X, const int64_t *nrhs, btc_solve_info *info);

/*
 * btc_refine_info -- synchronise with the handle's stream and report the
 * outcome of its last solve made through a runner (steps, converged, relres
 * as in btc_solve_info).
 */
BTC_API int btc_refine_info(btc_handle h, btc_solve_info *info);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of factor and solve requests.
 *
 * Not part of the paper, which factors one system at a time; it serves the
 * use the paper motivates (repeated solves of structured systems in model
 * predictive control).  A client owns one system shape (N, n) and a factor
 * kept resident on the device.  Requests are "refactor + solve" (a new matrix
 * of the client's shape) or "solve" (against the resident factor).  Every
 * btc_server_step call admits queued requests and enqueues the next level
 * step of every request in flight as one runner call, so requests at
 * different levels and phases share launches and new requests join at the
 * next step.  A refactor+solve request runs its first forward sweep
 * interlaced with the factorization (forward level l in the tick of factor
 * level l+1; section "Fused and Blocked Kernels").  Admission is in arrival order, one request in flight per
 * client (so a client's requests complete in order), within an HBM budget on
 * the resident factors + workspaces: idle clients are evicted least recently
 * used first, and a later "solve" of an evicted client is run as
 * "refactor + solve" with its last matrix (which must therefore stay valid).
 * Mixed-precision requests are refined in FP64 as by btc_solve; a request
 * whose refinement has converged is retired as soon as its flag comes back.
 * Times are host steady-clock seconds.
 */
typedef struct btc_server_s *btc_server;

typedef struct {
    int32_t precision;   /* btc_precision of every client */
    int32_t max_refine;  /* as in btc_options (0: default) */
    double tol;          /* as in btc_options (0: default) */
    size_t hbm_budget;   /* bytes for resident factors + workspaces (btc_footprint_bytes) */
    int32_t max_active;  /* cap on requests in flight (0: no cap) */
    int32_t sweep_ranges;  /* 0: one tick per sweep level; 1: sweeps in the library's level ranges
                              (btc_sweep_ranges), one tick per range (fewer ticks per request,
                              longer ticks: measured 4-6% fewer requests/s on the served mix) */
    int32_t lanes;         /* 1: one tick at a time over all clients on the server's stream, its
                              groups spread over four streams; 2..4: clients split by padded block
                              size class (<= 16, 32, 64, 96 and 128) into that many lanes, each
                              with its own ticks on a stream the server creates, so a lane of small
                              blocks is not held to the pace of the largest; every lane tick first
                              waits for the work queued on the server's stream so far (the
                              requests' inputs); 0: the library's choice, three lanes */
} btc_server_options;

typedef struct {
    int64_t ticket;
    int64_t client;
    double t_submit;     /* btc_server_submit */
    double t_admit;      /* admission (memory and the client's previous request permitting) */
    double t_done;       /* the device finished the request's last step (observed by step/poll) */
    int32_t refactored;  /* 1 if the request factored (new matrix, or a re-admitted client) */
    int32_t converged;   /* 1 if the result met the target: mixed precision, the refinement's
                            residual test passed; FP64, the factorization succeeded */
    int64_t info;        /* status of the client's factor as btc_status reports it (0: ok,
                            k > 0: block k not positive definite; X is then not written) */
    int32_t steps;       /* refinement corrections applied (0 for BTC_FP64) */
    int32_t pad;
    double relres;       /* mixed precision: the FP64 max-column relative residual of X as the
                            last convergence test measured it; FP64 path: -1 (not computed) */
} btc_server_completion;

BTC_API int btc_server_create(const btc_server_options *opt, void *stream, btc_server *out);

/* Register a client of shape (N, n); *client receives its id (0, 1, ...). */
BTC_API int btc_server_add_client(btc_server s, int64_t N, int64_t n, int64_t *client);

/*
 * Queue a request (device pointers, valid until the request completes):
 * A_diag / A_off non-NULL for "refactor + solve", NULL for "solve" (the first
 * request of a client must bring a matrix); B, X [N][n][nrhs].  A solve-only
 * request refers to the matrix of the client's previous refactorization
 * (requests of one client are admitted in submission order); if the client
 * was evicted meanwhile, that matrix is factored again, so it must stay valid
 * until a later refactorization of the client has completed.  Returns
 * BTC_ERR_UNSUPPORTED when the request's footprint (btc_footprint_bytes)
 * alone exceeds the HBM budget.
 */
BTC_API int btc_server_submit(btc_server s, int64_t client, const double *A_diag, const double *A_off,
                              const double *B, double *X, int64_t nrhs, int64_t *ticket);

/* Admit queued requests, then enqueue one tick (the next step of every
 * request in flight on the lane) on each lane with fewer than three ticks in
 * flight; if no lane can take one, first wait for the oldest tick in flight.
 * Returns the number of requests queued or in flight (>= 0) or an error
 * code. */
BTC_API int btc_server_step(btc_server s);

/* Hand out up to `max` completions (wait != 0: first wait for all enqueued work). */
BTC_API int btc_server_poll(btc_server s, btc_server_completion *out, int32_t max, int32_t *count, int wait);

BTC_API int btc_server_stats(btc_server s, int64_t *queued, int64_t *in_flight, size_t *resident_bytes);

/* The resident handle of a client (NULL if not resident); owned by the server. */
BTC_API btc_handle btc_server_client_handle(btc_server s, int64_t client);

/* The runner the server enqueues the steps of its first lane on (owned by
 * the server; for btc_runner_profile / btc_runner_profile_read). */
BTC_API btc_runner btc_server_runner(btc_server s);

/* The runner of lane `lane` (0 .. lanes-1; lane 0 is btc_server_runner), or
   NULL for another index. */
BTC_API btc_runner btc_server_lane_runner(btc_server s, int32_t lane);

/* Host seconds btc_server_step spent blocked on the oldest tick in flight
 * (no lane could take another), and the ticks enqueued over all lanes, since
 * creation or the last reset (reset != 0 zeroes them after reading). */
BTC_API int btc_server_host_stats(btc_server s, double *wait_s, int64_t *ticks, int reset);

BTC_API void btc_server_destroy(btc_server s);

/*
 * btc_set_allocator -- source of every DEVICE allocation the library makes
 * from now on (factors, solve workspaces, runner and graph descriptor
 * buffers; pinned host staging memory is not affected): alloc(bytes, stream,
 * ctx) returns memory of the current device usable in stream order on
 * `stream` (NULL on failure, reported as BTC_ERR_OOM), free_(ptr, stream,
 * ctx) releases it in that order.  Both NULL restores HIP's allocator
 * (hipMalloc; hipMallocAsync for the memory of one call).  Objects keep the
 * functions they allocated with, so the hook may change while they live; the
 * functions must stay callable until those objects are destroyed.  Intended
 * for a framework's caching allocator (the Python binding installs torch's).
 * Returns -1 when exactly one of the two functions is NULL.
 */
BTC_API int btc_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                              void (*free_)(void *ptr, void *stream, void *ctx), void *ctx);

/*
 * btc_autotune_strategy -- time the elimination orders (multi-stage; k-stage
 * with k = 0, 1, 2 and partition with p = 2, 4 where they apply: FP64,
 * n <= 64, k < floor(log2 N)+1, chunks of at least one block) on the
 * caller's matrix: reps repetitions of refactor + solve each after one
 * warm-up, HIP events on `stream`; the fastest becomes the choice of
 * BTC_STRATEGY_AUTO for (precision, N, padded n), process-wide.  ms (host,
 * 6 entries, nullable) receives the milliseconds per refactor + solve of
 * multi-stage, k = 0, 1, 2, p = 2, 4 (-1: not a candidate).  Overwrites X.
 * Returns 0, -k for argument k, or the error of a candidate.
 */
BTC_API int btc_autotune_strategy(int64_t N, int64_t n, int32_t precision, const double *A_diag,
                                  const double *A_off, const double *B, double *X, int64_t nrhs, int32_t reps,
                                  void *stream, double *ms);

/* btc_select_strategy -- the elimination order BTC_STRATEGY_AUTO takes for
 * (N, n, precision): *strategy (BTC_STRATEGY_MULTISTAGE, _KSTAGE or
 * _PARTITION) and *stages.  Host only. */
BTC_API int btc_select_strategy(int64_t N, int64_t n, int32_t precision, int32_t *strategy, int32_t *stages);

/* ------------------------------------------------------------------------
 * Block-banded and arrow extensions.  The paper names both structures as
 * extensions of the method without giving an algorithm for either (arrow
 * structures: section "Multi-Stage Permutation", after the remark that the
 * permutation also arises in block cyclic reduction; block-banded matrices of
 * a larger bandwidth: section "Conclusion").  FP64 inputs, all precisions
 * (the mixed modes refine every solve of the block-tridiagonal part to the
 * handle's target).
 * ------------------------------------------------------------------------ */
typedef struct btc_banded_s *btc_banded; /* opaque; owned by the library */
typedef struct btc_arrow_s *btc_arrow;   /* opaque; owned by the library */

/*
 * btc_banded_create -- factor a symmetric positive definite block-banded
 * matrix: N block rows of order n, block bandwidth b >= 1 (block (i, j) is
 * zero for |i - j| > b).  b consecutive block rows and columns are grouped
 * into one super-block of order b*n, which makes the matrix block tridiagonal
 * with ceil(N/b) super-blocks; that matrix is factored by the multi-stage
 * method (btc_factor with opt).  A missing part of the last super-block is
 * completed with identity rows and columns, decoupled from the band.
 *   A_band  device, FP64, shape (N, b+1, n, n) row-major: A_band[i][k] is the
 *           block at (i, i-k) (0-based); k = 0 the diagonal block, only its
 *           lower triangle read; blocks with i - k < 0 are not read.  Read
 *           during the call only: the super-blocks are packed into memory the
 *           object owns (from the allocator of btc_set_allocator).
 *   b*n <= BTC_MAX_BLOCK, else BTC_ERR_UNSUPPORTED.
 * Argument errors: -1..-7 for the argument at that position.  A breakdown is
 * reported by btc_banded_status.
 */
BTC_API int btc_banded_create(const btc_options *opt, int64_t N, int64_t n, int64_t b, const double *A_band,
                              void *stream, btc_banded *out);

/* btc_banded_refactor -- pack and factor a new band of the same (N, n, b). */
BTC_API int btc_banded_refactor(btc_banded h, const double *A_band, void *stream);

/*
 * btc_banded_solve -- X = A^{-1} B; B and X device FP64, (N*n) x nrhs
 * row-major, as btc_solve (refinement and info likewise).  When b does not
 * divide N the solve runs on zero-padded copies taken from the allocator for
 * the duration of the call.
 */
BTC_API int btc_banded_solve(btc_banded h, const double *B, double *X, int64_t nrhs, void *stream,
                             btc_solve_info *info);

/* btc_banded_status -- as btc_status; *info is a 1-based super-block index. */
BTC_API int btc_banded_status(btc_banded h, int64_t *info);

/* btc_banded_inner -- the block-tridiagonal handle of the super-blocks (for
 * btc_export_factor); owned by the banded object. */
BTC_API btc_handle btc_banded_inner(btc_banded h);

/* btc_banded_destroy -- wait for its work, free everything (NULL is a no-op). */
BTC_API void btc_banded_destroy(btc_banded h);

/*
 * btc_arrow_create -- factor the arrow matrix
 *       A = [[Psi, F], [F^T, C]]
 * with Psi the block-tridiagonal matrix of (A_diag, A_off, N, n) as in
 * btc_factor, F its dense border ((N*n) x m, row-major: row r of F holds the
 * m couplings of row r of Psi with the tip) and C the m x m tip (symmetric,
 * lower triangle read), 0 <= m <= 128.  Psi is eliminated first by the
 * multi-stage method (opt as in btc_factor), then the tip:
 *   Z = Psi^{-1} F,  S = C - F^T Z (Schur complement),  S = L_S L_S^T,
 * so that the Cholesky factor of A in this order is [[L, 0], [F^T L^{-T},
 * L_S]] with L the factor of Psi.  F is copied into memory the object owns;
 * A_diag / A_off follow btc_factor's rules (kept for the residual in the
 * mixed-precision modes); C is read during the call only.
 * Argument errors: -1..-10 for the argument at that position; m > 128 or
 * n > BTC_MAX_BLOCK: BTC_ERR_UNSUPPORTED.  Breakdowns: btc_arrow_status.
 */
BTC_API int btc_arrow_create(const btc_options *opt, int64_t N, int64_t n, int64_t m, const double *A_diag,
                             const double *A_off, const double *F, const double *C, void *stream,
                             btc_arrow *out);

/* btc_arrow_refactor -- factor a new arrow of the same (N, n, m). */
BTC_API int btc_arrow_refactor(btc_arrow h, const double *A_diag, const double *A_off, const double *F,
                               const double *C, void *stream);

/*
 * btc_arrow_solve -- X = A^{-1} B; B and X device FP64, (N*n + m) x nrhs
 * row-major (the rows of Psi first, then the m rows of the tip):
 *   y = Psi^{-1} b1 (btc_solve, into the first N*n rows of X; `info` is that
 *   solve's), x2 = L_S^{-T} L_S^{-1} (b2 - F^T y), x1 = y - Z x2.
 * Takes its partial products' workspace from the allocator for the call.
 */
BTC_API int btc_arrow_solve(btc_arrow h, const double *B, double *X, int64_t nrhs, void *stream,
                            btc_solve_info *info);

/* btc_arrow_status -- synchronise; *info_psi as btc_status for Psi, *info_tip
 * 0 or the 1-based column of the first non-positive pivot of S (meaningful
 * only when *info_psi is 0). */
BTC_API int btc_arrow_status(btc_arrow h, int64_t *info_psi, int64_t *info_tip);

/* btc_arrow_export -- synchronise and copy L_S (m x m, row-major, upper part
 * 0) and Z ((N*n) x m) to host memory (either pointer may be NULL). */
BTC_API int btc_arrow_export(btc_arrow h, double *Ls, double *Z);

/* btc_arrow_inner -- the handle of Psi (owned by the arrow object). */
BTC_API btc_handle btc_arrow_inner(btc_arrow h);

/* btc_arrow_destroy -- wait for its work, free everything (NULL is a no-op). */
BTC_API void btc_arrow_destroy(btc_arrow h);

/* btc_error_string -- static text for a return code. */
BTC_API const char *btc_error_string(int code);

/* btc_version -- library ABI version (major*10000 + minor*100 + patch). */
BTC_API int btc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BTC_H */
