// Internal host-side definitions of libbtc shared by the C-ABI entry points
// (btc_api.hip) and the step runner (btc_runner.hip): the handle, its device
// memory and workspace layout, and the descriptors its kernels take.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "btc.h"
#include "btc_device.h"
#include "btc_kernels.h"

namespace btc_host {

constexpr unsigned long long kInfoOk = ~0ull;

__global__ void k_set_u64(unsigned long long* p, unsigned long long v);

// Device memory source (btc_set_allocator): the caller's functions, or HIP's
// own allocator when none is set.  Every object that allocates keeps the
// source it allocated from, so that a later change of the hook does not
// mismatch allocations and frees.
struct Allocator {
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*free_)(void*, void*, void*) = nullptr;
    void* ctx = nullptr;
};

Allocator current_allocator();

// Long-lived memory (factors, handle workspaces, descriptor buffers).
inline hipError_t dev_alloc(const Allocator& a, void** p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    if (a.alloc) {
        *p = a.alloc(bytes, (void*)st, a.ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

inline void dev_free(const Allocator& a, void* p, hipStream_t st) {
    if (!p) return;
    if (a.free_)
        a.free_(p, (void*)st, a.ctx);
    else
        (void)hipFree(p);
}

// Memory of one call, ordered on its stream: freed on the stream once the
// call's work is enqueued (HIP's stream-ordered allocator when no hook is
// set; a hook receives the stream and must order the reuse itself, as a
// caching allocator bound to that stream does).
inline hipError_t dev_alloc_async(const Allocator& a, void** p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    if (a.alloc) {
        *p = a.alloc(bytes, (void*)st, a.ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMallocAsync(p, bytes, st);
}

inline void dev_free_async(const Allocator& a, void* p, hipStream_t st) {
    if (!p) return;
    if (a.free_)
        a.free_(p, (void*)st, a.ctx);
    else
        (void)hipFreeAsync(p, st);
}

}  // namespace btc_host

struct btc_handle_s {
    int64_t N = 0;
    int64_t n = 0;
    int32_t precision = BTC_FP64;
    int32_t max_refine = 0;
    double tol = 0.0;
    int32_t refine = BTC_REFINE_CLASSIC;
    int32_t gmres_m = BTC_DEFAULT_GMRES_M;
    // elimination order: the first nd_levels levels of the multi-stage order
    // (all of them for BTC_STRATEGY_MULTISTAGE), then, for
    // BTC_STRATEGY_KSTAGE, the remaining chain one block after the other
    int32_t strategy = BTC_STRATEGY_MULTISTAGE;
    int32_t nd_levels = 0;
    // BTC_STRATEGY_PARTITION: p chunks, N_1 blocks in the first, N_k in the others
    int32_t parts = 0;
    int64_t part_n1 = 0, part_nk = 0;
    int levels = 0;  // floor(log2 N) + 1
    int device = 0;
    // FP64 factor (BTC_FP64)
    double* Ld = nullptr;
    double* Rb = nullptr;
    double* Tb = nullptr;
    // mixed factor (BTC_FP32_IR): FP64 Schur complements, FP32 factor
    double* S64 = nullptr;
    float* L32 = nullptr;
    float* R32 = nullptr;
    float* T32 = nullptr;
    unsigned long long* info = nullptr;
    // solve workspace, grown on demand (one allocation); ws_ev marks the end
    // of the last btc_solve that used it on ws_stream (a solve on another
    // stream before that point takes a workspace of its own)
    void* ws = nullptr;
    int64_t ws_m = 0;
    hipStream_t ws_stream = nullptr;
    hipEvent_t ws_ev = nullptr;
    bool ws_ev_valid = false;
    btc_host::Allocator alloc;     // source of every device allocation of the handle
    hipStream_t stream = nullptr;  // stream of the last call
    std::vector<hipStream_t> streams;  // every stream a solve of the handle ran on
    // factor kernel family of every level, fixed when level 0 of a
    // factorization is enqueued (the tune table may change meanwhile)
    int8_t fkind[64] = {};
    bool factored = false;
    bool failed_known = false;     // a status check saw a breakdown
    const double* A_diag = nullptr;
    const double* A_off = nullptr;
    // optional per-launch timing
    struct Timed {
        hipEvent_t a, b;
        int phase, level;
    };
    bool prof = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[4][64] = {};
    int64_t prof_n[4][64] = {};
};

namespace btc_host {

// A step runner whose groups spread over its stream and `sides` side streams
// (btc_runner_create takes the most).
int runner_create(void* stream, int sides, btc_runner* out);

inline bool is_mixed(int32_t p) { return p == BTC_FP32_IR || p == BTC_BF16_IR; }
inline bool is_bf16(int32_t p) { return p == BTC_BF16_IR; }

inline int num_levels(int64_t N) {
    int L = 0;
    while ((((int64_t)1) << (L + 1)) <= N) ++L;
    return L + 1;
}

inline int64_t level_nodes(int64_t N, int l) {
    const int64_t s = (int64_t)1 << l;
    return (N + s) / (2 * s);
}

inline int to_code(hipError_t e) {
    if (e == hipSuccess) return BTC_OK;
    if (e == hipErrorOutOfMemory) return BTC_ERR_OOM;
    return BTC_ERR_HIP;
}

template <class P>
inline void dfree(btc_handle h, P*& p) {
    dev_free(h->alloc, (void*)p, h->stream);
    p = nullptr;
}

inline void free_all(btc_handle h) {
    if (!h) return;
    if (h->ws_ev) (void)hipEventDestroy(h->ws_ev);
    h->ws_ev = nullptr;
    for (auto& t : h->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    h->pending.clear();
    for (auto e : h->pool) (void)hipEventDestroy(e);
    h->pool.clear();
    dfree(h, h->Ld);
    dfree(h, h->Rb);
    dfree(h, h->Tb);
    dfree(h, h->S64);
    dfree(h, h->L32);
    dfree(h, h->R32);
    dfree(h, h->T32);
    dfree(h, h->info);
    dfree(h, h->ws);
}

inline hipEvent_t take_event(btc_handle h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrapper: brackets the launch with events when profiling is on.
// Phases: 0 factor, 1 forward sweep, 2 backward sweep, 3 residual/refinement.
template <class F>
inline hipError_t timed(btc_handle h, int phase, int level, hipStream_t st, F&& launch) {
    if (!h->prof) return launch();
    hipEvent_t a = take_event(h), b = take_event(h);
    if (!a || !b) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, st);
    hipError_t e = launch();
    (void)hipEventRecord(b, st);
    h->pending.push_back({a, b, phase, level});
    return e;
}

inline void drain_profile(btc_handle h) {
    for (auto& t : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess && t.level < 64) {
            h->prof_ms[t.phase][t.level] += ms;
            h->prof_n[t.phase][t.level] += 1;
        }
        h->pool.push_back(t.a);
        h->pool.push_back(t.b);
    }
    h->pending.clear();
}

inline size_t factor_bytes(int64_t N, int64_t n, int32_t prec) {
    const size_t nn = (size_t)N * (size_t)n * (size_t)n;
    if (is_mixed(prec)) return nn * (sizeof(double) + 3 * sizeof(float));
    return 3 * nn * sizeof(double);
}

// Solve workspace: FP64 path: Y, U, V (FP64); mixed: r, y, u, v, d (FP32);
// both: partial norms (FP64, N x m x 2), the residual's two FP64 scratch
// vectors and the refinement state.
inline size_t workspace_bytes(int64_t N, int64_t n, int32_t prec, int64_t m) {
    const size_t v = (size_t)N * (size_t)n * (size_t)m;
    const size_t tail = 2 * (size_t)N * (size_t)m * sizeof(double) + 2 * v * sizeof(double) + 4 * 256;
    if (is_mixed(prec)) return 5 * v * sizeof(float) + tail;
    return 3 * v * sizeof(double) + tail;
}

struct Workspace {
    double *Y = nullptr, *U = nullptr, *V = nullptr;                              // FP64 path
    float *r = nullptr, *y = nullptr, *u = nullptr, *v = nullptr, *d = nullptr;  // mixed
    double* part = nullptr;
    double *rp = nullptr, *rq = nullptr;  // residual scratch
    btc::IrState* ir = nullptr;
};

// Workspace layout of an (N, n, precision) system with m right-hand sides in
// the memory at `base` (workspace_bytes long, 256-byte aligned).
inline Workspace carve_at(void* base, int64_t N, int64_t n, int32_t prec, int64_t m) {
    Workspace w;
    const size_t v = (size_t)N * (size_t)n * (size_t)m;
    char* p = (char*)base;
    auto align = [](char* q) { return (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255); };
    if (is_mixed(prec)) {
        w.r = (float*)p;
        p += v * sizeof(float);
        w.y = (float*)p;
        p += v * sizeof(float);
        w.u = (float*)p;
        p += v * sizeof(float);
        w.v = (float*)p;
        p += v * sizeof(float);
        w.d = (float*)p;
        p += v * sizeof(float);
    } else {
        w.Y = (double*)p;
        p += v * sizeof(double);
        w.U = (double*)p;
        p += v * sizeof(double);
        w.V = (double*)p;
        p += v * sizeof(double);
    }
    p = align(p);
    w.part = (double*)p;
    p += 2 * (size_t)N * (size_t)m * sizeof(double);
    p = align(p);
    w.rp = (double*)p;
    p += v * sizeof(double);
    w.rq = (double*)p;
    p += v * sizeof(double);
    p = align(p);
    w.ir = (btc::IrState*)p;
    return w;
}

inline Workspace carve(btc_handle h, int64_t m) { return carve_at(h->ws, h->N, h->n, h->precision, m); }

inline int ensure_workspace(btc_handle h, int64_t m) {
    if (m <= h->ws_m && h->ws) return BTC_OK;
    if (h->ws) {
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        if (h->ws_stream && h->ws_stream != h->stream) (void)hipStreamSynchronize(h->ws_stream);
        dfree(h, h->ws);
    }
    h->ws_m = 0;
    h->ws_ev_valid = false;
    hipError_t e = dev_alloc(h->alloc, &h->ws, workspace_bytes(h->N, h->n, h->precision, m), h->stream);
    if (e != hipSuccess) {
        h->ws = nullptr;
        return to_code(e);
    }
    h->ws_m = m;
    return BTC_OK;
}

inline int32_t factor_flags(btc_handle h, int level);

inline btc::FactorDesc factor_desc(btc_handle h, const double* A_diag, const double* A_off, int level) {
    btc::FactorDesc d{};
    d.flags = factor_flags(h, level);
    d.A_diag = A_diag;
    d.A_off = A_off;
    if (is_mixed(h->precision)) {
        d.Ld = h->S64;
        d.L32 = h->L32;
        d.R32 = h->R32;
        d.T32 = h->T32;
    } else {
        d.Ld = h->Ld;
        d.Rb = h->Rb;
        d.Tb = h->Tb;
    }
    d.info = h->info;
    d.N = h->N;
    d.n = (int32_t)h->n;
    return d;
}

// Padded block size of the factor kernel of a handle.
inline int factor_np(btc_handle h) {
    return is_mixed(h->precision) ? btc::padded_block_mixed((int)h->n) : btc::padded_block((int)h->n);
}

// Autotuned kernel variants (process-wide table, default 0).
int tune_variant(int op, int kind, int np, int bucket);
void tune_set(int op, int kind, int np, int bucket, int variant);
void save_tune_cache();
// Elimination order for BTC_STRATEGY_AUTO: the measured fastest for
// (precision, N, padded n), else a rule.
void select_strategy(int64_t N, int64_t n, int32_t prec, int32_t* strategy, int32_t* stages);

// Chunk sizes of the partition order with p >= 2 chunks (Proposition 1):
// a chunk after the first costs (19/3 N_k - 1) n^3, the first (7/3 N_1 - 1)
// n^3, with N_1 = N - (p-1) - (p-1) N_k (p - 1 separating blocks).  The
// balance point (7N - 7p + 7) / (7p + 12) is rounded down and up, and the
// rounding whose larger phase cost is smaller kept (ties: down).  False when
// no chunk sizes of at least one block exist.
inline bool partition_sizes(int64_t N, int64_t p, int64_t& n1, int64_t& nk) {
    if (p < 2) return false;
    const double star = (7.0 * (double)N - 7.0 * (double)p + 7.0) / (7.0 * (double)p + 12.0);
    bool found = false;
    double best = 0.0;
    for (int64_t c = (int64_t)std::floor(star); c <= (int64_t)std::ceil(star); ++c) {
        if (c < 1) continue;
        const int64_t first = N - (p - 1) - (p - 1) * c;
        if (first < 1) continue;
        const double cost = std::max(7.0 / 3.0 * (double)first - 1.0, 19.0 / 3.0 * (double)c - 1.0);
        if (!found || cost < best) {
            found = true;
            best = cost;
            n1 = first;
            nk = c;
        }
    }
    return found;
}
void strategy_set(int64_t N, int64_t n, int32_t prec, int32_t strategy, int32_t stages);

// Factor kernel family of a handle at a level: 0 VALU FP64 (np < 16, or
// np 16/32 where the autotuner chose it), 1 MFMA FP64, 2 mixed,
// 3 tile-parallel FP64 (np > 64, or np 32/64 where the autotuner chose it),
// 4 tile-parallel mixed, 5 mixed with BF16 products, 6 tile-parallel mixed
// with BF16 products.  Variants of the tune table: np 64 and mixed np 32,
// 1 tile-parallel; FP64 np 16/32, 1 VALU; FP64 np 32, 2 tile-parallel.
inline int tuned_factor_kind(btc_handle h, int level) {
    const int np = factor_np(h);
    const bool mixed = is_mixed(h->precision);
    const int tiled = mixed ? (is_bf16(h->precision) ? 6 : 4) : 3;
    if (np > 64) return tiled;
    const int bucket = level > 0 ? 1 : 0;
    const int v = tune_variant(BTC_OP_FACTOR, mixed ? (is_bf16(h->precision) ? 2 : 1) : 0, np, bucket);
    if (np == 64 && v == 1) return tiled;
    if (mixed) return (np == 32 && v == 1) ? tiled : (is_bf16(h->precision) ? 5 : 2);
    if (np < 16) return 0;
    if (np == 32 && v == 2) return tiled;
    if (np <= 32 && v == 1) return 0;
    return 1;
}

// Fix the kernel family of every level from the tune table (when level 0 of
// a factorization is enqueued: all levels of one factorization then agree
// on the separator-update protocol).
inline void snapshot_factor_kinds(btc_handle h) {
    for (int l = 0; l < h->levels && l < 64; ++l) h->fkind[l] = (int8_t)tuned_factor_kind(h, l);
}

inline int factor_kind(btc_handle h, int level) { return h->fkind[level]; }

inline bool tiled_kind(int kind) { return kind == 3 || kind == 4 || kind == 6; }

// FactorDesc flags of a handle's level step: a level whose step and the
// next level's step are both tile-parallel applies the right neighbours'
// T^T T eagerly (its separators then receive both contributions in one
// pass), and the next level has no deferred updates.
inline int32_t factor_flags(btc_handle h, int level) {
    // the chain of a k-stage order applies the last level's deferred update
    auto eager = [h](int l) {
        return l >= 0 && l + 1 < h->nd_levels && tiled_kind(factor_kind(h, l)) && tiled_kind(factor_kind(h, l + 1));
    };
    return (eager(level) ? btc::kFactorEagerT : 0) | (eager(level - 1) ? btc::kFactorDeferredDone : 0);
}

// Right-hand-side columns per dependency-chain group of a sweep or residual
// launch (results do not depend on it).
inline int sweep_mc(int op, int kind, int np, int64_t m) {
    return (m <= 1 || tune_variant(op, kind, np, 0) == 1) ? 1 : 4;
}

// deferred: some item of the launch has deferred updates to apply (tile-
// parallel families: otherwise that kernel is not launched); part: tile-
// parallel families only, 0 the whole step or one of its kernels.
inline hipError_t launch_factor_kind(int kind, const btc::Launch<btc::FactorDesc>& L, int np, bool deferred,
                                     int64_t items, hipStream_t st, int part = 0) {
    switch (kind) {
        case 0: return btc::launch_factor_valu(L, np, items, st);
        case 1: return btc::launch_factor_mfma(L, np, items, st);
        case 2: return btc::launch_factor_mixed(L, np, false, items, st);
        case 3: return btc::launch_factor_tiled(L, np, 0, part, deferred, items, st);
        case 4: return btc::launch_factor_tiled(L, np, 1, part, deferred, items, st);
        case 5: return btc::launch_factor_mixed(L, np, true, items, st);
        case 6: return btc::launch_factor_tiled(L, np, 2, part, deferred, items, st);
        default: return hipErrorInvalidValue;
    }
}

inline hipError_t launch_factor_any(btc_handle h, const btc::Launch<btc::FactorDesc>& L, int64_t items, hipStream_t st) {
    const int np = factor_np(h);
    const bool deferred = L.level > 0 && !(L.single.flags & btc::kFactorDeferredDone);
    return launch_factor_kind(factor_kind(h, L.level), L, np, deferred, items, st);
}

inline btc::ChainDesc chain_desc(btc_handle h, const double* A_diag, const double* A_off, const double* B, double* X,
                                 int64_t m) {
    btc::ChainDesc c{};
    c.A_diag = A_diag;
    c.A_off = A_off;
    c.Ld = h->Ld;
    c.Rb = h->Rb;
    c.Tb = h->Tb;
    c.info = h->info;
    c.B = B;
    c.X = X;
    c.N = h->N;
    c.n = (int32_t)h->n;
    c.k = h->nd_levels;
    c.m = (int32_t)m;
    c.parts = h->strategy == BTC_STRATEGY_PARTITION ? h->parts : 0;
    c.n1 = h->part_n1;
    c.nk = h->part_nk;
    return c;
}

inline int launch_factor(btc_handle h, const double* A_diag, const double* A_off, hipStream_t st) {
    snapshot_factor_kinds(h);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, h->info, kInfoOk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return to_code(e);
    btc::Launch<btc::FactorDesc> L{};
    for (int l = 0; l < h->nd_levels; ++l) {
        L.single = factor_desc(h, A_diag, A_off, l);
        L.level = l;
        const int64_t nodes = level_nodes(h->N, l);
        e = timed(h, 0, l, st, [&] { return launch_factor_any(h, L, nodes, st); });
        if (e != hipSuccess) return to_code(e);
    }
    if (h->strategy == BTC_STRATEGY_KSTAGE) {
        const btc::ChainDesc c = chain_desc(h, A_diag, A_off, nullptr, nullptr, 0);
        e = timed(h, 0, h->nd_levels, st, [&] { return btc::launch_chain_factor(c, btc::padded_block((int)h->n), st); });
        if (e != hipSuccess) return to_code(e);
    } else if (h->strategy == BTC_STRATEGY_PARTITION) {
        const btc::ChainDesc c = chain_desc(h, A_diag, A_off, nullptr, nullptr, 0);
        e = timed(h, 0, 0, st, [&] { return btc::launch_part_factor(c, btc::padded_block((int)h->n), st); });
        if (e != hipSuccess) return to_code(e);
    }
    h->A_diag = A_diag;
    h->A_off = A_off;
    h->stream = st;
    h->factored = true;
    h->failed_known = false;
    return BTC_OK;
}

// Level ranges of a sweep, one launch each: a range of one level runs one
// wavefront per node (levels with many nodes: the most parallel form), a
// range of several levels one workgroup per subtree (launch_sweep's chunk
// form), which saves a launch and a dependency step per level.  A node step
// is latency bound (one wavefront streams its blocks slab by slab: about
// 15 us FP32, 45 us FP64 at n = 96), so a range takes only levels whose
// subtree nodes the workgroup's wavefronts cover in one round each: its time
// is then one node step per level, as with one launch per level.  Greedy
// from level 0: a level with at least kSweepNodesPerLevel nodes is a range
// of its own; otherwise the range grows while every level of a subtree has
// at most kChunkWaves nodes.
constexpr int64_t kSweepNodesPerLevel = 4096;

inline int64_t chunk_rounds(int64_t N, int l0, int l1, int kw) {
    int64_t r = 0;
    for (int l = l0; l < l1; ++l) {
        const int64_t per = (int64_t)1 << (l1 - l - 1);
        const int64_t nodes = level_nodes(N, l);
        const int64_t c = per < nodes ? per : nodes;
        r += (c + kw - 1) / kw;
    }
    return r;
}

// Sweep launch shapes (tune key BTC_TUNE_SWEEP_SHAPE): 0 level ranges with
// 4-wavefront workgroups, 1 one launch per level, 2 level ranges with
// 8-wavefront workgroups.
inline int sweep_shape(int32_t prec, int64_t n) {
    return tune_variant(BTC_TUNE_SWEEP_SHAPE, is_mixed(prec) ? 1 : 0, btc::padded_block((int)n), 0);
}
inline int shape_waves(int shape) { return shape == 2 ? 8 : 4; }

// Subtrees of the range [l0, l1): those j with a level-l0 node in (j 2^l1, (j+1) 2^l1).
inline int64_t chunk_count(int64_t N, int l0, int l1) {
    return ((N - ((int64_t)1 << l0)) >> l1) + 1;
}

// bounds[0] = 0 < bounds[1] < ... < bounds[r] = levels; returns r.
inline int sweep_ranges(int64_t N, int levels, int* bounds, int shape = 0) {
    int r = 0, l0 = 0;
    bounds[0] = 0;
    const int kw = shape_waves(shape);
    while (l0 < levels) {
        int l1 = l0 + 1;
        if (shape != 1 && level_nodes(N, l0) < kSweepNodesPerLevel)
            while (l1 < levels && chunk_rounds(N, l0, l1 + 1, kw) <= l1 + 1 - l0) ++l1;
        bounds[++r] = l1;
        l0 = l1;
    }
    return r;
}

// One range of a sweep (forward or backward) of one instance.
template <class T>
inline hipError_t sweep_range(btc_handle h, btc::Launch<btc::SweepDesc<T>>& L, int l0, int l1, bool bwd,
                              hipStream_t st) {
    const int np = btc::padded_block((int)h->n);
    const int op = bwd ? BTC_OP_BACKWARD : BTC_OP_FORWARD;
    const int mc = sweep_mc(op, sizeof(T) == 4, np, L.single.m);
    const bool chunk = l1 > l0 + 1;
    L.level = chunk ? (l0 | (l1 << 8)) : l0;
    const int64_t items = chunk ? chunk_count(h->N, l0, l1) : level_nodes(h->N, l0);
    const int kw = shape_waves(sweep_shape(h->precision, h->n));
    // profiled per range, attributed to its first level
    return timed(h, bwd ? 2 : 1, l0, st, [&] { return btc::launch_sweep(L, np, items, bwd, mc, st, chunk, kw); });
}

template <class T>
inline hipError_t chain_solve(btc_handle, const btc::SweepDesc<T>&, hipStream_t) {
    return hipErrorInvalidValue;  // the k-stage orders are FP64 only
}

template <>
inline hipError_t chain_solve<double>(btc_handle h, const btc::SweepDesc<double>& d, hipStream_t st) {
    btc::ChainDesc c = chain_desc(h, nullptr, nullptr, d.B, d.X, d.m);
    c.Y = d.Y;
    c.U = d.U;
    c.V = d.V;
    if (h->strategy == BTC_STRATEGY_PARTITION)
        return timed(h, 1, 0, st, [&] { return btc::launch_part_solve(c, btc::padded_block((int)h->n), st); });
    return timed(h, 1, h->nd_levels, st, [&] { return btc::launch_chain_solve(c, btc::padded_block((int)h->n), st); });
}

template <class T>
inline hipError_t sweeps(btc_handle h, const btc::SweepDesc<T>& d, hipStream_t st) {
    btc::Launch<btc::SweepDesc<T>> L{};
    L.single = d;
    int b[66];
    // the levels of the multi-stage order (all of them, or the first k), in
    // ranges; a k-stage order solves along its chain in between
    const int r = sweep_ranges(h->N, h->nd_levels, b, sweep_shape(h->precision, h->n));
    for (int k = 0; k < r; ++k) {
        hipError_t e = sweep_range(h, L, b[k], b[k + 1], false, st);
        if (e != hipSuccess) return e;
    }
    if (h->strategy == BTC_STRATEGY_KSTAGE || h->strategy == BTC_STRATEGY_PARTITION) {
        hipError_t e = chain_solve(h, d, st);
        if (e != hipSuccess) return e;
    }
    for (int k = r - 1; k >= 0; --k) {
        hipError_t e = sweep_range(h, L, b[k], b[k + 1], true, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

inline btc::SweepDesc<double> sweep_desc64(btc_handle h, const Workspace& w, const double* B, double* X, int64_t m) {
    btc::SweepDesc<double> p{};
    p.Ld = h->Ld;
    p.Rb = h->Rb;
    p.Tb = h->Tb;
    p.B = B;
    p.X = X;
    p.Y = w.Y;
    p.U = w.U;
    p.V = w.V;
    p.info = h->info;
    p.N = h->N;
    p.n = (int32_t)h->n;
    p.m = (int32_t)m;
    return p;
}

inline btc::SweepDesc<float> sweep_desc32(btc_handle h, const Workspace& w, const double* B, double* X, int64_t m,
                                   bool first) {
    btc::SweepDesc<float> p{};
    p.Ld = h->L32;
    p.Rb = h->R32;
    p.Tb = h->T32;
    p.B = w.r;
    p.B64 = first ? B : nullptr;
    p.X = w.d;
    p.Y = w.y;
    p.U = w.u;
    p.V = w.v;
    p.X64 = X;
    p.info = h->info;
    p.skip = &w.ir->done;
    p.N = h->N;
    p.n = (int32_t)h->n;
    p.m = (int32_t)m;
    p.first = first ? 1 : 0;
    return p;
}

inline btc::ResidualDesc residual_desc(btc_handle h, const Workspace& w, const double* B, const double* X, int64_t m,
                                bool to_fp32) {
    btc::ResidualDesc r{};
    r.A_diag = h->A_diag;
    r.A_off = h->A_off;
    r.B = B;
    r.X = X;
    r.R32 = to_fp32 ? w.r : nullptr;
    r.part = w.part;
    r.P = w.rp;
    r.Q = w.rq;
    r.state = w.ir;
    r.N = h->N;
    r.n = (int32_t)h->n;
    r.m = (int32_t)m;
    return r;
}

inline btc::IrDesc ir_desc(btc_handle h, const Workspace& w, int64_t m, double tol, int max_steps) {
    btc::IrDesc d{};
    d.state = w.ir;
    d.part = w.part;
    d.N = h->N;
    d.n = (int32_t)h->n;
    d.m = (int32_t)m;
    d.tol = tol;
    d.max_steps = max_steps;
    return d;
}

// Solve entry points (btc_api.hip): the enqueue of one solve with a given
// workspace, the shared argument checks (0: go on, 1: nothing to do, < 0:
// error), and the record of a stream a handle was used on.
int solve_with(btc_handle h, const Workspace& w, const double* B, double* X, int64_t nrhs, hipStream_t st,
               btc_solve_info* info);
int check_solve(btc_handle h, const double* B, double* X, int64_t nrhs);
void note_stream(btc_handle h, hipStream_t st);

inline int read_info(btc_handle h, hipStream_t st, unsigned long long* v) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return to_code(e);
    e = hipMemcpy(v, h->info, sizeof(*v), hipMemcpyDeviceToHost);
    return to_code(e);
}


}  // namespace btc_host
