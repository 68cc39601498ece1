// Step runner: executes a list of level steps of many handles with one
// kernel launch per (operation, kernel, padded block size) group.  Each step
// contributes its work items (the nodes of one level, the block rows of a
// residual, or one refinement test) and its descriptor; descriptors and items
// of a call are packed into one upload from a pinned staging buffer
// (double-buffered, so the host can prepare the next call while the device
// runs the current one).  Batched factorization and solve of many
// independent instances, and the continuous-batching server, are built on it.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "btc.h"
#include "btc_handle.h"
#include "btc_kernels.h"
#include "btc_work.h"

using namespace btc_host;

namespace {

__global__ void k_reset_infos(unsigned long long* const* __restrict__ ptrs, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) *ptrs[t] = kInfoOk;
}

// One group = one launch.
struct Group {
    int stage = 0;
    int op;    // btc_op
    int kind;  // FACTOR: factor kernel family (factor_kind); sweeps: 0 double, 1 float,
               // 2 / 3 the same over level ranges (subtree launches)
    bool deferred = false;  // FACTOR: some item has deferred updates to apply
    int m_max = 1;   // sweeps / residual: largest number of right-hand sides
    int np;
    bool count = false;    // work accounted (profiler on)
    bool prof = false;     // bracketed by timing events
    int lane = 0;          // 0: the runner's stream, k: side stream k-1
    Work work;             // algorithmic work of the launch (when profiled)
    Work part[4];          // tile-parallel factor: work of each of its kernels (1..3)
    std::vector<char> descs;  // packed descriptors (all of one type)
    size_t desc_size = 0;
    std::vector<btc::WorkItem> items;
    size_t off_desc = 0, off_items = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The groups of one runner call and the status words its level-0 factor
// steps reset; offsets are into the device buffer the call is launched from.
struct Call {
    std::map<std::tuple<int, int, int, int>, Group> groups;  // (stage, op, kind, np)
    std::vector<unsigned long long*> resets;
    size_t off_resets = 0;
};

}  // namespace

struct btc_runner_s {
    hipStream_t st = nullptr;
    btc_host::Allocator alloc;  // source of the descriptor buffers
    struct Slot {
        char* host = nullptr;
        size_t hcap = 0;
        char* dev = nullptr;
        size_t dcap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    } slot[2];
    int cur = 0;
    // Groups of one call are independent: they run concurrently on the main
    // stream and up to kSide side streams (fork after the upload, join before
    // the call returns, so later work on the main stream sees all of it).
    static constexpr int kSide = 3;
    int nside = kSide;  // side streams in use
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {};
    // launch profiler: op filter (-2 off, -1 every group), kind filter (-1 any)
    int prof_op = -2, prof_kind = -1;
    struct Pending {
        std::tuple<int, int, int, int> key;  // op, kind, np, part
        hipEvent_t a, b;
        Work work;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::tuple<int, int, int, int>, btc_kernel_stat> totals;
    // graph recording (btc_graph_begin .. btc_graph_end)
    bool recording = false;
    std::vector<Call> rec;
    std::vector<btc_handle> rec_handles;
    // host time of btc_runner_run (seconds) and the part of it spent waiting
    // for the device to release a staging slot
    double host_run_s = 0.0, host_wait_s = 0.0;
    int64_t host_calls = 0;
};

struct btc_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char* dev = nullptr;
    btc_host::Allocator alloc;
    hipStream_t cap = nullptr;
};

namespace {

bool prof_match(const btc_runner_s* r, int op, int kind) {
    if (r->prof_op == -2) return false;
    return (r->prof_op == -1 || r->prof_op == op) && (r->prof_kind == -1 || r->prof_kind == kind);
}

hipEvent_t take_event(btc_runner_s* r) {
    if (!r->pool.empty()) {
        hipEvent_t e = r->pool.back();
        r->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold finished timing pairs into the totals (all of them when wait).
void drain_prof(btc_runner_s* r, bool wait) {
    size_t done = 0;
    for (; done < r->pending.size(); ++done) {
        auto& p = r->pending[done];
        if (!wait && hipEventQuery(p.b) != hipSuccess) break;
        if (wait) (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        btc_kernel_stat& t = r->totals[p.key];
        t.op = std::get<0>(p.key);
        t.kind = std::get<1>(p.key);
        t.np = std::get<2>(p.key);
        t.part = std::get<3>(p.key);
        t.launches += 1;
        t.items += p.work.items;
        t.ms += ms;
        t.bytes += p.work.bytes;
        t.flops += p.work.flops;
        r->pool.push_back(p.a);
        r->pool.push_back(p.b);
    }
    r->pending.erase(r->pending.begin(), r->pending.begin() + done);
}

// Work of a launch that the profiler counts but does not time.
void add_untimed(btc_runner_s* r, const std::tuple<int, int, int, int>& key, const Work& w) {
    btc_kernel_stat& t = r->totals[key];
    t.op = std::get<0>(key);
    t.kind = std::get<1>(key);
    t.np = std::get<2>(key);
    t.part = std::get<3>(key);
    t.launches += 1;
    t.items += w.items;
    t.bytes += w.bytes;
    t.flops += w.flops;
}

}  // namespace

namespace {

int slot_reserve(btc_runner r, btc_runner_s::Slot& s, size_t bytes) {
    if (s.pending) {
        const auto t0 = std::chrono::steady_clock::now();
        const hipError_t e = hipEventSynchronize(s.ev);
        r->host_wait_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (e != hipSuccess) return BTC_ERR_HIP;
        s.pending = false;
    }
    if (bytes > s.hcap) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = nullptr;
        const size_t cap = std::max(bytes, (size_t)1 << 16) * 2;
        if (hipHostMalloc((void**)&s.host, cap, hipHostMallocDefault) != hipSuccess) {
            s.hcap = 0;
            return BTC_ERR_OOM;
        }
        s.hcap = cap;
    }
    if (bytes > s.dcap) {
        // the device buffer may still be read by launches of an earlier call
        if (hipStreamSynchronize(r->st) != hipSuccess) return BTC_ERR_HIP;
        dev_free(r->alloc, s.dev, r->st);
        s.dev = nullptr;
        const size_t cap = std::max(bytes, (size_t)1 << 16) * 2;
        if (dev_alloc(r->alloc, (void**)&s.dev, cap, r->st) != hipSuccess) {
            s.dcap = 0;
            return BTC_ERR_OOM;
        }
        s.dcap = cap;
    }
    return BTC_OK;
}

template <class D>
void push_desc(Group& g, const D& d) {
    g.desc_size = sizeof(D);
    const size_t o = g.descs.size();
    g.descs.resize(o + sizeof(D));
    memcpy(g.descs.data() + o, &d, sizeof(D));
}

template <class D>
btc::Launch<D> make_launch(const Group& g, char* dev) {
    btc::Launch<D> L{};
    L.descs = (const D*)(dev + g.off_desc);
    L.items = (const btc::WorkItem*)(dev + g.off_items);
    return L;
}

int validate(const btc_step& s) {
    btc_handle h = s.h;
    if (!h) return -3;
    if (h->strategy != BTC_STRATEGY_MULTISTAGE) return -3;  // level steps exist in the multi-stage order only
    if (s.op < BTC_OP_FACTOR || s.op > BTC_OP_REFINE_TEST) return -3;
    if (s.stage < 0 || s.stage > 7) return -3;
    if (s.op == BTC_OP_FACTOR || s.op == BTC_OP_FORWARD || s.op == BTC_OP_BACKWARD) {
        if (s.level < 0 || s.level >= h->levels) return -3;
    }
    if (s.level_end != 0) {
        if (s.op != BTC_OP_FORWARD && s.op != BTC_OP_BACKWARD) return -3;
        if (s.level_end <= s.level || s.level_end > h->levels) return -3;
    }
    if (s.op == BTC_OP_FACTOR) {
        if (s.level == 0 && (!s.A_diag || (h->N > 1 && !s.A_off))) return -3;
        if (s.level > 0 && !h->A_diag) return -3;
    } else {
        if (s.nrhs < 1) return -3;
        if (s.op != BTC_OP_REFINE_INIT && s.op != BTC_OP_REFINE_TEST && (!s.B || !s.X)) return -3;
        if (s.op == BTC_OP_RESIDUAL && !h->A_diag) return -3;
    }
    return BTC_OK;
}

}  // namespace

extern "C" {

namespace {

void add_work(const btc_runner_s* r, Group& g, const btc_step& s, bool mixed) {
    if (r->prof_op == -2) return;
    g.count = true;
    g.prof = prof_match(r, g.op, g.kind);
    const btc_handle h = s.h;
    const int l1 = s.level_end > s.level ? s.level_end : s.level + 1;
    for (int l = s.level; l < l1; ++l) {
        const Work w = level_work(s.op, mixed, h->N, h->n, s.op == BTC_OP_FACTOR ? 0 : s.nrhs, l);
        g.work.bytes += w.bytes;
        g.work.flops += w.flops;
        g.work.items += w.items;
    }
    if (s.op == BTC_OP_FACTOR && tiled_kind(g.kind))
        for (int k = 1; k <= 3; ++k) {
            const Work pw = tiled_part_work(k, mixed, h->N, h->n, s.level, factor_flags(h, s.level));
            g.part[k].bytes += pw.bytes;
            g.part[k].flops += pw.flops;
            g.part[k].items += pw.items;
        }
}

}  // namespace

BTC_API int btc_runner_create(void* stream, btc_runner* out) {
    return btc_host::runner_create(stream, btc_runner_s::kSide, out);
}

}  // extern "C"

int btc_host::runner_create(void* stream, int sides, btc_runner* out) {
    if (!out) return -2;
    if (sides < 0 || sides > btc_runner_s::kSide) return -3;
    *out = nullptr;
    btc_runner r = new (std::nothrow) btc_runner_s();
    if (!r) return BTC_ERR_OOM;
    r->st = (hipStream_t)stream;
    r->nside = sides;
    r->alloc = current_allocator();
    bool ok = true;
    for (auto& s : r->slot) ok = ok && hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&r->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < sides; ++k) {
        ok = ok && hipStreamCreateWithFlags(&r->side[k], hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&r->join[k], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        btc_runner_destroy(r);
        return BTC_ERR_HIP;
    }
    *out = r;
    return BTC_OK;
}

extern "C" {

BTC_API void btc_runner_destroy(btc_runner r) {
    if (!r) return;
    (void)hipStreamSynchronize(r->st);
    drain_prof(r, true);
    for (auto e : r->pool) (void)hipEventDestroy(e);
    for (int k = 0; k < btc_runner_s::kSide; ++k)
        if (r->side[k]) (void)hipStreamSynchronize(r->side[k]);
    for (auto& s : r->slot) {
        if (s.host) (void)hipHostFree(s.host);
        dev_free(r->alloc, s.dev, r->st);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    for (int k = 0; k < btc_runner_s::kSide; ++k) {
        if (r->side[k]) (void)hipStreamDestroy(r->side[k]);
        if (r->join[k]) (void)hipEventDestroy(r->join[k]);
    }
    if (r->fork) (void)hipEventDestroy(r->fork);
    delete r;
}

namespace {

// Validate the steps and grow the workspaces they need (growing one
// synchronises, so this runs before anything of the call is queued).
int prepare_steps(btc_runner r, int32_t count, const btc_step* steps, hipStream_t st) {
    for (int32_t k = 0; k < count; ++k) {
        const int rc = validate(steps[k]);
        if (rc != BTC_OK) return rc;
        btc_handle h = steps[k].h;
        if (steps[k].op != BTC_OP_FACTOR) {
            if (steps[k].nrhs > h->ws_m || !h->ws) {
                // a recorded call already points into this workspace
                if (r->recording && h->ws &&
                    std::find(r->rec_handles.begin(), r->rec_handles.end(), h) != r->rec_handles.end())
                    return BTC_ERR_UNSUPPORTED;
                if (h->ws) (void)hipStreamSynchronize(st);
                h->stream = st;
                const int e = ensure_workspace(h, steps[k].nrhs);
                if (e != BTC_OK) return e;
            }
            // the workspace is now in use on the runner's stream
            h->ws_stream = st;
            h->ws_ev_valid = false;
        }
    }

    if (r->recording)
        for (int32_t k = 0; k < count; ++k) r->rec_handles.push_back(steps[k].h);
    return BTC_OK;
}

// Group the steps of one call by (operation, kernel family, padded size).
void build_call(btc_runner r, int32_t count, const btc_step* steps, hipStream_t st, Call& c) {
    auto& groups = c.groups;
    auto& resets = c.resets;
    for (int32_t k = 0; k < count; ++k) {
        const btc_step& s = steps[k];
        btc_handle h = s.h;
        const bool mixed = is_mixed(h->precision);
        h->stream = st;
        if (s.op == BTC_OP_FACTOR) {
            if (s.level == 0) {
                snapshot_factor_kinds(h);
                resets.push_back(h->info);
                h->A_diag = s.A_diag;
                h->A_off = s.A_off;
                h->factored = true;
                h->failed_known = false;
            }
            const int np = factor_np(h);
            const int kind = factor_kind(h, s.level);
            Group& g = groups[std::make_tuple(s.stage, s.op, kind, np)];
            g.stage = s.stage;
            g.op = s.op;
            g.kind = kind;
            g.np = np;
            const btc::FactorDesc fd = factor_desc(h, h->A_diag, h->A_off, s.level);
            g.deferred = g.deferred || (s.level > 0 && !(fd.flags & btc::kFactorDeferredDone));
            const int32_t inst = (int32_t)(g.descs.size() / sizeof(btc::FactorDesc));
            push_desc(g, fd);
            add_work(r, g, s, mixed);
            const int64_t nodes = level_nodes(h->N, s.level);
            for (int64_t q = 0; q < nodes; ++q) g.items.push_back({inst, s.level, q});
            continue;
        }
        const Workspace w = carve(h, h->ws_m);
        const int np = btc::padded_block((int)h->n);
        if (s.op == BTC_OP_FORWARD || s.op == BTC_OP_BACKWARD) {
            const bool range = s.level_end > s.level + 1;
            const int kind = (mixed ? 1 : 0) + (range ? 2 : 0);
            Group& g = groups[std::make_tuple(s.stage, s.op, kind, np)];
            g.stage = s.stage;
            g.op = s.op;
            g.kind = kind;
            g.np = np;
            g.m_max = std::max<int>(g.m_max, (int)s.nrhs);
            int32_t inst;
            if (mixed) {
                inst = (int32_t)(g.descs.size() / sizeof(btc::SweepDesc<float>));
                push_desc(g, sweep_desc32(h, w, s.B, s.X, s.nrhs, s.first != 0));
            } else {
                inst = (int32_t)(g.descs.size() / sizeof(btc::SweepDesc<double>));
                push_desc(g, sweep_desc64(h, w, s.B, s.X, s.nrhs));
            }
            add_work(r, g, s, mixed);
            if (range) {
                const int64_t cnt = chunk_count(h->N, s.level, s.level_end);
                for (int64_t q = 0; q < cnt; ++q) g.items.push_back({inst, s.level | (s.level_end << 8), q});
            } else {
                const int64_t nodes = level_nodes(h->N, s.level);
                for (int64_t q = 0; q < nodes; ++q) g.items.push_back({inst, s.level, q});
            }
        } else if (s.op == BTC_OP_RESIDUAL) {
            Group& g = groups[std::make_tuple(s.stage, s.op, 0, np)];
            g.stage = s.stage;
            g.op = s.op;
            g.kind = 0;
            g.np = np;
            g.m_max = std::max<int>(g.m_max, (int)s.nrhs);
            const int32_t inst = (int32_t)(g.descs.size() / sizeof(btc::ResidualDesc));
            push_desc(g, residual_desc(h, w, s.B, s.X, s.nrhs, mixed));
            add_work(r, g, s, mixed);
            for (int64_t q = 0; q < h->N; ++q) g.items.push_back({inst, 0, q});
        } else {
            Group& g = groups[std::make_tuple(s.stage, s.op, 0, 0)];
            g.stage = s.stage;
            g.op = s.op;
            g.kind = 0;
            g.np = 0;
            const int32_t inst = (int32_t)(g.descs.size() / sizeof(btc::IrDesc));
            const double tol = mixed ? h->tol : 0.0;
            const int steps_budget = mixed ? 1 + h->max_refine : 1;
            push_desc(g, ir_desc(h, w, s.nrhs, tol, steps_budget));
            add_work(r, g, s, mixed);
            g.items.push_back({inst, 0, 0});
        }
    }

}

// Offsets of the call's reset list, descriptors and items from `base`;
// returns the end.
size_t layout_call(Call& c, size_t base) {
    c.off_resets = base;
    size_t bytes = align256(base + c.resets.size() * sizeof(unsigned long long*));
    for (auto& kv : c.groups) {
        Group& g = kv.second;
        g.off_desc = bytes;
        bytes = align256(bytes + g.descs.size());
        g.off_items = bytes;
        bytes = align256(bytes + g.items.size() * sizeof(btc::WorkItem));
    }
    return bytes;
}

void write_call(const Call& c, char* host) {
    if (!c.resets.empty()) memcpy(host + c.off_resets, c.resets.data(), c.resets.size() * sizeof(unsigned long long*));
    for (auto& kv : c.groups) {
        const Group& g = kv.second;
        memcpy(host + g.off_desc, g.descs.data(), g.descs.size());
        memcpy(host + g.off_items, g.items.data(), g.items.size() * sizeof(btc::WorkItem));
    }
}

// Enqueue the call (its descriptors already in `dev`): status resets, then
// the groups stage by stage, the independent groups of a stage spread over
// the runner's streams.
int launch_call(btc_runner r, Call& c, char* dev, hipStream_t st, bool timing) {
    hipError_t e = hipSuccess;
    auto& groups = c.groups;
    const auto& resets = c.resets;
    if (!resets.empty()) {
        const int n = (int)resets.size();
        hipLaunchKernelGGL(k_reset_infos, dim3((n + 255) / 256), dim3(256), 0, st,
                           (unsigned long long* const*)(dev + c.off_resets), n);
        e = hipGetLastError();
        if (e != hipSuccess) return to_code(e);
    }
    if (timing && !r->pending.empty()) drain_prof(r, false);
    auto launch_group = [&](const Group& g) -> int {
        const int64_t items = (int64_t)g.items.size();
        hipStream_t gs = g.lane == 0 ? st : r->side[g.lane - 1];
        hipEvent_t ea = nullptr, eb = nullptr;
        const bool split = g.prof && timing && g.op == BTC_OP_FACTOR && tiled_kind(g.kind);
        if (g.prof && timing && !split) {
            ea = take_event(r);
            eb = ea ? take_event(r) : nullptr;
            if (!eb) {
                if (ea) r->pool.push_back(ea);
                return BTC_ERR_HIP;
            }
            (void)hipEventRecord(ea, gs);
        }
        switch (g.op) {
            case BTC_OP_FACTOR: {
                auto L = make_launch<btc::FactorDesc>(g, dev);
                if (!split) {
                    e = launch_factor_kind(g.kind, L, g.np, g.deferred, items, gs);
                    break;
                }
                // one timing pair per kernel of the tile-parallel step
                for (int part = g.deferred ? 1 : 2; part <= 3 && e == hipSuccess; ++part) {
                    hipEvent_t pa = take_event(r);
                    hipEvent_t pb = pa ? take_event(r) : nullptr;
                    if (!pb) {
                        if (pa) r->pool.push_back(pa);
                        return BTC_ERR_HIP;
                    }
                    (void)hipEventRecord(pa, gs);
                    e = launch_factor_kind(g.kind, L, g.np, g.deferred, items, gs, part);
                    (void)hipEventRecord(pb, gs);
                    r->pending.push_back({std::make_tuple(g.op, g.kind, g.np, part), pa, pb, g.part[part]});
                }
                break;
            }
            case BTC_OP_FORWARD:
            case BTC_OP_BACKWARD: {
                const bool bwd = g.op == BTC_OP_BACKWARD;
                const bool range = g.kind >= 2;
                const int fk = g.kind & 1;
                const int kw = shape_waves(tune_variant(BTC_TUNE_SWEEP_SHAPE, fk, g.np, 0));
                if (fk == 1)
                    e = btc::launch_sweep(make_launch<btc::SweepDesc<float>>(g, dev), g.np, items, bwd, sweep_mc(g.op, 1, g.np, g.m_max), gs, range, kw);
                else
                    e = btc::launch_sweep(make_launch<btc::SweepDesc<double>>(g, dev), g.np, items, bwd, sweep_mc(g.op, 0, g.np, g.m_max), gs, range, kw);
                break;
            }
            case BTC_OP_RESIDUAL:
                e = btc::launch_residual(make_launch<btc::ResidualDesc>(g, dev), g.np, items, sweep_mc(BTC_OP_RESIDUAL, 0, g.np, g.m_max), gs);
                break;
            case BTC_OP_REFINE_INIT:
                e = btc::launch_ir_init(make_launch<btc::IrDesc>(g, dev), items, gs);
                break;
            default:
                e = btc::launch_ir_check(make_launch<btc::IrDesc>(g, dev), items, gs);
                break;
        }
        const auto key = std::make_tuple(g.op, g.kind, g.np, 0);
        if (g.prof && timing && !split) {
            (void)hipEventRecord(eb, gs);
            r->pending.push_back({key, ea, eb, g.work});
        } else if (g.count && timing && !split) {
            add_untimed(r, key, g.work);
        }
        return e != hipSuccess ? to_code(e) : BTC_OK;
    };
    for (auto it = groups.begin(); it != groups.end();) {
        const int stage = it->second.stage;
        auto end = it;
        while (end != groups.end() && end->second.stage == stage) ++end;
        // stream of every group of the stage: largest estimated work first,
        // each onto the least loaded of the main and side streams
        // (convergence tests run after every other group of their stage, on
        // the runner's stream once the side streams have joined: a stage may
        // hold a residual step and the test that reads it)
        std::vector<std::pair<double, Group*>> order;
        for (auto g = it; g != end; ++g) {
            Group& gr = g->second;
            if (gr.op == BTC_OP_REFINE_TEST) {
                gr.lane = 0;
                continue;
            }
            const double np = (double)std::max(gr.np, 8);
            const double w = (gr.op == BTC_OP_FACTOR ? np : 1.0) * np * np * (double)gr.items.size();
            order.push_back({w, &gr});
        }
        std::sort(order.begin(), order.end(), [](const std::pair<double, Group*>& a, const std::pair<double, Group*>& b) {
            return a.first > b.first;
        });
        double load[1 + btc_runner_s::kSide] = {};
        bool used[1 + btc_runner_s::kSide] = {};
        for (auto& o : order) {
            int best = 0;
            for (int k = 1; k <= r->nside; ++k)
                if (load[k] < load[best]) best = k;
            load[best] += o.first;
            used[best] = true;
            o.second->lane = best;
        }
        bool forked = false;
        for (int k = 1; k <= btc_runner_s::kSide; ++k) {
            if (!used[k]) continue;
            if (!forked) {
                e = hipEventRecord(r->fork, st);
                if (e != hipSuccess) return to_code(e);
                forked = true;
            }
            e = hipStreamWaitEvent(r->side[k - 1], r->fork, 0);
            if (e != hipSuccess) return to_code(e);
        }
        for (auto g = it; g != end; ++g) {
            if (g->second.op == BTC_OP_REFINE_TEST) continue;
            const int rc = launch_group(g->second);
            if (rc != BTC_OK) return rc;
        }
        for (int k = 1; k <= btc_runner_s::kSide; ++k) {
            if (!used[k]) continue;
            e = hipEventRecord(r->join[k - 1], r->side[k - 1]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, r->join[k - 1], 0);
            if (e != hipSuccess) return to_code(e);
        }
        for (auto g = it; g != end; ++g) {
            if (g->second.op != BTC_OP_REFINE_TEST) continue;
            const int rc = launch_group(g->second);
            if (rc != BTC_OK) return rc;
        }
        it = end;
    }
    return BTC_OK;
}


}  // namespace

namespace {
int runner_run(btc_runner r, int32_t count, const btc_step* steps);
}

BTC_API int btc_runner_run(btc_runner r, int32_t count, const btc_step* steps) {
    if (!r) return -1;
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = runner_run(r, count, steps);
    r->host_run_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    r->host_calls += 1;
    return rc;
}

BTC_API int btc_runner_host_stats(btc_runner r, double* run_s, double* wait_s, int64_t* calls, int reset) {
    if (!r) return -1;
    if (run_s) *run_s = r->host_run_s;
    if (wait_s) *wait_s = r->host_wait_s;
    if (calls) *calls = r->host_calls;
    if (reset) {
        r->host_run_s = r->host_wait_s = 0.0;
        r->host_calls = 0;
    }
    return BTC_OK;
}

namespace {
int runner_run(btc_runner r, int32_t count, const btc_step* steps) {
    if (count < 0) return -2;
    if (count > 0 && !steps) return -3;
    if (count == 0) return BTC_OK;
    hipStream_t st = r->st;
    int rc = prepare_steps(r, count, steps, st);
    if (rc != BTC_OK) return rc;
    Call c;
    build_call(r, count, steps, st, c);
    if (r->recording) {
        r->rec.push_back(std::move(c));
        return BTC_OK;
    }
    const size_t bytes = layout_call(c, 0);
    btc_runner_s::Slot& sl = r->slot[r->cur];
    rc = slot_reserve(r, sl, bytes);
    if (rc != BTC_OK) return rc;
    write_call(c, sl.host);
    hipError_t e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return to_code(e);
    (void)hipEventRecord(sl.ev, st);
    sl.pending = true;
    r->cur ^= 1;
    return launch_call(r, c, sl.dev, st, true);
}
}  // namespace


BTC_API int btc_graph_begin(btc_runner r) {
    if (!r) return -1;
    if (r->recording) return BTC_ERR_UNSUPPORTED;
    r->recording = true;
    r->rec.clear();
    r->rec_handles.clear();
    return BTC_OK;
}

BTC_API void btc_graph_destroy(btc_graph g) {
    if (!g) return;
    if (g->cap) (void)hipStreamSynchronize(g->cap);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    dev_free(g->alloc, g->dev, g->cap);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
}

BTC_API int btc_graph_end(btc_runner r, btc_graph* out) {
    if (!r) return -1;
    if (!out) return -2;
    *out = nullptr;
    if (!r->recording) return BTC_ERR_UNSUPPORTED;
    r->recording = false;
    std::vector<Call> calls;
    calls.swap(r->rec);
    r->rec_handles.clear();
    btc_graph g = new (std::nothrow) btc_graph_s();
    if (!g) return BTC_ERR_OOM;
    size_t bytes = 0;
    for (auto& c : calls) bytes = layout_call(c, bytes);
    std::vector<char> host(std::max<size_t>(bytes, 256));
    for (auto& c : calls) write_call(c, host.data());
    // the recorded work of the runner's stream must be done before the
    // descriptors are uploaded and the capture starts
    hipError_t e = hipStreamSynchronize(r->st);
    g->alloc = current_allocator();
    if (e == hipSuccess) e = dev_alloc(g->alloc, (void**)&g->dev, host.size(), r->st);
    if (e == hipSuccess) e = hipMemcpy(g->dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        btc_graph_destroy(g);
        return to_code(e);
    }
    int rc = BTC_OK;
    for (auto& c : calls) {
        rc = launch_call(r, c, g->dev, g->cap, false);
        if (rc != BTC_OK) break;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->cap, &graph);
    g->graph = graph;
    if (rc == BTC_OK && e != hipSuccess) rc = to_code(e);
    if (rc == BTC_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = to_code(e);
    }
    if (rc != BTC_OK) {
        btc_graph_destroy(g);
        return rc;
    }
    *out = g;
    return BTC_OK;
}

BTC_API int btc_graph_launch(btc_graph g, void* stream) {
    if (!g) return -1;
    return to_code(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

BTC_API int btc_runner_profile(btc_runner r, int32_t op, int32_t kind) {
    if (!r) return -1;
    if (op < -2 || op > BTC_OP_REFINE_TEST) return -2;
    if (kind < -1) return -3;
    (void)hipStreamSynchronize(r->st);
    drain_prof(r, true);
    r->totals.clear();
    r->prof_op = op;
    r->prof_kind = kind;
    return BTC_OK;
}

BTC_API int btc_runner_profile_read(btc_runner r, btc_kernel_stat* out, int32_t max, int32_t* count) {
    if (!r) return -1;
    if (max < 0 || (max > 0 && !out)) return -2;
    if (!count) return -4;
    const hipError_t e = hipStreamSynchronize(r->st);
    drain_prof(r, true);
    std::vector<btc_kernel_stat> v;
    for (auto& kv : r->totals) v.push_back(kv.second);
    std::sort(v.begin(), v.end(), [](const btc_kernel_stat& a, const btc_kernel_stat& b) { return a.ms > b.ms; });
    const int32_t c = (int32_t)std::min<size_t>(v.size(), (size_t)max);
    for (int32_t k = 0; k < c; ++k) out[k] = v[k];
    *count = c;
    r->totals.clear();
    return to_code(e);
}

BTC_API int btc_level_work(int32_t op, int32_t precision, int64_t N, int64_t n, int64_t nrhs, int32_t level,
                           double* bytes, double* flops) {
    if (op < BTC_OP_FACTOR || op > BTC_OP_REFINE_TEST) return -1;
    if (precision != BTC_FP64 && !is_mixed(precision)) return -2;
    if (N < 1) return -3;
    if (n < 1) return -4;
    if (nrhs < 0 || (op != BTC_OP_FACTOR && nrhs < 1)) return -5;
    if ((op <= BTC_OP_BACKWARD) && (level < 0 || level >= num_levels(N))) return -6;
    const Work w = level_work(op, is_mixed(precision), N, n, op == BTC_OP_FACTOR ? 0 : nrhs, level);
    if (bytes) *bytes = w.bytes;
    if (flops) *flops = w.flops;
    return BTC_OK;
}

BTC_API int btc_sweep_ranges(int64_t N, int32_t* bounds, int32_t max) {
    if (N < 1) return -1;
    if (!bounds) return -2;
    int b[66];
    const int r = sweep_ranges(N, num_levels(N), b);
    if (r + 1 > max) return -2;
    for (int k = 0; k <= r; ++k) bounds[k] = b[k];
    return r;
}

BTC_API int btc_runner_query(btc_runner r) {
    if (!r) return -1;
    const hipError_t e = hipStreamQuery(r->st);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return to_code(e);
}

BTC_API int btc_runner_sync(btc_runner r) {
    if (!r) return -1;
    return to_code(hipStreamSynchronize(r->st));
}

// ---------------------------------------------------------------------------
// Batched factorization and solve of independent instances on a runner: the
// levels of every instance are walked together, one group of launches per
// level, so that each launch carries the nodes of all instances at that level.

BTC_API int btc_factor_batched(btc_runner r, int32_t count, const btc_handle* h, const double* const* A_diag,
                               const double* const* A_off, int64_t* info) {
    if (!r) return -1;
    if (count < 0) return -2;
    if (count > 0 && (!h || !A_diag || !A_off)) return -3;
    if (info && r->recording) return -6;
    int levels = 0;
    for (int32_t k = 0; k < count; ++k) {
        if (!h[k]) return -3;
        levels = std::max(levels, h[k]->levels);
    }
    std::vector<btc_step> steps;
    for (int l = 0; l < levels; ++l) {
        steps.clear();
        for (int32_t k = 0; k < count; ++k) {
            if (l >= h[k]->levels) continue;
            btc_step s{};
            s.h = h[k];
            s.op = BTC_OP_FACTOR;
            s.level = l;
            s.A_diag = A_diag[k];
            s.A_off = A_off[k];
            steps.push_back(s);
        }
        const int rc = btc_runner_run(r, (int32_t)steps.size(), steps.data());
        if (rc != BTC_OK) return rc;
    }
    if (!info) return BTC_OK;
    const hipError_t e = hipStreamSynchronize(r->st);
    if (e != hipSuccess) return to_code(e);
    for (int32_t k = 0; k < count; ++k) {
        const int rc = btc_status(h[k], &info[k]);
        if (rc != BTC_OK) return rc;
    }
    return BTC_OK;
}

BTC_API int btc_solve_batched(btc_runner r, int32_t count, const btc_handle* h, const double* const* B,
                              double* const* X, const int64_t* nrhs, btc_solve_info* info) {
    if (!r) return -1;
    if (count < 0) return -2;
    if (count > 0 && (!h || !B || !X)) return -3;
    if (count > 0 && !nrhs) return -6;
    if (info && r->recording) return -7;
    int levels = 0, rounds = 1;
    bool any_mixed = false;
    for (int32_t k = 0; k < count; ++k) {
        if (nrhs[k] < 1) return -6;
        if (!h[k] || !h[k]->factored) return -3;
        if (is_mixed(h[k]->precision) && B[k] == X[k]) return -4;
        levels = std::max(levels, h[k]->levels);
        if (is_mixed(h[k]->precision)) {
            any_mixed = true;
            rounds = std::max(rounds, 1 + h[k]->max_refine);
        }
    }
    // each instance's sweeps in its level ranges; call q runs range q of
    // every instance that has one (backward: counted from the top)
    std::vector<std::vector<int>> bounds((size_t)count);
    int max_ranges = 0;
    for (int32_t k = 0; k < count; ++k) {
        bounds[(size_t)k].resize(66);
        const int nr = sweep_ranges(h[k]->N, h[k]->levels, bounds[(size_t)k].data(),
                                    sweep_shape(h[k]->precision, h[k]->n));
        bounds[(size_t)k].resize((size_t)nr + 1);
        max_ranges = std::max(max_ranges, nr);
    }
    (void)levels;
    std::vector<btc_step> steps;
    auto run_op = [&](int op, int q, bool mixed_only, int first) -> int {
        steps.clear();
        for (int32_t k = 0; k < count; ++k) {
            if (mixed_only && !is_mixed(h[k]->precision)) continue;
            btc_step s{};
            if (op == BTC_OP_FORWARD || op == BTC_OP_BACKWARD) {
                const auto& b = bounds[(size_t)k];
                const int nr = (int)b.size() - 1;
                if (q >= nr) continue;
                const int rg = op == BTC_OP_FORWARD ? q : nr - 1 - q;
                s.level = b[(size_t)rg];
                s.level_end = b[(size_t)rg + 1] > b[(size_t)rg] + 1 ? b[(size_t)rg + 1] : 0;
            }
            s.h = h[k];
            s.op = op;
            s.B = B[k];
            s.X = X[k];
            s.nrhs = nrhs[k];
            s.first = first;
            steps.push_back(s);
        }
        return btc_runner_run(r, (int32_t)steps.size(), steps.data());
    };
    int rc = BTC_OK;
    if (any_mixed) rc = run_op(BTC_OP_REFINE_INIT, 0, true, 0);
    for (int round = 0; round < rounds && rc == BTC_OK; ++round) {
        // FP64 instances take part in the first round only
        const bool only_mixed = round > 0;
        for (int q = 0; q < max_ranges && rc == BTC_OK; ++q) rc = run_op(BTC_OP_FORWARD, q, only_mixed, round == 0);
        for (int q = 0; q < max_ranges && rc == BTC_OK; ++q) rc = run_op(BTC_OP_BACKWARD, q, only_mixed, round == 0);
        if (any_mixed && rc == BTC_OK) rc = run_op(BTC_OP_RESIDUAL, 0, true, 0);
        if (any_mixed && rc == BTC_OK) rc = run_op(BTC_OP_REFINE_TEST, 0, true, 0);
    }
    if (rc != BTC_OK || !info) return rc;
    const hipError_t e = hipStreamSynchronize(r->st);
    if (e != hipSuccess) return to_code(e);
    for (int32_t k = 0; k < count; ++k) {
        if (is_mixed(h[k]->precision)) {
            rc = btc_refine_info(h[k], &info[k]);
        } else {
            int64_t st = 0;
            rc = btc_status(h[k], &st);
            if (rc == BTC_OK && st != 0) rc = BTC_ERR_NOT_SPD;
            if (rc == BTC_OK) {
                info[k].steps = 0;
                info[k].converged = 1;
                info[k].relres = -1.0;  // not computed by the FP64 path
                info[k].inner = 0;
                info[k].pad = 0;
            }
        }
        if (rc == BTC_ERR_NOT_SPD) {
            info[k].steps = 0;
            info[k].converged = 0;
            info[k].relres = -1.0;
            info[k].inner = 0;
            info[k].pad = 0;
            rc = BTC_OK;
        }
        if (rc != BTC_OK) return rc;
    }
    return BTC_OK;
}

}  // extern "C"
