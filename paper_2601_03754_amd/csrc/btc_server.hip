// Request server with continuous batching.
//
// Clients own one block-tridiagonal system shape each (N, n) and a resident
// factor (a handle).  Requests are either "refactor + solve" (a new matrix of
// the client's shape, then a solve) or "solve" against the resident factor.
// Every request is a plan of level steps (factor levels, forward / backward
// sweep levels, and for the mixed-precision path the FP64 residual and
// convergence test of each refinement round).  A tick takes the next step of
// every in-flight request and hands them to the step runner as one list, so
// requests at different levels and phases share launches, and a request that
// arrives while others are mid-tree starts at the next tick.
//
// Admission: requests are admitted in arrival order, subject to
//   * one request in flight per client (the handle and its workspace are the
//     client's; this also keeps each client's requests in order);
//   * the HBM budget: a client's factor + workspace is allocated when its
//     first request is admitted and stays resident; when the budget would be
//     exceeded, resident clients with no request in flight are evicted, least
//     recently used first, and a later "solve" request of an evicted client is
//     run as "refactor + solve" with the client's last matrix.
// Lanes (option): clients split by padded block size class, each class set
// with its own stream, runner and ticks, so small blocks are not held to the
// pace of the largest; a step call enqueues a tick on every lane with room.
// Completion: each tick records an event; a request completes when the event
// of the tick holding its last step has fired.  A mixed-precision request
// whose refinement has converged is retired early: the convergence flags of
// a tick's test steps are written into pinned host memory by one small
// kernel after them and read when the tick's event fires; the steps still
// queued for that request would only have returned at once.
#include <hip/hip_runtime.h>
#include <string.h>

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <vector>

#include "btc.h"
#include "btc_handle.h"
#include "btc_kernels.h"

using namespace btc_host;

namespace {

// Outcome of a request step as the host reads it: the factor's status word,
// and for the mixed paths the refinement state after a convergence test.
struct ReqStatus {
    unsigned long long info;  // ~0: every pivot block positive definite
    int32_t done;             // refinement finished (converged, stalled, NaN or budget spent)
    int32_t steps;            // low-precision solves applied
    int32_t converged;
    int32_t pad;
    double relres;
};

// Copy of request outcomes (device) into the pinned ring (host memory the
// device writes through its mapped address).
constexpr int kGather = 64;
struct StatusGather {
    const unsigned long long* info[kGather];
    const btc::IrState* ir[kGather];  // null: no refinement state (FP64 path)
    int32_t dst[kGather];
    int32_t count;
    ReqStatus* ring;
};

__global__ void k_gather_status(StatusGather a) {
    const int t = threadIdx.x;
    if (t < a.count) {
        ReqStatus r{};
        r.info = *a.info[t];
        if (a.ir[t]) {
            const btc::IrState s = *a.ir[t];
            r.done = s.done;
            r.steps = s.steps;
            r.converged = s.converged;
            r.relres = s.relres;
        } else {
            r.done = 1;
            r.converged = 1;
            r.relres = -1.0;
        }
        a.ring[a.dst[t]] = r;
    }
    __threadfence_system();
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Client {
    int64_t N = 0, n = 0;
    btc_handle h = nullptr;
    // matrix of the client's newest ADMITTED refactorization (admission is
    // in per-client order, so this is the matrix every later solve-only
    // request of the client refers to, also after an eviction)
    const double* A_diag = nullptr;
    const double* A_off = nullptr;
    bool has_matrix = false;  // some submitted request brought a matrix
    int lane = 0;             // the lane (stream and runner) of the client's steps
    bool busy = false;
    uint64_t last_use = 0;
    size_t bytes = 0;
};

struct Req {
    int64_t ticket = 0;
    int64_t client = 0;
    const double* A_diag = nullptr;
    const double* A_off = nullptr;
    const double* B = nullptr;
    double* X = nullptr;
    int64_t nrhs = 1;
    double t_submit = 0.0;
    double t_admit = 0.0;
    std::vector<btc_step> plan;
    std::vector<uint8_t> joint;  // joint[k]: plan step k runs in the same tick as step k+1
    std::vector<uint8_t> par;    // par[k]: step k runs in the same stage as step k-1 of its tick
    size_t pc = 0;
    bool refactored = false;
    bool retired = false;
    uint64_t last_tick = 0;  // id of the newest tick that references this request
};

struct Poll {
    Req* r;
    int slot;        // pinned ring slot of the gathered status
    bool last;       // the request's last plan step is in this tick
};

struct Tick {
    uint64_t id = 0;
    hipEvent_t ev = nullptr;
    std::vector<Poll> polls;  // status copies of refinement tests and of finishing requests
};

// A lane: a stream, a runner on it, and the ticks in flight on it.  Clients
// of one padded block size class share a lane; lanes tick independently.
struct Lane {
    hipStream_t st = nullptr;
    bool own = false;  // stream created by the server
    btc_runner runner = nullptr;
    std::deque<Tick> ticks;
};

// Ticks a lane keeps in flight: the running one, the next one queued behind
// it, and one more being enqueued (the runner's two descriptor slots).
constexpr size_t kLaneDepth = 3;
constexpr int kSizeClasses = 4;
// Lanes when the caller leaves the choice to the library: three keep the
// server's streams, with the caller's, within the four hardware queues HIP
// opens by default (measured on the served mix: one lane 8 200, two 10 400,
// three 12 600, four 8 400 requests/s of the mixed path).
constexpr int kDefaultLanes = 3;
// Side streams of each lane's runner when there are several lanes: none
// (measured on the served mix: with lanes, the fork and join of side
// streams cost more than the concurrency they add, 30-60% fewer requests/s).
constexpr int kLaneSides = 0;

}  // namespace

struct btc_server_s {
    btc_server_options opt{};
    // the caller's stream: with one lane the server's ticks run on it; with
    // several, every lane tick first waits for the work queued on it so far
    // (the requests' inputs)
    hipStream_t user_st = nullptr;
    hipEvent_t user_ev = nullptr;
    std::vector<Lane> lanes;
    std::vector<Client> clients;
    std::deque<Req*> pending;
    std::vector<Req*> active;
    std::vector<hipEvent_t> ev_pool;
    ReqStatus* flags = nullptr;      // pinned ring of request outcomes (host view)
    ReqStatus* flags_dev = nullptr;  // the same memory as the device sees it
    int flag_cap = 0, flag_next = 0;
    size_t resident = 0;
    uint64_t clock = 0;
    uint64_t next_tick = 1;
    int64_t next_ticket = 1;
    std::vector<btc_server_completion> done;
    std::vector<btc_step> scratch;
    double host_wait_s = 0.0;  // btc_server_step blocked on the oldest tick
    int64_t lane_ticks = 0;    // ticks enqueued over all lanes
};

namespace {

// Evict idle resident clients other than `keep`, least recently used first,
// until `more` bytes fit in the budget.  0: they fit; 1: they do not (some
// client still holds memory while a request of it is in flight: wait).
int make_room(btc_server s, const Client* keep, size_t more) {
    while (s->resident + more > s->opt.hbm_budget) {
        Client* victim = nullptr;
        for (auto& o : s->clients)
            if (&o != keep && o.h && !o.busy && (!victim || o.last_use < victim->last_use)) victim = &o;
        if (!victim) return 1;
        // steps issued before an early retirement may still run on its lane
        (void)hipStreamSynchronize(s->lanes[(size_t)victim->lane].st);
        btc_destroy(victim->h);
        victim->h = nullptr;
        s->resident -= victim->bytes;
        victim->bytes = 0;
    }
    return 0;
}

// Resident memory for a request of client c with nrhs right-hand sides.
// 0: admitted; 1: wait for memory; < 0: error.  Requests whose footprint
// alone exceeds the budget are refused at submission, so after every idle
// client is evicted only clients with requests in flight hold memory, and
// they release it (become evictable) when those requests complete.
int admit_client(btc_server s, Client& c, int64_t nrhs) {
    const int32_t prec = s->opt.precision;
    if (c.h) {
        if (nrhs > c.h->ws_m) {
            const size_t more = btc_footprint_bytes(c.N, c.n, prec, nrhs) - c.bytes;
            if (make_room(s, &c, more)) return 1;
            if (ensure_workspace(c.h, nrhs) != BTC_OK) return BTC_ERR_OOM;
            s->resident += more;
            c.bytes += more;
        }
        return BTC_OK;
    }
    const size_t need = btc_footprint_bytes(c.N, c.n, prec, nrhs);
    if (need == 0) return BTC_ERR_UNSUPPORTED;
    if (make_room(s, &c, need)) return 1;
    btc_options o{};
    o.precision = prec;
    o.max_refine = s->opt.max_refine;
    o.tol = s->opt.tol;
    btc_handle h = nullptr;
    int rc = btc_create(c.N, c.n, &o, &h);
    if (rc != BTC_OK) return rc;
    h->stream = s->lanes[(size_t)c.lane].st;
    rc = ensure_workspace(h, nrhs);
    if (rc != BTC_OK) {
        btc_destroy(h);
        return rc;
    }
    c.h = h;
    c.bytes = need;
    s->resident += need;
    return BTC_OK;
}

// The steps of a request, in order, grouped into ticks; within a tick a
// request's steps run in successive stages of one runner call (a step
// marked par shares its predecessor's stage).  Sweeps run in the library's
// level ranges (sweep_ranges): one tick per range.
//   * A refactor+solve request interlaces the factorization with the first
//     forward sweep (the paper's interlaced factor and forward substitution,
//     section "Fused and Blocked Kernels"): a forward range ending at level l
//     only reads factor blocks below level l, final once factor level l-1
//     has run, so it shares the tick (and stage) of factor level l, which
//     writes only blocks of level l and above.
//   * The top forward range and the top backward range share a tick.
//   * Mixed precision: the refinement set-up precedes the first forward
//     range in its tick; the residual and its convergence test follow the
//     last backward range in its tick, and the next round's first forward
//     range follows them (it does nothing once the test has stopped the
//     refinement).
void build_plan(btc_server s, Req* r, Client& c) {
    btc_handle h = c.h;
    const int L = h->levels;
    const bool factor = r->A_diag != nullptr || !h->factored;
    if (r->A_diag) {
        // requests are admitted in per-client order: from here on this is
        // the matrix an evicted client's solve-only requests refactor with
        c.A_diag = r->A_diag;
        c.A_off = r->A_off;
    }
    int b[66];
    int nr = L;
    if (!s->opt.sweep_ranges)
        for (int l = 0; l <= L; ++l) b[l] = l;
    else
        nr = sweep_ranges(h->N, L, b, sweep_shape(h->precision, h->n));
    auto push = [&](const btc_step& t, bool par) {
        r->plan.push_back(t);
        r->joint.push_back(0);
        r->par.push_back(par ? 1 : 0);
    };
    // the previous step shares its tick with the next one
    auto join_next = [&]() { r->joint.back() = 1; };
    btc_step f{};
    f.h = h;
    f.op = BTC_OP_FACTOR;
    f.A_diag = c.A_diag;
    f.A_off = c.A_off;
    btc_step t{};
    t.h = h;
    t.B = r->B;
    t.X = r->X;
    t.nrhs = r->nrhs;
    auto range = [&](btc_step& x, int op, int q) {
        x.op = op;
        x.level = b[q];
        x.level_end = b[q + 1] > b[q] + 1 ? b[q + 1] : 0;
    };
    const bool mixed = is_mixed(h->precision);
    const int rounds = mixed ? 1 + h->max_refine : 1;
    if (factor) r->refactored = true;
    for (int k = 0; k < rounds; ++k) {
        t.first = (k == 0) ? 1 : 0;
        int q = 0;  // next forward range
        if (k == 0 && factor) {
            // tick l: factor level l (with the refinement set-up at level 0)
            // and the forward range ending at level l; the top forward range
            // (ending at level L) starts the tick after
            for (int l = 0; l < L; ++l) {
                f.level = l;
                push(f, false);
                if (l == 0 && mixed) {
                    t.op = BTC_OP_REFINE_INIT;
                    t.level = 0;
                    t.level_end = 0;
                    join_next();
                    push(t, true);
                }
                if (q < nr && b[q + 1] == l) {
                    range(t, BTC_OP_FORWARD, q++);
                    join_next();
                    push(t, true);
                }
            }
        } else if (k == 0 && mixed) {
            t.op = BTC_OP_REFINE_INIT;
            t.level = 0;
            t.level_end = 0;
            push(t, false);
            join_next();  // the first forward range follows in the same tick
        } else if (k > 0 && nr > 1) {
            // after the previous round's test, in its tick (with a single
            // range the round starts a tick of its own: a tick holds at most
            // one round's sweeps)
            join_next();
        }
        for (; q < nr; ++q) {
            range(t, BTC_OP_FORWARD, q);
            push(t, false);
        }
        // top backward range right after the top forward range
        join_next();
        for (int g = nr - 1; g >= 0; --g) {
            range(t, BTC_OP_BACKWARD, g);
            push(t, false);
        }
        if (mixed) {
            // residual and test after the last backward range, in its tick
            join_next();
            t.level = 0;
            t.level_end = 0;
            t.op = BTC_OP_RESIDUAL;
            push(t, false);
            join_next();
            t.op = BTC_OP_REFINE_TEST;
            push(t, true);
        }
    }
}

void complete(btc_server s, Req* r, double t, const ReqStatus& st) {
    if (r->retired) return;
    r->retired = true;
    Client& c = s->clients[(size_t)r->client];
    c.busy = false;
    c.last_use = ++s->clock;
    btc_server_completion d{};
    d.ticket = r->ticket;
    d.client = r->client;
    d.t_submit = r->t_submit;
    d.t_admit = r->t_admit;
    d.t_done = t;
    d.refactored = r->refactored ? 1 : 0;
    d.info = st.info == kInfoOk ? 0 : (int64_t)st.info;
    const bool mixed = is_mixed(s->opt.precision);
    d.steps = mixed ? std::max(0, st.steps - 1) : 0;
    d.converged = (d.info == 0 && st.converged) ? 1 : 0;
    d.relres = d.info == 0 ? st.relres : -1.0;
    s->done.push_back(d);
}

// Retire every tick whose event has fired (in order on each lane; with wait,
// every tick).
void harvest(btc_server s, bool wait) {
    for (Lane& ln : s->lanes) {
        while (!ln.ticks.empty()) {
            Tick& t = ln.ticks.front();
            if (wait) {
                (void)hipEventSynchronize(t.ev);
            } else if (hipEventQuery(t.ev) != hipSuccess) {
                break;
            }
            const double tn = now_s();
            for (auto& p : t.polls) {
                const ReqStatus st = s->flags[p.slot];
                // a request is done after its last step, or earlier once its
                // refinement has stopped (the steps still queued for it return
                // at once), or once its factorization has broken down
                if (p.last || st.done != 0 || st.info != kInfoOk) complete(s, p.r, tn, st);
            }
            s->ev_pool.push_back(t.ev);
            ln.ticks.pop_front();
        }
    }
    // drop retired requests that no outstanding tick refers to any more
    uint64_t oldest = UINT64_MAX;
    for (const Lane& ln : s->lanes)
        if (!ln.ticks.empty()) oldest = std::min(oldest, ln.ticks.front().id);
    auto it = std::remove_if(s->active.begin(), s->active.end(), [oldest](Req* r) {
        if (r->retired && r->last_tick < oldest) {
            delete r;
            return true;
        }
        return false;
    });
    s->active.erase(it, s->active.end());
}

// Padded block size class of n: 0 (up to 16), 1 (32), 2 (64), 3 (96, 128).
int size_class(int64_t n) {
    const int np = btc::padded_block((int)n);
    return np <= 16 ? 0 : np <= 32 ? 1 : np <= 64 ? 2 : 3;
}

// One tick on lane li: the next steps of every in-flight request of the
// lane's clients, as one runner call, then the gather of the tick's request
// outcomes and the tick's event.  Returns 1 if the lane had steps to run.
int issue_tick(btc_server s, int li, int* rc_out) {
    Lane& ln = s->lanes[(size_t)li];
    Tick t;
    t.id = s->next_tick;
    s->scratch.clear();
    for (Req* r : s->active) {
        if (r->retired || r->pc >= r->plan.size()) continue;  // done, or waiting for its last tick
        if (s->clients[(size_t)r->client].lane != li) continue;
        r->last_tick = t.id;
        bool more = true, test = false;
        int stage = -1;
        while (more && r->pc < r->plan.size()) {
            const bool par = r->par[r->pc] != 0 && stage >= 0;
            if (!par && stage >= 7) break;  // stages of a runner call: the rest goes in the next tick
            more = r->joint[r->pc] != 0;
            btc_step st = r->plan[r->pc++];
            stage += par ? 0 : 1;
            st.stage = stage;
            s->scratch.push_back(st);
            test = test || st.op == BTC_OP_REFINE_TEST;
        }
        const bool last = r->pc == r->plan.size();
        if (test || last) {
            t.polls.push_back({r, s->flag_next, last});
            s->flag_next = (s->flag_next + 1) % s->flag_cap;
        }
    }
    *rc_out = BTC_OK;
    if (s->scratch.empty()) return 0;
    s->next_tick++;
    if (s->user_ev) {
        if (hipEventRecord(s->user_ev, s->user_st) != hipSuccess ||
            hipStreamWaitEvent(ln.st, s->user_ev, 0) != hipSuccess) {
            *rc_out = BTC_ERR_HIP;
            return 1;
        }
    }
    int rc = btc_runner_run(ln.runner, (int32_t)s->scratch.size(), s->scratch.data());
    if (rc != BTC_OK) {
        *rc_out = rc;
        return 1;
    }
    // the outcomes of this tick's tests and finishing requests, copied into
    // the pinned ring by one small kernel (not one copy command each)
    StatusGather ga{};
    ga.ring = s->flags_dev;
    const bool mixed = is_mixed(s->opt.precision);
    for (size_t k = 0; k < t.polls.size(); ++k) {
        const auto& p = t.polls[k];
        btc_handle h = p.r->plan[0].h;
        const Workspace w = carve(h, h->ws_m);
        s->flags[p.slot] = ReqStatus{};
        ga.info[ga.count] = h->info;
        ga.ir[ga.count] = mixed ? w.ir : nullptr;
        ga.dst[ga.count] = p.slot;
        if (++ga.count == kGather || k + 1 == t.polls.size()) {
            hipLaunchKernelGGL(k_gather_status, dim3(1), dim3(kGather), 0, ln.st, ga);
            if (hipGetLastError() != hipSuccess) {
                *rc_out = BTC_ERR_HIP;
                return 1;
            }
            ga.count = 0;
        }
    }
    if (!s->ev_pool.empty()) {
        t.ev = s->ev_pool.back();
        s->ev_pool.pop_back();
    } else if (hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess) {
        *rc_out = BTC_ERR_HIP;
        return 1;
    }
    if (hipEventRecord(t.ev, ln.st) != hipSuccess) {
        *rc_out = BTC_ERR_HIP;
        return 1;
    }
    ln.ticks.push_back(std::move(t));
    s->lane_ticks += 1;
    return 1;
}

}  // namespace

extern "C" {

BTC_API int btc_server_create(const btc_server_options* opt, void* stream, btc_server* out) {
    if (!opt) return -1;
    if (opt->precision != BTC_FP64 && !is_mixed(opt->precision)) return -1;
    if (opt->max_refine < 0 || opt->max_active < 0 || !(opt->tol >= 0.0) || opt->lanes < 0) return -1;
    if (!out) return -3;
    *out = nullptr;
    btc_server s = new (std::nothrow) btc_server_s();
    if (!s) return BTC_ERR_OOM;
    s->opt = *opt;
    if (s->opt.max_refine == 0)
        s->opt.max_refine = is_bf16(s->opt.precision) ? BTC_DEFAULT_MAX_REFINE_BF16 : BTC_DEFAULT_MAX_REFINE;
    if (s->opt.tol == 0.0) s->opt.tol = BTC_DEFAULT_TOL;
    if (s->opt.max_active == 0) s->opt.max_active = 1 << 20;
    const int nl = s->opt.lanes == 0 ? kDefaultLanes : s->opt.lanes == 1 ? 1 : std::min<int>(s->opt.lanes, kSizeClasses);
    s->lanes.resize((size_t)nl);
    s->user_st = (hipStream_t)stream;
    int rc = BTC_OK;
    if (nl > 1 && hipEventCreateWithFlags(&s->user_ev, hipEventDisableTiming) != hipSuccess) rc = BTC_ERR_HIP;
    for (int k = 0; k < nl && rc == BTC_OK; ++k) {
        Lane& ln = s->lanes[(size_t)k];
        if (nl == 1) {
            ln.st = (hipStream_t)stream;
        } else if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess) {
            rc = BTC_ERR_HIP;
            break;
        } else {
            ln.own = true;
        }
        // one lane spreads a tick's groups over three side streams; several
        // lanes run side by side, each on its stream alone
        rc = runner_create(ln.st, nl == 1 ? 3 : kLaneSides, &ln.runner);
    }
    if (rc == BTC_OK) {
        s->flag_cap = 1 << 16;
        if (hipHostMalloc((void**)&s->flags, sizeof(ReqStatus) * s->flag_cap, hipHostMallocMapped) != hipSuccess)
            rc = BTC_ERR_OOM;
        else if (hipHostGetDevicePointer((void**)&s->flags_dev, s->flags, 0) != hipSuccess)
            rc = BTC_ERR_HIP;
    }
    if (rc != BTC_OK) {
        btc_server_destroy(s);
        return rc;
    }
    *out = s;
    return BTC_OK;
}

BTC_API int btc_server_add_client(btc_server s, int64_t N, int64_t n, int64_t* client) {
    if (!s) return -1;
    if (N < 1) return -2;
    if (n < 1) return -3;
    if (n > BTC_MAX_BLOCK) return BTC_ERR_UNSUPPORTED;
    if (!client) return -4;
    Client c;
    c.N = N;
    c.n = n;
    // size classes spread evenly over the lanes
    c.lane = size_class(n) * (int)s->lanes.size() / kSizeClasses;
    s->clients.push_back(c);
    *client = (int64_t)s->clients.size() - 1;
    return BTC_OK;
}

BTC_API int btc_server_submit(btc_server s, int64_t client, const double* A_diag, const double* A_off,
                              const double* B, double* X, int64_t nrhs, int64_t* ticket) {
    if (!s) return -1;
    if (client < 0 || client >= (int64_t)s->clients.size()) return -2;
    Client& c = s->clients[(size_t)client];
    if (A_diag && c.N > 1 && !A_off) return -4;
    if (!A_diag && !c.has_matrix) return -3;  // a first request must bring the matrix
    if (!B) return -5;
    if (!X || (is_mixed(s->opt.precision) && X == B)) return -6;
    if (nrhs < 1) return -7;
    // a request that could never be admitted, even alone
    if (btc_footprint_bytes(c.N, c.n, s->opt.precision, nrhs) > s->opt.hbm_budget) return BTC_ERR_UNSUPPORTED;
    Req* r = new (std::nothrow) Req();
    if (!r) return BTC_ERR_OOM;
    r->ticket = s->next_ticket++;
    r->client = client;
    r->A_diag = A_diag;
    r->A_off = A_off;
    r->B = B;
    r->X = X;
    r->nrhs = nrhs;
    r->t_submit = now_s();
    if (A_diag) c.has_matrix = true;
    s->pending.push_back(r);
    if (ticket) *ticket = r->ticket;
    return BTC_OK;
}

BTC_API int btc_server_step(btc_server s) {
    if (!s) return -1;
    harvest(s, false);

    // admission, in arrival order
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        if ((int)s->active.size() >= s->opt.max_active) break;
        Req* r = *it;
        Client& c = s->clients[(size_t)r->client];
        if (c.busy) {
            ++it;
            continue;
        }
        const int rc = admit_client(s, c, r->nrhs);
        if (rc == 1) break;  // out of budget: keep arrival order
        if (rc != BTC_OK) return rc;
        c.busy = true;
        c.last_use = ++s->clock;
        r->t_admit = now_s();
        build_plan(s, r, c);
        s->active.push_back(r);
        it = s->pending.erase(it);
    }

    // one tick on every lane with fewer than kLaneDepth ticks in flight; if
    // no lane could take one, wait for the oldest tick in flight
    for (;;) {
        bool issued = false, blocked = false;
        for (int li = 0; li < (int)s->lanes.size(); ++li) {
            if (s->lanes[(size_t)li].ticks.size() >= kLaneDepth) {
                blocked = true;
                continue;
            }
            int rc = BTC_OK;
            issued = issue_tick(s, li, &rc) != 0 || issued;
            if (rc != BTC_OK) return rc;
        }
        if (issued || !blocked) break;
        Lane* old = nullptr;
        for (Lane& ln : s->lanes)
            if (!ln.ticks.empty() && (!old || ln.ticks.front().id < old->ticks.front().id)) old = &ln;
        const double t0 = now_s();
        (void)hipEventSynchronize(old->ticks.front().ev);
        s->host_wait_s += now_s() - t0;
        harvest(s, false);
    }
    return (int)(s->pending.size() + s->active.size());
}

BTC_API int btc_server_poll(btc_server s, btc_server_completion* out, int32_t max, int32_t* count, int wait) {
    if (!s) return -1;
    if (max < 0) return -3;
    if (!count) return -4;
    harvest(s, wait != 0);
    const int32_t k = std::min<int32_t>(max, (int32_t)s->done.size());
    if (k > 0 && !out) return -2;
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[(size_t)i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *count = k;
    return BTC_OK;
}

BTC_API int btc_server_stats(btc_server s, int64_t* queued, int64_t* in_flight, size_t* resident_bytes) {
    if (!s) return -1;
    if (queued) *queued = (int64_t)s->pending.size();
    if (in_flight) *in_flight = (int64_t)s->active.size();
    if (resident_bytes) *resident_bytes = s->resident;
    return BTC_OK;
}

BTC_API btc_handle btc_server_client_handle(btc_server s, int64_t client) {
    if (!s || client < 0 || client >= (int64_t)s->clients.size()) return nullptr;
    return s->clients[(size_t)client].h;
}

BTC_API void btc_server_destroy(btc_server s) {
    if (!s) return;
    for (auto& ln : s->lanes)
        if (ln.st) (void)hipStreamSynchronize(ln.st);
    for (Req* r : s->pending) delete r;
    for (Req* r : s->active) delete r;
    for (auto& ln : s->lanes)
        for (auto& t : ln.ticks)
            if (t.ev) (void)hipEventDestroy(t.ev);
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
    for (auto& c : s->clients)
        if (c.h) btc_destroy(c.h);
    for (auto& ln : s->lanes) {
        if (ln.runner) btc_runner_destroy(ln.runner);
        if (ln.own && ln.st) (void)hipStreamDestroy(ln.st);
    }
    if (s->flags) (void)hipHostFree(s->flags);
    if (s->user_ev) (void)hipEventDestroy(s->user_ev);
    delete s;
}

}  // extern "C"

BTC_API btc_runner btc_server_runner(btc_server s) { return s && !s->lanes.empty() ? s->lanes[0].runner : nullptr; }

BTC_API int btc_server_host_stats(btc_server s, double* wait_s, int64_t* ticks, int reset) {
    if (!s) return -1;
    if (wait_s) *wait_s = s->host_wait_s;
    if (ticks) *ticks = s->lane_ticks;
    if (reset) {
        s->host_wait_s = 0.0;
        s->lane_ticks = 0;
    }
    return BTC_OK;
}

BTC_API btc_runner btc_server_lane_runner(btc_server s, int32_t lane) {
    if (!s || lane < 0 || lane >= (int32_t)s->lanes.size()) return nullptr;
    return s->lanes[(size_t)lane].runner;
}
