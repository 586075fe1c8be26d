// server.hip -- the serving loop (rmpc_server_*, rmpc_submit, rmpc_poll*): a library thread
// that turns a FIFO queue of requests into overlapping persistent launches on a pool of
// launch slots.  Host code only; the launches are the batch kernel of raycast.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "rmpc_host.h"

namespace rmpc_host {

using Clock = std::chrono::steady_clock;

namespace {

constexpr int kMaxSlots = 8;
constexpr int kDefaultPending = 65536;
constexpr double kLaunchTimeoutS = 60.0;
constexpr std::chrono::microseconds kIdleWatch(1000);   // queue watch before the server thread sleeps
constexpr size_t kWarmPieceBytes = size_t(64) << 10;    // one warm-up copy (up to the staging size)
constexpr int kWarmDepthMax = 1024;                      // warm-up copies queued per stream

// A request between rmpc_submit and its launch.
struct Req {
    uint64_t ticket = 0;
    rmpc::BatchQuery Q;          // validated descriptor (tiles placed at launch)
    int32_t n_tiles = 0;
    const float *points_host = nullptr;
    size_t stage_bytes = 0;      // device staging for host points (0 = none)
    size_t stage_off = 0;
    Clock::time_point t_submit;
};

struct Done {
    rmpc_result res;
    double latency_s;
};

struct Slot {
    LaunchSlot ls;
    bool busy = false;
    uint64_t seq = 0;
    Clock::time_point t_launch;
    Clock::time_point t_check;       // next stream check (see kStreamCheck)
    std::vector<Req> members;
};

}  // namespace

struct ServerState {
    rmpc_server_config cfg;
    rmpc_sched::Limits lim;
    int max_pending = kDefaultPending;
    size_t staging_off = 0;      // arena offset of the staging memory
    uint8_t *staging = nullptr;
    rmpc_sched::Arena stage_alloc;   // used by the server thread only
    Slot slots[kMaxSlots];
    int n_slots = 0;

    std::mutex mu;               // guards everything below
    std::condition_variable cv;
    std::deque<Req> pending;
    std::unordered_map<uint64_t, Done> done;
    std::deque<uint64_t> done_order;
    std::unordered_set<uint64_t> outstanding;   // queued or running
    uint64_t last_wait_ticket = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    rmpc_status error = RMPC_OK;
    std::string error_msg;
    rmpc_server_counters ctr;
    // written under mu, read without it: the server thread takes mu only when a request waits
    // (or to sleep), and pollers only when a result or an error is there, so that a caller
    // polling in a tight loop does not keep the server thread off the lock
    std::atomic<int64_t> n_pending{0};       // == pending.size()
    std::atomic<int64_t> n_ready{0};         // == done_order.size()
    std::atomic<bool> failed{false};         // error != RMPC_OK

    std::thread th;
};

namespace {

// Set the sticky error and wake every waiter (called with mu held).
void set_error(ServerState *S, rmpc_status st, const std::string &msg)
{
    if (S->error == RMPC_OK) {
        S->error = st;
        S->error_msg = msg;
        S->failed.store(true, std::memory_order_release);
    }
}

// Collect a finished slot: results to the done table, staging back to the allocator.
void collect(ServerState *S, Slot &sl, Clock::time_point now)
{
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t k = 0; k < sl.members.size(); ++k) {
        const Req &r = sl.members[k];
        Done d;
        d.res = sl.ls.results_host[k];
        d.latency_s = std::chrono::duration<double>(now - r.t_submit).count();
        S->done.emplace(r.ticket, d);
        S->outstanding.erase(r.ticket);
        S->done_order.push_back(r.ticket);
    }
    S->n_ready.store((int64_t)S->done_order.size(), std::memory_order_release);
    S->ctr.completed += sl.members.size();
    S->ctr.in_flight -= sl.members.size();
    rmpc_sched::release_launch(sl.members, S->stage_alloc);
    sl.members.clear();
    sl.busy = false;
}

// Spins for `ticks` of the GPU's constant-rate clock (and at most 2^24 iterations).
__global__ void warm_spin_kernel(uint64_t ticks)
{
    const uint64_t t0 = wall_clock64();
    for (uint32_t n = 0; n < (1u << 24) && wall_clock64() - t0 < ticks; ++n) {
    }
}

// Before the server takes requests, every slot's stream does once what serving makes it do, so
// that the runtime grows its per-stream state now and not under load, where each growth held
// the server thread for milliseconds while requests queued behind it:
//  * copies from pinned host memory queued deep behind a running kernel, to twice the depth that
//    a launch of max_batch scans makes (measured: the first time a stream held more than about
//    four outstanding copies, and a few times after as the depth rose, one copy call took
//    6-11 ms; at a constant depth, never again);
//  * an empty batch launch (no queries, no tiles: every block leaves at once), as the first
//    launch of the batch kernel in a process took ~3 ms.
rmpc_status warm_slots(rmpc_ctx *ctx, ServerState *S)
{
    const size_t stage = S->cfg.staging_bytes / kAlign * kAlign;
    if (stage) {
        const size_t piece = std::min<size_t>(stage, kWarmPieceBytes);
        const size_t n_pieces = stage / piece;
        const int depth = std::min(2 * (S->cfg.max_batch + 1), kWarmDepthMax);
        void *h = nullptr;
        RMPC_HIP(hipHostMalloc(&h, piece, 0));
        hipError_t e = hipSuccess;
        for (int round = 0; round < 3 && e == hipSuccess; ++round) {
            for (int i = 0; i < S->n_slots && e == hipSuccess; ++i) {
                warm_spin_kernel<<<1, 64, 0, S->slots[i].ls.stream>>>(20000);   // 200 us at 100 MHz
                e = hipGetLastError();
            }
            for (int k = 0; k < depth && e == hipSuccess; ++k)
                for (int i = 0; i < S->n_slots && e == hipSuccess; ++i)
                    e = hipMemcpyAsync(S->staging + piece * ((size_t)k % n_pieces), h, piece,
                                       hipMemcpyHostToDevice, S->slots[i].ls.stream);
            for (int i = 0; i < S->n_slots && e == hipSuccess; ++i) e = hipStreamSynchronize(S->slots[i].ls.stream);
        }
        (void)hipHostFree(h);
        if (e != hipSuccess) return fail(RMPC_E_HIP, std::string("server warm-up: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < S->n_slots; ++i) {
        LaunchSlot &ls = S->slots[i].ls;
        if (ls.graph) RMPC_HIP(hipGraphUpload(ls.graph, ls.stream));
        uint64_t seq = 0;
        if (rmpc_status st = slot_launch(ctx, ls, 0, 0, S->cfg.launch, nullptr, &seq)) return st;
        RMPC_HIP(hipStreamSynchronize(ls.stream));
    }
    return RMPC_OK;
}

// Copies of host points and the launch of a formed batch on slot sl (server thread).
rmpc_status launch_slot(rmpc_ctx *ctx, ServerState *S, Slot &sl)
{
    const int nq = (int)sl.members.size();
    int tile = 0;
    for (int k = 0; k < nq; ++k) {
        Req &r = sl.members[(size_t)k];
        if (r.stage_bytes) {
            float *dst = reinterpret_cast<float *>(S->staging + r.stage_off);
            RMPC_HIP(hipMemcpyAsync(dst, r.points_host, sizeof(float) * 3 * (size_t)r.Q.scan.n_points,
                                    hipMemcpyHostToDevice, sl.ls.stream));
            r.Q.scan.points = dst;
        }
        rmpc::BatchQuery &Q = sl.ls.q_host[k];
        Q = r.Q;
        Q.tile_begin = tile;
        tile += Q.n_tiles;
    }
    uint64_t seq = 0;
    if (rmpc_status st = slot_launch(ctx, sl.ls, nq, tile, S->cfg.launch, nullptr, &seq)) return st;
    sl.seq = seq;
    sl.busy = true;
    sl.t_launch = Clock::now();
    sl.t_check = sl.t_launch + kStreamCheck;
    return RMPC_OK;
}

void server_loop(rmpc_ctx *ctx, ServerState *S)
{
    (void)hipSetDevice(ctx->device);
    uint64_t spins = 0;
    for (;;) {
        // 1. completions (lock-free reads of the completion words)
        bool in_flight = false;
        for (int i = 0; i < S->n_slots; ++i) {
            Slot &sl = S->slots[i];
            if (!sl.busy) continue;
            if (__atomic_load_n(sl.ls.done_host, __ATOMIC_ACQUIRE) == sl.seq) {
                collect(S, sl, Clock::now());
                continue;
            }
            in_flight = true;
            // the stream is checked for errors only for launches older than kStreamCheck, once
            // per kStreamCheck, as wait_done does
            if ((spins & 255) == 0 && Clock::now() >= sl.t_check) {
                sl.t_check = Clock::now() + kStreamCheck;
                const hipError_t e = hipStreamQuery(sl.ls.stream);
                std::string msg;
                if (e == hipSuccess && __atomic_load_n(sl.ls.done_host, __ATOMIC_ACQUIRE) != sl.seq)
                    msg = "launch finished without publishing its results";
                else if (e != hipSuccess && e != hipErrorNotReady)
                    msg = std::string("launch failed: ") + hipGetErrorString(e);
                else if (std::chrono::duration<double>(Clock::now() - sl.t_launch).count() > kLaunchTimeoutS)
                    msg = "launch did not finish within 60 s";
                if (!msg.empty()) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    set_error(S, RMPC_E_HIP, msg);
                    S->cv.notify_all();
                    return;
                }
            }
        }
        // 2. admission: a free slot takes requests from the front of the queue
        int free_slot = -1;
        for (int i = 0; i < S->n_slots && free_slot < 0; ++i)
            if (!S->slots[i].busy) free_slot = i;
        if (in_flight && !(free_slot >= 0 && S->n_pending.load(std::memory_order_acquire) > 0) &&
            !S->failed.load(std::memory_order_acquire)) {
            // launches running and nothing to admit: keep watching the completion words
            ++spins;
            __builtin_ia32_pause();
            continue;
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->error != RMPC_OK) return;
        if (free_slot >= 0 && !S->pending.empty()) {
            Slot &sl = S->slots[free_slot];
            const rmpc_sched::Formed f = rmpc_sched::form_launch(S->pending, S->lim, S->stage_alloc, sl.members);
            if (f.staging_wait && S->pending.front().ticket != S->last_wait_ticket) {
                ++S->ctr.staging_waits;               // counted once per request that waits
                S->last_wait_ticket = S->pending.front().ticket;
            }
            if (f.n > 0) {
                S->ctr.pending -= (uint64_t)f.n;
                S->n_pending.store((int64_t)S->pending.size(), std::memory_order_release);
                S->ctr.in_flight += (uint64_t)f.n;
                S->ctr.launches += 1;
                S->ctr.batch_max = std::max<uint64_t>(S->ctr.batch_max, (uint64_t)f.n);
                S->ctr.staging_peak = std::max<uint64_t>(S->ctr.staging_peak, S->stage_alloc.in_use());
                lk.unlock();
                const rmpc_status st = launch_slot(ctx, S, sl);
                if (st != RMPC_OK) {
                    lk.lock();
                    set_error(S, st, g_last_error);
                    S->cv.notify_all();
                    return;
                }
                continue;
            }
        }
        if (!in_flight) {
            if (S->stop && S->pending.empty()) return;
            if (S->pending.empty()) {
                // nothing running: watch the queue for a while, then sleep until a request
                // arrives or stop is asked (at steady request rates the next request comes
                // within the watch, and a sleeping thread can take milliseconds to wake)
                lk.unlock();
                const Clock::time_point t_idle = Clock::now();
                while (S->n_pending.load(std::memory_order_acquire) == 0 && Clock::now() - t_idle < kIdleWatch)
                    __builtin_ia32_pause();
                lk.lock();
                S->cv.wait(lk, [S] { return S->stop || !S->pending.empty(); });
            }
            continue;
        }
        lk.unlock();
        ++spins;
        __builtin_ia32_pause();
    }
}

rmpc_status check_server_config(const rmpc_server_config *c)
{
    if (!c) return fail(RMPC_E_INVALID, "config is NULL");
    if (c->n_slots < 1 || c->n_slots > kMaxSlots) return fail(RMPC_E_INVALID, "n_slots out of [1, 8]");
    if (c->max_batch < 1 || c->max_batch > rmpc::kBatchMaxQueries)
        return fail(RMPC_E_INVALID, "max_batch out of [1, 4096]");
    if (c->max_tiles < 0 || c->max_tiles > rmpc::kBatchMaxTiles)
        return fail(RMPC_E_INVALID, "max_tiles out of [0, 262144]");
    if (c->max_pending < 0) return fail(RMPC_E_INVALID, "max_pending is negative");
    if (rmpc_status st = check_params(&c->map_params)) return st;
    if (rmpc_status st = check_params(&c->scan_params)) return st;
    return check_config(&c->launch);
}

}  // namespace

void server_destroy(rmpc_ctx *ctx)
{
    ServerState *S = ctx->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    for (int i = 0; i < S->n_slots; ++i) slot_destroy(ctx, S->slots[i].ls);
    if (S->staging) ctx->alloc.release(S->staging_off);
    ctx->server = nullptr;
    delete S;
}

}  // namespace rmpc_host

using namespace rmpc_host;

extern "C" {

rmpc_status rmpc_server_start(rmpc_ctx *ctx, const rmpc_server_config *cfg)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (ctx->server) return fail(RMPC_E_INVALID, "the server is already running");
    if (rmpc_status st = check_server_config(cfg)) return st;
    DeviceGuard dg(ctx->device);
    ServerState *S = new ServerState();
    S->cfg = *cfg;
    S->lim.max_queries = cfg->max_batch;
    S->lim.max_tiles = cfg->max_tiles > 0 ? cfg->max_tiles : rmpc::kBatchMaxTiles;
    S->max_pending = cfg->max_pending > 0 ? cfg->max_pending : kDefaultPending;
    std::memset(&S->ctr, 0, sizeof S->ctr);
    ctx->server = S;             // server_destroy now undoes whatever follows
    if (cfg->staging_bytes) {
        if (!ctx->alloc.alloc(cfg->staging_bytes, &S->staging_off)) {
            server_destroy(ctx);
            return fail(RMPC_E_NOMEM, "arena too small for the staging memory");
        }
        S->staging = ctx->arena + S->staging_off;
        S->stage_alloc.init(cfg->staging_bytes / kAlign * kAlign);
    }
    for (int i = 0; i < cfg->n_slots; ++i) {
        S->n_slots = i + 1;
        rmpc_status st = slot_create(ctx, S->slots[i].ls, cfg->max_batch, S->lim.max_tiles);
        // every slot's graph is captured now, so that no request waits for a capture
        if (!st && cfg->launch.use_graph) st = slot_graph(ctx, S->slots[i].ls, cfg->launch);
        if (st) {
            const std::string msg = g_last_error;
            server_destroy(ctx);
            return fail(st, msg);
        }
    }
    if (rmpc_status st = warm_slots(ctx, S)) {
        const std::string msg = g_last_error;
        server_destroy(ctx);
        return fail(st, msg);
    }
    S->th = std::thread(server_loop, ctx, S);
    return RMPC_OK;
}

rmpc_status rmpc_submit(rmpc_ctx *ctx, const rmpc_request *req, uint64_t *ticket)
{
    const Clock::time_point t0 = Clock::now();
    if (!ctx || !req || !ticket) return fail(RMPC_E_INVALID, "NULL argument");
    ServerState *S = ctx->server;
    if (!S) return fail(RMPC_E_STOPPED, "no server is running");
    Req r;
    r.t_submit = t0;
    rmpc_query_desc d = req->q;
    const bool host_points = d.kind == RMPC_KIND_SCAN && req->points_host != nullptr;
    if (host_points) {
        if (d.n > 0 && !S->staging) return fail(RMPC_E_NOMEM, "scan points from host memory need staging memory");
        d.points_dev = reinterpret_cast<const float *>(req->points_host);    // validated non-NULL only
    }
    if (rmpc_status st = batch_describe(ctx, d, 0, &S->cfg.map_params, &S->cfg.scan_params, S->cfg.launch, r.Q)) {
        g_last_error = "request: " + g_last_error.substr(g_last_error.find(": ") + 2);
        return st;
    }
    r.n_tiles = r.Q.n_tiles;
    if (r.n_tiles > S->lim.max_tiles) return fail(RMPC_E_INVALID, "request needs more tiles than one launch holds");
    if (host_points && d.n > 0) {
        r.points_host = req->points_host;
        r.stage_bytes = sizeof(float) * 3 * (size_t)d.n;
        if ((r.stage_bytes + kAlign - 1) / kAlign * kAlign > S->cfg.staging_bytes / kAlign * kAlign)
            return fail(RMPC_E_NOMEM, "scan points larger than the staging memory");
        r.Q.scan.points = nullptr;   // set to the staging copy at launch
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error != RMPC_OK) return fail(RMPC_E_STOPPED, "server stopped: " + S->error_msg);
    if (S->stop) return fail(RMPC_E_STOPPED, "server is stopping");
    if ((int)S->pending.size() >= S->max_pending) {
        ++S->ctr.refused;
        return fail(RMPC_E_NOMEM, "request queue full");
    }
    r.ticket = S->next_ticket++;
    *ticket = r.ticket;
    S->outstanding.insert(r.ticket);
    S->pending.push_back(std::move(r));
    S->n_pending.store((int64_t)S->pending.size(), std::memory_order_release);
    ++S->ctr.submitted;
    ++S->ctr.pending;
    S->cv.notify_one();
    return RMPC_OK;
}

rmpc_status rmpc_poll(rmpc_ctx *ctx, uint64_t ticket, rmpc_result *out, int32_t *done, double *latency_s)
{
    if (!ctx || !out || !done) return fail(RMPC_E_INVALID, "NULL argument");
    ServerState *S = ctx->server;
    if (!S) return fail(RMPC_E_STOPPED, "no server is running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it != S->done.end()) {
        *out = it->second.res;
        if (latency_s) *latency_s = it->second.latency_s;
        *done = 1;
        S->done.erase(it);
        return RMPC_OK;
    }
    if (S->error != RMPC_OK) return fail(RMPC_E_STOPPED, "server stopped: " + S->error_msg);
    if (!S->outstanding.count(ticket)) return fail(RMPC_E_INVALID, "unknown or retired ticket");
    *done = 0;
    return RMPC_OK;
}

rmpc_status rmpc_poll_completed(rmpc_ctx *ctx, int32_t max, uint64_t *tickets, rmpc_result *out,
                                double *latency_s, int32_t *n_out)
{
    if (!ctx || !tickets || !out || !n_out) return fail(RMPC_E_INVALID, "NULL argument");
    if (max < 0) return fail(RMPC_E_INVALID, "max is negative");
    ServerState *S = ctx->server;
    if (!S) return fail(RMPC_E_STOPPED, "no server is running");
    if (S->n_ready.load(std::memory_order_acquire) == 0 && !S->failed.load(std::memory_order_acquire)) {
        *n_out = 0;                                      // nothing there: no lock taken
        return RMPC_OK;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t n = 0;
    while (n < max && !S->done_order.empty()) {
        const uint64_t t = S->done_order.front();
        S->done_order.pop_front();
        auto it = S->done.find(t);
        if (it == S->done.end()) continue;               // already retired by rmpc_poll
        tickets[n] = t;
        out[n] = it->second.res;
        if (latency_s) latency_s[n] = it->second.latency_s;
        S->done.erase(it);
        ++n;
    }
    S->n_ready.store((int64_t)S->done_order.size(), std::memory_order_release);
    *n_out = n;
    if (n == 0 && S->error != RMPC_OK) return fail(RMPC_E_STOPPED, "server stopped: " + S->error_msg);
    return RMPC_OK;
}

rmpc_status rmpc_server_stats(rmpc_ctx *ctx, rmpc_server_counters *out)
{
    if (!ctx || !out) return fail(RMPC_E_INVALID, "NULL argument");
    ServerState *S = ctx->server;
    if (!S) return fail(RMPC_E_STOPPED, "no server is running");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->ctr;
    return RMPC_OK;
}

rmpc_status rmpc_server_stop(rmpc_ctx *ctx)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    ServerState *S = ctx->server;
    if (!S) return fail(RMPC_E_STOPPED, "no server is running");
    DeviceGuard dg(ctx->device);
    rmpc_status st = RMPC_OK;
    std::string msg;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    if (S->error != RMPC_OK) {
        st = RMPC_E_HIP;
        msg = "server failed: " + S->error_msg;
    }
    server_destroy(ctx);
    return st == RMPC_OK ? RMPC_OK : fail(st, msg);
}

}  // extern "C"
