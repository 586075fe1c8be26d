// capi.hip -- the C ABI (include/rmpcast.h): context, caller-owned device arena, resident
// maps, argument validation and the blocking query calls.  Host code only; all per-ray
// work runs in the kernels of raycast.hip and setup_kernels.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <list>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "rmpcast.h"
#include "rmpc_kernels.h"

namespace {

thread_local std::string g_last_error;

rmpc_status fail(rmpc_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define RMPC_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(RMPC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kMinArena = 2u << 20;
constexpr int kMaxDim = 4096;

// First-fit sub-allocator over the caller's arena (offsets only; never touches memory).
class Arena {
  public:
    void init(size_t bytes) { free_.clear(); free_[0] = bytes; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_[*off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && start + len == nx->first) { len += nx->second; nx = free_.erase(nx); }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) { start = pv->first; len += pv->second; free_.erase(pv); }
        }
        free_[start] = len;
    }

  private:
    std::map<size_t, size_t> free_, used_;
};

struct MapEntry {
    rmpc_map_desc desc;
    rmpc::MapView view;
    size_t off;
};

}  // namespace

struct rmpc_ctx {
    int device;
    uint8_t *arena;
    size_t arena_bytes;
    Arena alloc;
    float *dirs;            // structure of arrays, RMPC_MAX_RAYS per component
    int32_t *order;         // all Halton indices in direction-coherent (Hilbert) order
    int32_t *counts;        // compaction scratch
    // ordered ray lists for a ladder of list sizes (all built at creation): a query with N
    // rays walks the list of the smallest size >= N and skips entries >= N
    std::vector<int32_t> ladder;            // ascending sizes, last = RMPC_MAX_RAYS
    std::vector<const int32_t *> ladder_lists;
    float *partials;
    uint32_t *ticket;
    rmpc_result *result_host;   // pinned, written by the kernels
    uint64_t *done_host;        // pinned completion word (sequence number of the last result)
    uint64_t seq;
    std::map<int32_t, MapEntry> maps;
    int32_t next_map_id;
    rmpc_launch_config cfg[2];  // RMPC_CONFIG_QUERY, RMPC_CONFIG_BATCH
    // batch state (allocated on first use)
    bool batch_ready;
    rmpc::BatchHeader *b_hdr;
    rmpc::BatchQuery *b_q;
    uint32_t *b_work;
    uint32_t *b_tickets;
    float *b_partials;
    rmpc_result *b_results_host;
    rmpc::BatchHeader *b_hdr_host;
    rmpc::BatchQuery *b_q_host;
    hipStream_t own_stream;
    hipEvent_t ev_dep;
    hipGraphExec_t graph_exec;
    int graph_blocks, graph_lookahead;
    int cu_count;
    // kernel timing (rmpc_set_profiling)
    bool profiling;
    hipEvent_t ev0, ev1;
    double prof_ms;
    int64_t prof_n;
};

namespace {

// Runs a call with the context's device current, restoring the caller's afterwards.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool finite3(const double *p) { return p && std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

rmpc_status check_params(const rmpc_params *p)
{
    if (!p) return fail(RMPC_E_INVALID, "params is NULL");
    const double vals[] = {p->c, p->eta_rep, p->nu_rep, p->eta_damp, p->nu_damp, p->radius,
                           p->eps, p->max_range_m, p->rank_tol, p->min_range_m};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(RMPC_E_INVALID, "non-finite policy parameter");
    if (!(p->c > 0 && p->nu_rep > 0 && p->nu_damp > 0 && p->radius > 0 && p->eps > 0 &&
          p->max_range_m > 0 && p->rank_tol >= 0 && p->min_range_m >= 0 && p->eta_rep >= 0 &&
          p->eta_damp >= 0))
        return fail(RMPC_E_INVALID, "policy parameter out of range");
    return RMPC_OK;
}

rmpc::PolicyF policy_f(const rmpc_params *p, const double v[3])
{
    rmpc::PolicyF P;
    P.vx = (float)v[0];
    P.vy = (float)v[1];
    P.vz = (float)v[2];
    P.c = (float)p->c;
    P.eta_rep = (float)p->eta_rep;
    P.inv_nu_rep = (float)(1.0 / p->nu_rep);
    P.eta_damp = (float)p->eta_damp;
    P.inv_nu_damp = (float)(1.0 / p->nu_damp);
    P.radius = (float)p->radius;
    P.inv_radius = (float)(1.0 / p->radius);
    P.eps = (float)p->eps;
    return P;
}

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Brick edge (log2) per axis for a storage type: about 128-256 bytes per brick.
void brick_shape(int dtype, int lb[3])
{
    lb[0] = lb[1] = lb[2] = 2;                      // 4 x 4 x 4
    if (dtype == RMPC_OCC_U8) lb[0] = 3;             // 8 x 4 x 4 bytes
    if (const char *e = std::getenv("RMPC_BRICK_LOG2")) {
        int a, b, c;
        if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a >= 0 && b >= 0 && c >= 0 &&
            a <= 4 && b <= 4 && c <= 4) {
            lb[0] = a; lb[1] = b; lb[2] = c;
        }
    }
}

size_t elem_bytes(int dtype) { return dtype == RMPC_TSDF_F32 ? 4 : (dtype == RMPC_TSDF_F16 ? 2 : 1); }

// Index of cell (x, y) along a Hilbert curve filling an n x n grid (n a power of two).
uint64_t hilbert_index(uint32_t n, uint32_t x, uint32_t y)
{
    uint64_t d = 0;
    for (uint32_t s = n / 2; s > 0; s /= 2) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        if (ry == 0) {                       // turn the quadrant so the curve stays connected
            if (rx == 1) { x = n - 1 - x; y = n - 1 - y; }
            std::swap(x, y);
        }
    }
    return d;
}

// Scheduling order of the ray table: directions folded onto the octahedron's square map and
// sorted along a 1024 x 1024 Hilbert curve, so consecutive rays point in nearby directions.
// Only the order in which rays are assigned to lanes depends on it, never a result bit
// beyond the summation order.
std::vector<int32_t> coherent_order(const std::vector<float> &soa, int n)
{
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    for (int i = 0; i < n; ++i) {
        const float x = soa[i], y = soa[i + n], z = soa[i + 2 * n];
        const float l1 = std::fabs(x) + std::fabs(y) + std::fabs(z);
        float px = x / l1, py = y / l1;
        if (z < 0.0f) {
            const float ox = (1.0f - std::fabs(py)) * (px >= 0.0f ? 1.0f : -1.0f);
            const float oy = (1.0f - std::fabs(px)) * (py >= 0.0f ? 1.0f : -1.0f);
            px = ox; py = oy;
        }
        const uint32_t qx = std::min<uint32_t>(1023u, (uint32_t)((px + 1.0f) * 512.0f));
        const uint32_t qy = std::min<uint32_t>(1023u, (uint32_t)((py + 1.0f) * 512.0f));
        key[i] = {hilbert_index(1024, qx, qy), i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[i] = key[i].second;
    return order;
}

// The ordered list used for n rays: the smallest ladder size >= n.
void ray_list(const rmpc_ctx *ctx, int32_t n, const int32_t **list, int32_t *list_len)
{
    const auto it = std::lower_bound(ctx->ladder.begin(), ctx->ladder.end(), n);
    const size_t k = (size_t)(it - ctx->ladder.begin());
    *list = ctx->ladder_lists[k];
    *list_len = ctx->ladder[k];
}

// List sizes 65536 * 2^(-k/8), rounded up, down to 1: consecutive sizes differ by at most
// 9 %, so a query never walks more than 9 % idle list entries.
std::vector<int32_t> list_ladder()
{
    std::vector<int32_t> v;
    for (int k = 0; k < 200; ++k) {
        const int32_t n = (int32_t)std::ceil(RMPC_MAX_RAYS * std::pow(2.0, -k / 8.0));
        if (v.empty() || n < v.back()) v.push_back(n);
        if (n == 1) break;
    }
    std::reverse(v.begin(), v.end());
    return v;
}

// Lanes per ray: enough segments that a query keeps about kLaneTarget lanes busy, each
// segment at least 4 voxels long, at most 16.
int segments_for(int32_t n_rays, double span, int lane_target_log2)
{
    const long target = 1l << lane_target_log2;
    int S = 1;
    while (S < 16 && (long)n_rays * S * 2 <= target && span / (2 * S) >= 4.0) S *= 2;
    return S;
}

// Validates the query state and fills the geometry part of RayArgs.
rmpc_status setup_query(rmpc_ctx *ctx, int32_t map_id, const double x[3], int32_t n_rays,
                        const rmpc_params *params, const rmpc_launch_config &cfg, rmpc::RayArgs &A,
                        const MapEntry **me_out)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (!finite3(x)) return fail(RMPC_E_INVALID, "position is NULL or not finite");
    if (n_rays < 1 || n_rays > RMPC_MAX_RAYS) return fail(RMPC_E_INVALID, "n_rays out of [1, 65536]");
    if (rmpc_status st = check_params(params)) return st;
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    const MapEntry &me = it->second;
    const int32_t n[3] = {me.desc.nx, me.desc.ny, me.desc.nz};
    std::memset(&A, 0, sizeof A);
    uint32_t start_flags = 0;
    for (int a = 0; a < 3; ++a) {
        const float g = (float)((x[a] - me.desc.origin_m[a]) / me.desc.voxel_m);
        if (!(g >= 0.0f) || !(g < (float)n[a])) return fail(RMPC_E_OUT_OF_BOUNDS, "position outside the grid");
        A.g[a] = g;
        A.v0[a] = (int32_t)std::floor(g);
        const double fr = (double)g - std::floor((double)g);
        if (fr < 1e-5 || 1.0 - fr < 1e-5) start_flags |= RMPC_RAY_START_FACE;
    }
    ray_list(ctx, n_rays, &A.rays, &A.n_list);
    A.map = me.view;
    A.dirs = ctx->dirs;
    A.dir_stride = RMPC_MAX_RAYS;
    A.n_rays = n_rays;
    A.lin0 = A.v0[0] + n[0] * (A.v0[1] + n[1] * A.v0[2]);
    A.start_flags = start_flags;
    const double tmax = params->max_range_m / me.desc.voxel_m;
    A.tmax_lo = (float)(tmax * (1.0 - 1e-6) - 2e-5);
    A.tmax_hi = (float)(tmax * (1.0 + 1e-6) + 2e-5);
    const double diag = std::sqrt((double)n[0] * n[0] + (double)n[1] * n[1] + (double)n[2] * n[2]) + 2.0;
    A.tmax_v = std::min(tmax, diag);
    A.segments = segments_for(n_rays, A.tmax_v, cfg.lane_target_log2);
    if ((long)A.n_list * A.segments > (long)rmpc::kMaxPartialSlots * 256)
        return fail(RMPC_E_INVALID, "too many lanes for one launch");
    A.lookahead = cfg.lookahead;
    A.max_range = params->max_range_m;
    A.h = me.desc.voxel_m;
    A.radius64 = params->radius;
    A.rank_tol = params->rank_tol;
    A.partials = ctx->partials;
    A.ticket = ctx->ticket;
    A.result = ctx->result_host;
    A.done = ctx->done_host;
    A.seq = 0;
    *me_out = &me;
    return RMPC_OK;
}

// Wait for a query's result: spin on the completion word the kernel sets after writing the
// result (a few microseconds sooner than a stream synchronisation), checking the stream for
// errors now and then.
rmpc_status wait_result(rmpc_ctx *ctx, hipStream_t s, uint64_t seq)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(ctx->done_host, __ATOMIC_ACQUIRE) == seq) return RMPC_OK;
        if ((it & 1023) == 0) {
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
                return fail(RMPC_E_HIP, "query kernel did not finish within 60 s");
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (__atomic_load_n(ctx->done_host, __ATOMIC_ACQUIRE) == seq) return RMPC_OK;
                return fail(RMPC_E_HIP, "kernel finished without publishing its result");
            }
            if (e != hipErrorNotReady) return fail(RMPC_E_HIP, std::string("query kernel: ") + hipGetErrorString(e));
        }
        __builtin_ia32_pause();
    }
}

// After a synchronised launch: add the dispatch's own duration to the profile.
rmpc_status account_profile(rmpc_ctx *ctx)
{
    if (!ctx->profiling) return RMPC_OK;
    float ms = 0.0f;
    RMPC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->prof_ms += ms;
    ctx->prof_n += 1;
    return RMPC_OK;
}


// ---------------------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------------------

rmpc_status check_config(const rmpc_launch_config *c)
{
    if (!c) return fail(RMPC_E_INVALID, "config is NULL");
    if (c->lookahead != 4 && c->lookahead != 8 && c->lookahead != 16)
        return fail(RMPC_E_INVALID, "lookahead must be 4, 8 or 16");
    if (c->lane_target_log2 < 10 || c->lane_target_log2 > 22)
        return fail(RMPC_E_INVALID, "lane_target_log2 out of [10, 22]");
    if (c->blocks_per_cu < 0 || c->blocks_per_cu > 64) return fail(RMPC_E_INVALID, "blocks_per_cu out of [0, 64]");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(RMPC_E_INVALID, "use_graph must be 0 or 1");
    return RMPC_OK;
}

// Device and pinned buffers of the batch path, allocated on first use.
rmpc_status batch_prepare(rmpc_ctx *ctx)
{
    if (ctx->batch_ready) return RMPC_OK;
    const size_t rows = (size_t)rmpc::kBatchMaxTiles + (size_t)rmpc::kGroups * rmpc::kBatchMaxQueries;
    size_t o_hdr, o_q, o_work, o_tk, o_part;
    if (!ctx->alloc.alloc(sizeof(rmpc::BatchHeader), &o_hdr) ||
        !ctx->alloc.alloc(sizeof(rmpc::BatchQuery) * rmpc::kBatchMaxQueries, &o_q) ||
        !ctx->alloc.alloc(256, &o_work) ||
        !ctx->alloc.alloc(sizeof(uint32_t) * (rmpc::kGroups + 1) * rmpc::kBatchMaxQueries, &o_tk) ||
        !ctx->alloc.alloc(sizeof(float) * 32 * rows, &o_part))
        return fail(RMPC_E_NOMEM, "arena too small for the batch buffers");
    ctx->b_hdr = reinterpret_cast<rmpc::BatchHeader *>(ctx->arena + o_hdr);
    ctx->b_q = reinterpret_cast<rmpc::BatchQuery *>(ctx->arena + o_q);
    ctx->b_work = reinterpret_cast<uint32_t *>(ctx->arena + o_work);
    ctx->b_tickets = reinterpret_cast<uint32_t *>(ctx->arena + o_tk);
    ctx->b_partials = reinterpret_cast<float *>(ctx->arena + o_part);
    RMPC_HIP(hipMemset(ctx->b_work, 0, 256));
    RMPC_HIP(hipMemset(ctx->b_tickets, 0, sizeof(uint32_t) * (rmpc::kGroups + 1) * rmpc::kBatchMaxQueries));
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->b_results_host),
                           sizeof(rmpc_result) * rmpc::kBatchMaxQueries, hipHostMallocCoherent));
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->b_hdr_host), sizeof(rmpc::BatchHeader), 0));
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->b_q_host),
                           sizeof(rmpc::BatchQuery) * rmpc::kBatchMaxQueries, 0));
    RMPC_HIP(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
    RMPC_HIP(hipEventCreateWithFlags(&ctx->ev_dep, hipEventDisableTiming));
    RMPC_HIP(hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, ctx->device));
    ctx->batch_ready = true;
    return RMPC_OK;
}

// Validate query k of a batch and fill its device descriptor (tiles not yet placed).
rmpc_status batch_describe(rmpc_ctx *ctx, const rmpc_query_desc &d, int k, const rmpc_params *mp,
                           const rmpc_params *sp, const rmpc_launch_config &cfg, rmpc::BatchQuery &Q)
{
    std::memset(&Q, 0, sizeof Q);
    if (d.kind == RMPC_KIND_MAP) {
        if (!finite3(d.v)) return fail(RMPC_E_INVALID, "query " + std::to_string(k) + ": velocity not finite");
        const MapEntry *me = nullptr;
        if (rmpc_status st = setup_query(ctx, d.map_id, d.x, d.n, mp, cfg, Q.ray, &me)) {
            g_last_error = "query " + std::to_string(k) + ": " + g_last_error;
            return st;
        }
        Q.kind = 0;
        Q.ray.pol = policy_f(mp, d.v);
        for (int a = 0; a < 3; ++a) Q.ray.vel64[a] = d.v[a];
        Q.n_tiles = (Q.ray.n_list * Q.ray.segments + rmpc::kBlockThreads - 1) / rmpc::kBlockThreads;
    } else if (d.kind == RMPC_KIND_SCAN) {
        if (!finite3(d.v)) return fail(RMPC_E_INVALID, "query " + std::to_string(k) + ": velocity not finite");
        if (d.n < 0 || d.n > (1 << 24)) return fail(RMPC_E_INVALID, "query " + std::to_string(k) + ": n_points out of [0, 2^24]");
        if (d.n > 0 && !d.points_dev) return fail(RMPC_E_INVALID, "query " + std::to_string(k) + ": points_dev is NULL");
        if (rmpc_status st = check_params(sp)) {
            g_last_error = "query " + std::to_string(k) + ": " + g_last_error;
            return st;
        }
        Q.kind = 1;
        rmpc::ScanArgs &A = Q.scan;
        A.points = d.points_dev;
        A.n_points = d.n;
        A.min_range2 = sp->min_range_m * sp->min_range_m;
        for (int a = 0; a < 3; ++a) A.vel64[a] = d.v[a];
        A.radius64 = sp->radius;
        A.pol = policy_f(sp, d.v);
        A.rank_tol = sp->rank_tol;
        Q.n_tiles = rmpc::scan_grid_blocks(d.n);
    } else {
        return fail(RMPC_E_INVALID, "query " + std::to_string(k) + ": unknown kind");
    }
    return RMPC_OK;
}

// One launch over queries [k0, k1) whose descriptors are in ctx->b_q_host[0 ..).
rmpc_status batch_launch(rmpc_ctx *ctx, int nq, int n_tiles, const rmpc_launch_config &cfg,
                         hipStream_t user, rmpc_result *out)
{
    const uint64_t seq = ++ctx->seq;
    ctx->b_hdr_host->n_queries = nq;
    ctx->b_hdr_host->n_tiles = n_tiles;
    ctx->b_hdr_host->seq = seq;
    const int per_cu = cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : rmpc::batch_blocks_per_cu(cfg.lookahead);
    const int blocks = std::max(1, std::min(per_cu * ctx->cu_count, n_tiles));
    rmpc::BatchArgs B;
    B.hdr = ctx->b_hdr;
    B.q = ctx->b_q;
    B.work = ctx->b_work;
    B.tickets = ctx->b_tickets;
    B.partials = ctx->b_partials;
    B.group_row_base = rmpc::kBatchMaxTiles;
    B.results = ctx->b_results_host;
    B.done = ctx->done_host;
    // the launch runs on the context's own stream, after the caller's stream's work
    hipStream_t s = ctx->own_stream;
    const int gblocks = per_cu * ctx->cu_count;
    if (cfg.use_graph &&
        (!ctx->graph_exec || ctx->graph_blocks != gblocks || ctx->graph_lookahead != cfg.lookahead)) {
        // the grid is fixed (resident blocks) and the per-batch data sit in device memory, so
        // one captured launch serves every batch
        if (ctx->graph_exec) { RMPC_HIP(hipGraphExecDestroy(ctx->graph_exec)); ctx->graph_exec = nullptr; }
        hipGraph_t g;
        RMPC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const hipError_t le = rmpc::launch_batch(B, gblocks, cfg.lookahead, s);
        const hipError_t ce = hipStreamEndCapture(s, &g);
        if (le != hipSuccess) return fail(RMPC_E_HIP, std::string("batch capture: ") + hipGetErrorString(le));
        if (ce != hipSuccess) return fail(RMPC_E_HIP, std::string("batch capture: ") + hipGetErrorString(ce));
        const hipError_t ie = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(RMPC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
        ctx->graph_blocks = gblocks;
        ctx->graph_lookahead = cfg.lookahead;
    }
    RMPC_HIP(hipEventRecord(ctx->ev_dep, user));
    RMPC_HIP(hipStreamWaitEvent(s, ctx->ev_dep, 0));
    RMPC_HIP(hipMemcpyAsync(ctx->b_hdr, ctx->b_hdr_host, sizeof(rmpc::BatchHeader), hipMemcpyHostToDevice, s));
    RMPC_HIP(hipMemcpyAsync(ctx->b_q, ctx->b_q_host, sizeof(rmpc::BatchQuery) * (size_t)nq,
                            hipMemcpyHostToDevice, s));
    if (cfg.use_graph) {
        RMPC_HIP(hipGraphLaunch(ctx->graph_exec, s));
    } else {
        RMPC_HIP(rmpc::launch_batch(B, blocks, cfg.lookahead, s));
    }
    if (rmpc_status st = wait_result(ctx, s, seq)) return st;
    std::memcpy(out, ctx->b_results_host, sizeof(rmpc_result) * (size_t)nq);
    // the caller's later work may reuse the point buffers: order it after this launch
    RMPC_HIP(hipEventRecord(ctx->ev_dep, s));
    RMPC_HIP(hipStreamWaitEvent(user, ctx->ev_dep, 0));
    return RMPC_OK;
}

rmpc_status run_batch(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n, const rmpc_params *mp,
                      const rmpc_params *sp, hipStream_t user, const rmpc_launch_config &cfg,
                      rmpc_result *out)
{
    if (rmpc_status st = batch_prepare(ctx)) return st;
    // validate everything before launching anything
    std::vector<rmpc::BatchQuery> all((size_t)n);
    for (int k = 0; k < n; ++k)
        if (rmpc_status st = batch_describe(ctx, q[k], k, mp, sp, cfg, all[(size_t)k])) return st;
    int k0 = 0;
    while (k0 < n) {
        int nq = 0, tiles = 0;
        while (k0 + nq < n && nq < rmpc::kBatchMaxQueries &&
               tiles + all[(size_t)(k0 + nq)].n_tiles <= rmpc::kBatchMaxTiles) {
            rmpc::BatchQuery &Q = ctx->b_q_host[nq];
            Q = all[(size_t)(k0 + nq)];
            Q.tile_begin = tiles;
            tiles += Q.n_tiles;
            ++nq;
        }
        if (nq == 0) return fail(RMPC_E_INVALID, "a query needs more tiles than one launch holds");
        if (rmpc_status st = batch_launch(ctx, nq, tiles, cfg, user, out + k0)) return st;
        k0 += nq;
    }
    return RMPC_OK;
}

// Cache key of a tuned configuration: architecture, storage types present, ray-count bucket.
std::string tune_key(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n)
{
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    bool dt[3] = {false, false, false};
    bool scan = false;
    double mean = 0.0;
    for (int k = 0; k < n; ++k) {
        if (q[k].kind == RMPC_KIND_SCAN) { scan = true; continue; }
        auto it = ctx->maps.find(q[k].map_id);
        if (it != ctx->maps.end()) dt[it->second.desc.dtype] = true;
        mean += q[k].n;
    }
    mean /= std::max(1, n);
    int bucket = 0;
    while ((1 << (bucket + 1)) <= mean) ++bucket;
    return arch + "|" + (dt[0] ? "f32" : "") + (dt[1] ? "f16" : "") + (dt[2] ? "u8" : "") +
           (scan ? "+scan" : "") + "|n2^" + std::to_string(bucket) + "|q" + std::to_string(n >= 64 ? 64 : n);
}

// Tiny JSON cache: one object of "key": [lookahead, lane_target_log2, blocks_per_cu].
bool cache_lookup(const char *path, const std::string &key, rmpc_launch_config *c)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    const std::string pat = "\"" + key + "\": [";
    const size_t at = text.find(pat);
    if (at == std::string::npos) return false;
    int a, b, d;
    if (std::sscanf(text.c_str() + at + pat.size(), "%d, %d, %d", &a, &b, &d) != 3) return false;
    c->lookahead = a;
    c->lane_target_log2 = b;
    c->blocks_per_cu = d;
    return check_config(c) == RMPC_OK;
}

void cache_store(const char *path, const std::string &key, const rmpc_launch_config &c)
{
    if (!path) return;
    std::vector<std::pair<std::string, std::string>> entries;
    if (FILE *f = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, f)) {
            const char *q1 = std::strchr(line, '"');
            if (!q1) continue;
            const char *q2 = std::strchr(q1 + 1, '"');
            const char *lb = q2 ? std::strchr(q2, '[') : nullptr;
            const char *rb = lb ? std::strchr(lb, ']') : nullptr;
            if (!rb) continue;
            entries.emplace_back(std::string(q1 + 1, q2), std::string(lb, rb + 1));
        }
        std::fclose(f);
    }
    const std::string val = "[" + std::to_string(c.lookahead) + ", " + std::to_string(c.lane_target_log2) +
                            ", " + std::to_string(c.blocks_per_cu) + "]";
    bool found = false;
    for (auto &e : entries)
        if (e.first == key) { e.second = val; found = true; }
    if (!found) entries.emplace_back(key, val);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i)
        std::fprintf(f, "  \"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                     i + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

const char *rmpc_last_error(void) { return g_last_error.c_str(); }

rmpc_status rmpc_create(int device, void *arena_dev, size_t arena_bytes, rmpc_ctx **out)
{
    if (!out || !arena_dev) return fail(RMPC_E_INVALID, "NULL argument");
    if (arena_bytes < kMinArena) return fail(RMPC_E_INVALID, "arena smaller than 2 MiB");
    int ndev = 0;
    RMPC_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(RMPC_E_INVALID, "no such device");
    DeviceGuard dg(device);
    hipPointerAttribute_t attr;
    RMPC_HIP(hipPointerGetAttributes(&attr, arena_dev));
    if (attr.type != hipMemoryTypeDevice || attr.device != device)
        return fail(RMPC_E_INVALID, "arena is not device memory of this GPU");
    rmpc_ctx *c = new rmpc_ctx();
    c->device = device;
    c->arena = static_cast<uint8_t *>(arena_dev);
    c->arena_bytes = arena_bytes;
    c->alloc.init(arena_bytes);
    c->next_map_id = 0;
    c->cfg[RMPC_CONFIG_QUERY] = rmpc_launch_config{rmpc::kLookahead, 17, 0, 0};
    c->cfg[RMPC_CONFIG_BATCH] = rmpc_launch_config{8, 14, 0, 0};
    c->batch_ready = false;
    c->own_stream = nullptr;
    c->ev_dep = nullptr;
    c->graph_exec = nullptr;
    c->graph_blocks = c->graph_lookahead = 0;
    c->cu_count = 0;
    c->profiling = false;
    c->ev0 = c->ev1 = nullptr;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    size_t o_dirs, o_part, o_ticket, o_order, o_counts;
    if (!c->alloc.alloc(sizeof(float) * 3 * RMPC_MAX_RAYS, &o_dirs) ||
        !c->alloc.alloc(sizeof(int32_t) * RMPC_MAX_RAYS, &o_order) ||
        !c->alloc.alloc(sizeof(int32_t) * 1024, &o_counts) ||
        !c->alloc.alloc(sizeof(float) * (rmpc::kMaxPartialSlots + 8) * 32, &o_part) ||
        !c->alloc.alloc(256, &o_ticket)) {
        delete c;
        return fail(RMPC_E_NOMEM, "arena too small for the context tables");
    }
    c->dirs = reinterpret_cast<float *>(c->arena + o_dirs);
    c->order = reinterpret_cast<int32_t *>(c->arena + o_order);
    c->counts = reinterpret_cast<int32_t *>(c->arena + o_counts);
    c->partials = reinterpret_cast<float *>(c->arena + o_part);
    c->ticket = reinterpret_cast<uint32_t *>(c->arena + o_ticket);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c->result_host), sizeof(rmpc_result),
                                 hipHostMallocCoherent);
    if (e != hipSuccess) {
        delete c;
        return fail(RMPC_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    std::memset(c->result_host, 0, sizeof(rmpc_result));
    e = hipHostMalloc(reinterpret_cast<void **>(&c->done_host), 64, hipHostMallocCoherent);
    if (e != hipSuccess) {
        (void)hipHostFree(c->result_host);
        delete c;
        return fail(RMPC_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *c->done_host = 0;
    c->seq = 0;
    rmpc::DirsArgs da{c->dirs, RMPC_MAX_RAYS};
    e = hipMemsetAsync(c->ticket, 0, 256, nullptr);
    if (e == hipSuccess) e = rmpc::launch_directions(da, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) {
        std::vector<float> soa(3 * (size_t)RMPC_MAX_RAYS);
        e = hipMemcpy(soa.data(), c->dirs, sizeof(float) * soa.size(), hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            const std::vector<int32_t> order = coherent_order(soa, RMPC_MAX_RAYS);
            e = hipMemcpy(c->order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
        }
    }
    c->ladder = list_ladder();
    for (size_t k = 0; k < c->ladder.size() && e == hipSuccess; ++k) {
        const int32_t n = c->ladder[k];
        if (n == RMPC_MAX_RAYS) { c->ladder_lists.push_back(c->order); continue; }
        size_t off;
        if (!c->alloc.alloc(sizeof(int32_t) * (size_t)n, &off)) {
            (void)hipHostFree(c->result_host);
            (void)hipHostFree(c->done_host);
            delete c;
            return fail(RMPC_E_NOMEM, "arena too small for the ray lists");
        }
        int32_t *list = reinterpret_cast<int32_t *>(c->arena + off);
        rmpc::CompactArgs ca{c->order, RMPC_MAX_RAYS, n, c->counts, list};
        e = rmpc::launch_compact(ca, nullptr);
        c->ladder_lists.push_back(list);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipHostFree(c->result_host);
        delete c;
        return fail(RMPC_E_HIP, std::string("context setup: ") + hipGetErrorString(e));
    }
    *out = c;
    return RMPC_OK;
}

rmpc_status rmpc_destroy(rmpc_ctx *ctx)
{
    if (!ctx) return RMPC_OK;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipHostFree(ctx->result_host);
    (void)hipHostFree(ctx->done_host);
    if (ctx->batch_ready) {
        (void)hipHostFree(ctx->b_results_host);
        (void)hipHostFree(ctx->b_hdr_host);
        (void)hipHostFree(ctx->b_q_host);
    }
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->ev_dep) (void)hipEventDestroy(ctx->ev_dep);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return RMPC_OK;
}

rmpc_status rmpc_map_upload(rmpc_ctx *ctx, const rmpc_map_desc *desc, const void *voxels,
                            int voxels_on_device, void *hip_stream, int32_t *map_id_out)
{
    if (!ctx || !desc || !voxels || !map_id_out) return fail(RMPC_E_INVALID, "NULL argument");
    if (desc->nx < 1 || desc->ny < 1 || desc->nz < 1 || desc->nx > kMaxDim || desc->ny > kMaxDim ||
        desc->nz > kMaxDim)
        return fail(RMPC_E_INVALID, "grid dimensions out of [1, 4096]");
    if (desc->dtype != RMPC_TSDF_F32 && desc->dtype != RMPC_TSDF_F16 && desc->dtype != RMPC_OCC_U8)
        return fail(RMPC_E_INVALID, "unknown dtype");
    if (!(desc->voxel_m > 0) || !std::isfinite(desc->voxel_m) || !finite3(desc->origin_m))
        return fail(RMPC_E_INVALID, "voxel size or origin invalid");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int lb[3];
    brick_shape(desc->dtype, lb);
    rmpc::MapView v;
    std::memset(&v, 0, sizeof v);
    v.nx = desc->nx; v.ny = desc->ny; v.nz = desc->nz; v.dtype = desc->dtype;
    v.lbx = lb[0]; v.lby = lb[1]; v.lbz = lb[2];
    v.nbx = (desc->nx + (1 << lb[0]) - 1) >> lb[0];
    v.nby = (desc->ny + (1 << lb[1]) - 1) >> lb[1];
    v.nbz = (desc->nz + (1 << lb[2]) - 1) >> lb[2];
    const uint64_t n_dst = (uint64_t)v.nbx * v.nby * v.nbz << (lb[0] + lb[1] + lb[2]);
    if (n_dst >= (1ull << 32)) return fail(RMPC_E_INVALID, "grid too large for 32-bit voxel offsets");
    const size_t eb = elem_bytes(desc->dtype);
    size_t off;
    if (!ctx->alloc.alloc(n_dst * eb, &off)) return fail(RMPC_E_NOMEM, "arena full (map)");
    v.data = ctx->arena + off;
    const size_t n_log = (size_t)desc->nx * desc->ny * desc->nz;
    const void *src = voxels;
    size_t tmp_off = 0;
    bool tmp = false;
    if (!voxels_on_device) {
        if (!ctx->alloc.alloc(n_log * eb, &tmp_off)) {
            ctx->alloc.release(off);
            return fail(RMPC_E_NOMEM, "arena full (upload staging)");
        }
        tmp = true;
        hipError_t e = hipMemcpyAsync(ctx->arena + tmp_off, voxels, n_log * eb, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            ctx->alloc.release(off);
            ctx->alloc.release(tmp_off);
            return fail(RMPC_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        }
        src = ctx->arena + tmp_off;
    }
    rmpc::LayoutArgs la{src, v, (int32_t)eb, n_dst};
    hipError_t e = rmpc::launch_layout(la, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tmp) ctx->alloc.release(tmp_off);
    if (e != hipSuccess) {
        ctx->alloc.release(off);
        return fail(RMPC_E_HIP, std::string("map layout: ") + hipGetErrorString(e));
    }
    const int32_t id = ctx->next_map_id++;
    ctx->maps[id] = MapEntry{*desc, v, off};
    *map_id_out = id;
    return RMPC_OK;
}

rmpc_status rmpc_map_release(rmpc_ctx *ctx, int32_t map_id)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    DeviceGuard dg(ctx->device);
    RMPC_HIP(hipDeviceSynchronize());
    ctx->alloc.release(it->second.off);
    ctx->maps.erase(it);
    return RMPC_OK;
}

rmpc_status rmpc_query(rmpc_ctx *ctx, int32_t map_id, const double x[3], const double v[3],
                       int32_t n_rays, const rmpc_params *params, void *hip_stream,
                       rmpc_result *out)
{
    if (!out) return fail(RMPC_E_INVALID, "out is NULL");
    if (!finite3(v)) return fail(RMPC_E_INVALID, "velocity is NULL or not finite");
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rmpc::RayArgs A;
    const MapEntry *me = nullptr;
    if (rmpc_status st = setup_query(ctx, map_id, x, n_rays, params, ctx->cfg[RMPC_CONFIG_QUERY], A, &me))
        return st;
    A.seq = ++ctx->seq;
    A.pol = policy_f(params, v);
    for (int a = 0; a < 3; ++a) A.vel64[a] = v[a];
    RMPC_HIP(rmpc::launch_raycast(A, s, false, ctx->profiling ? ctx->ev0 : nullptr, ctx->ev1));
    if (rmpc_status st = wait_result(ctx, s, A.seq)) return st;
    std::memcpy(out, ctx->result_host, sizeof(rmpc_result));
    if (ctx->profiling) RMPC_HIP(hipEventSynchronize(ctx->ev1));
    return account_profile(ctx);
}

rmpc_status rmpc_trace_debug(rmpc_ctx *ctx, int32_t map_id, const double x[3], int32_t n_rays,
                             const rmpc_params *params, void *hip_stream, int32_t *hit_lin_dev,
                             double *dist_dev, uint8_t *flags_dev, int32_t *visits_dev)
{
    if (!hit_lin_dev || !dist_dev || !flags_dev) return fail(RMPC_E_INVALID, "NULL output");
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rmpc::RayArgs A;
    const MapEntry *me = nullptr;
    if (rmpc_status st = setup_query(ctx, map_id, x, n_rays, params, ctx->cfg[RMPC_CONFIG_QUERY], A, &me))
        return st;
    A.seq = ++ctx->seq;
    A.dbg_hit = hit_lin_dev;
    A.dbg_dist = dist_dev;
    A.dbg_flags = flags_dev;
    A.dbg_visits = visits_dev;
    RMPC_HIP(rmpc::launch_raycast(A, s, true));
    RMPC_HIP(hipStreamSynchronize(s));
    return RMPC_OK;
}

rmpc_status rmpc_scan_query(rmpc_ctx *ctx, const float *points_dev, int32_t n_points,
                            const double v[3], const rmpc_params *params, void *hip_stream,
                            rmpc_result *out)
{
    if (!ctx || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (n_points < 0 || n_points > (1 << 24)) return fail(RMPC_E_INVALID, "n_points out of [0, 2^24]");
    if (n_points > 0 && !points_dev) return fail(RMPC_E_INVALID, "points_dev is NULL");
    if (!finite3(v)) return fail(RMPC_E_INVALID, "velocity is NULL or not finite");
    if (rmpc_status st = check_params(params)) return st;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rmpc::ScanArgs A;
    std::memset(&A, 0, sizeof A);
    A.points = points_dev;
    A.n_points = n_points;
    A.min_range2 = params->min_range_m * params->min_range_m;
    for (int a = 0; a < 3; ++a) A.vel64[a] = v[a];
    A.radius64 = params->radius;
    A.pol = policy_f(params, v);
    A.rank_tol = params->rank_tol;
    A.partials = ctx->partials;
    A.ticket = ctx->ticket;
    A.result = ctx->result_host;
    A.done = ctx->done_host;
    A.seq = ++ctx->seq;
    RMPC_HIP(rmpc::launch_scan(A, s, ctx->profiling ? ctx->ev0 : nullptr, ctx->ev1));
    if (rmpc_status st = wait_result(ctx, s, A.seq)) return st;
    std::memcpy(out, ctx->result_host, sizeof(rmpc_result));
    if (ctx->profiling) RMPC_HIP(hipEventSynchronize(ctx->ev1));
    return account_profile(ctx);
}


rmpc_status rmpc_config_set(rmpc_ctx *ctx, int32_t which, const rmpc_launch_config *cfg)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (which != RMPC_CONFIG_QUERY && which != RMPC_CONFIG_BATCH) return fail(RMPC_E_INVALID, "unknown config");
    if (rmpc_status st = check_config(cfg)) return st;
    ctx->cfg[which] = *cfg;
    return RMPC_OK;
}

rmpc_status rmpc_config_get(rmpc_ctx *ctx, int32_t which, rmpc_launch_config *cfg)
{
    if (!ctx || !cfg) return fail(RMPC_E_INVALID, "NULL argument");
    if (which != RMPC_CONFIG_QUERY && which != RMPC_CONFIG_BATCH) return fail(RMPC_E_INVALID, "unknown config");
    *cfg = ctx->cfg[which];
    return RMPC_OK;
}

rmpc_status rmpc_query_batch(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n,
                             const rmpc_params *map_params, const rmpc_params *scan_params,
                             void *hip_stream, rmpc_result *out)
{
    if (!ctx || !q || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (n < 1) return fail(RMPC_E_INVALID, "n must be >= 1");
    DeviceGuard dg(ctx->device);
    return run_batch(ctx, q, n, map_params, scan_params, static_cast<hipStream_t>(hip_stream),
                     ctx->cfg[RMPC_CONFIG_BATCH], out);
}

rmpc_status rmpc_tune_batch(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n,
                            const rmpc_params *map_params, const rmpc_params *scan_params,
                            void *hip_stream, const char *cache_path, rmpc_launch_config *best)
{
    if (!ctx || !q) return fail(RMPC_E_INVALID, "NULL argument");
    if (n < 1) return fail(RMPC_E_INVALID, "n must be >= 1");
    DeviceGuard dg(ctx->device);
    hipStream_t user = static_cast<hipStream_t>(hip_stream);
    const std::string key = tune_key(ctx, q, n);
    rmpc_launch_config chosen = ctx->cfg[RMPC_CONFIG_BATCH];
    if (!cache_lookup(cache_path, key, &chosen)) {
        std::vector<rmpc_result> res((size_t)n);
        double best_ms = 1e30;
        const int max_per_cu = std::max(1, rmpc::batch_blocks_per_cu(8));
        for (int la : {4, 8, 16})
            for (int lt : {12, 14, 16, 18})
                for (int bpc : {0, std::max(1, max_per_cu / 2)}) {
                    rmpc_launch_config c{la, lt, bpc, 0};
                    if (rmpc_status st = run_batch(ctx, q, n, map_params, scan_params, user, c, res.data()))
                        return st;                                   // warm-up (and validation)
                    const auto t0 = std::chrono::steady_clock::now();
                    for (int r = 0; r < 3; ++r)
                        if (rmpc_status st = run_batch(ctx, q, n, map_params, scan_params, user, c, res.data()))
                            return st;
                    const double ms = std::chrono::duration<double, std::milli>(
                                          std::chrono::steady_clock::now() - t0).count() / 3.0;
                    if (ms < best_ms) { best_ms = ms; chosen = c; }
                }
        cache_store(cache_path, key, chosen);
    }
    chosen.use_graph = ctx->cfg[RMPC_CONFIG_BATCH].use_graph;
    ctx->cfg[RMPC_CONFIG_BATCH] = chosen;
    if (best) *best = chosen;
    return RMPC_OK;
}

rmpc_status rmpc_set_profiling(rmpc_ctx *ctx, int enable)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (enable && !ctx->ev0) {
        RMPC_HIP(hipEventCreate(&ctx->ev0));
        RMPC_HIP(hipEventCreate(&ctx->ev1));
    }
    ctx->profiling = enable != 0;
    ctx->prof_ms = 0.0;
    ctx->prof_n = 0;
    return RMPC_OK;
}

rmpc_status rmpc_get_profile(rmpc_ctx *ctx, double *kernel_ms, int64_t *launches)
{
    if (!ctx || !kernel_ms || !launches) return fail(RMPC_E_INVALID, "NULL argument");
    *kernel_ms = ctx->prof_ms;
    *launches = ctx->prof_n;
    return RMPC_OK;
}

rmpc_status rmpc_directions(rmpc_ctx *ctx, int32_t n, float *out_host)
{
    if (!ctx || !out_host) return fail(RMPC_E_INVALID, "NULL argument");
    if (n < 1 || n > RMPC_MAX_RAYS) return fail(RMPC_E_INVALID, "n out of [1, 65536]");
    DeviceGuard dg(ctx->device);
    float *tmp = static_cast<float *>(std::malloc(sizeof(float) * 3 * (size_t)n));
    if (!tmp) return fail(RMPC_E_NOMEM, "host allocation failed");
    hipError_t e = hipSuccess;
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
        e = hipMemcpy(tmp + (size_t)a * n, ctx->dirs + (size_t)a * RMPC_MAX_RAYS, sizeof(float) * n,
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        std::free(tmp);
        return fail(RMPC_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    for (int32_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) out_host[3 * (size_t)i + a] = tmp[(size_t)a * n + i];
    std::free(tmp);
    return RMPC_OK;
}

}  // extern "C"
