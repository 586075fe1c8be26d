// batch.hip -- many queries in one persistent launch (rmpc_query_batch), the launch-config
// autotuner with its on-disk cache (rmpc_tune_batch), and the launch slots that the batch
// path and the serving loop share.  Host code, and one trivial kernel that starts a new stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "rmpc_host.h"

namespace rmpc_host {

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

namespace {

// Writes zero to a word that is zero already (the first work word of a new slot).
__global__ void stream_touch_kernel(uint32_t *w)
{
    if (threadIdx.x == 0) w[0] = 0u;
}

}  // namespace

// The header and the query descriptors of a launch sit in one block (the header padded to 256
// bytes), on the device and in pinned host memory, so that one copy sends both.
constexpr size_t kDescHead = 256;
static_assert(sizeof(rmpc::BatchHeader) <= kDescHead, "the header fits its 256 bytes");

rmpc_status slot_create(rmpc_ctx *ctx, LaunchSlot &slot, int max_queries, int max_tiles)
{
    slot = LaunchSlot();
    const size_t rows = (size_t)max_tiles;
    const size_t tk_bytes = sizeof(uint32_t) * (size_t)max_queries;
    const size_t desc_bytes = kDescHead + sizeof(rmpc::BatchQuery) * (size_t)max_queries;
    const size_t sizes[4] = {desc_bytes, 256, tk_bytes, sizeof(float) * rmpc::kPartialWords * rows};
    size_t off[4];
    for (int i = 0; i < 4; ++i) {
        if (!ctx->alloc.alloc(sizes[i], &off[i])) {
            for (size_t o : slot.arena_offsets) ctx->alloc.release(o);
            slot.arena_offsets.clear();
            return fail(RMPC_E_NOMEM, "arena too small for the batch buffers");
        }
        slot.arena_offsets.push_back(off[i]);
    }
    slot.max_queries = max_queries;
    slot.max_tiles = max_tiles;
    slot.hdr = reinterpret_cast<rmpc::BatchHeader *>(ctx->arena + off[0]);
    slot.q = reinterpret_cast<rmpc::BatchQuery *>(ctx->arena + off[0] + kDescHead);
    slot.work = reinterpret_cast<uint32_t *>(ctx->arena + off[1]);
    slot.tickets = reinterpret_cast<uint32_t *>(ctx->arena + off[2]);
    slot.partials = reinterpret_cast<float *>(ctx->arena + off[3]);
    RMPC_HIP(hipMemset(slot.work, 0, 256));
    RMPC_HIP(hipMemset(slot.tickets, 0, tk_bytes));
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&slot.results_host),
                           sizeof(rmpc_result) * (size_t)max_queries, hipHostMallocCoherent));
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&slot.done_host), 64, hipHostMallocCoherent));
    *slot.done_host = 0;
    uint8_t *desc_host = nullptr;
    RMPC_HIP(hipHostMalloc(reinterpret_cast<void **>(&desc_host), desc_bytes, 0));
    slot.hdr_host = reinterpret_cast<rmpc::BatchHeader *>(desc_host);
    slot.q_host = reinterpret_cast<rmpc::BatchQuery *>(desc_host + kDescHead);
    if (!ctx->stream_pool.empty()) {
        slot.stream = ctx->stream_pool.back();
        ctx->stream_pool.pop_back();
    } else {
        RMPC_HIP(hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking));
    }
    RMPC_HIP(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming));
    // a first kernel and first copies (the header alone and the whole descriptor block) on the
    // new stream, so that the runtime sets up its queues now and not under the first batches (a
    // serving slot's first launches would wait)
    std::memset(desc_host, 0, desc_bytes);
    RMPC_HIP(hipMemcpyAsync(slot.hdr, slot.hdr_host, sizeof(rmpc::BatchHeader), hipMemcpyHostToDevice, slot.stream));
    RMPC_HIP(hipMemcpyAsync(slot.hdr, desc_host, desc_bytes, hipMemcpyHostToDevice, slot.stream));
    stream_touch_kernel<<<1, 64, 0, slot.stream>>>(slot.work);
    RMPC_HIP(hipGetLastError());
    RMPC_HIP(hipStreamSynchronize(slot.stream));
    return RMPC_OK;
}

void slot_destroy(rmpc_ctx *ctx, LaunchSlot &slot)
{
    if (slot.stream) (void)hipStreamSynchronize(slot.stream);
    if (slot.graph) (void)hipGraphExecDestroy(slot.graph);
    if (slot.ev) (void)hipEventDestroy(slot.ev);
    if (slot.stream) ctx->stream_pool.push_back(slot.stream);
    if (slot.results_host) (void)hipHostFree(slot.results_host);
    if (slot.done_host) (void)hipHostFree(slot.done_host);
    if (slot.hdr_host) (void)hipHostFree(slot.hdr_host);      // the descriptor block (q_host lies in it)
    for (size_t o : slot.arena_offsets) ctx->alloc.release(o);
    slot = LaunchSlot();
}

rmpc_status batch_describe(rmpc_ctx *ctx, const rmpc_query_desc &d, int k, const rmpc_params *mp,
                           const rmpc_params *sp, const rmpc_launch_config &cfg, rmpc::BatchQuery &Q)
{
    const std::string where = "query " + std::to_string(k) + ": ";
    std::memset(&Q, 0, sizeof Q);
    if (d.kind == RMPC_KIND_MAP) {
        if (!finite3(d.v)) return fail(RMPC_E_INVALID, where + "velocity not finite");
        if (rmpc_status st = setup_query(ctx, d.map_id, d.x, d.n, mp, cfg, Q.ray)) {
            g_last_error = where + g_last_error;
            return st;
        }
        if (Q.ray.sparse && Q.ray.subvoxel)
            return fail(RMPC_E_INVALID, where + "subvoxel distances on sparse maps are queried one at a time (rmpc_query)");
        Q.kind = 0;
        Q.ray.pol = policy_f(mp, d.v);
        for (int a = 0; a < 3; ++a) Q.ray.vel64[a] = d.v[a];
        Q.n_tiles = (Q.ray.n_list * Q.ray.segments + rmpc::kBlockThreads - 1) / rmpc::kBlockThreads;
    } else if (d.kind == RMPC_KIND_SCAN) {
        if (!finite3(d.v)) return fail(RMPC_E_INVALID, where + "velocity not finite");
        if (d.n < 0 || d.n > kMaxScanPoints) return fail(RMPC_E_INVALID, where + "n_points out of [0, 2^24]");
        if (d.n > 0 && !d.points_dev) return fail(RMPC_E_INVALID, where + "points_dev is NULL");
        if (rmpc_status st = check_params(sp)) {
            g_last_error = where + g_last_error;
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
        return fail(RMPC_E_INVALID, where + "unknown kind");
    }
    return RMPC_OK;
}

namespace {

rmpc::BatchArgs slot_args(LaunchSlot &slot)
{
    rmpc::BatchArgs B;
    B.hdr = slot.hdr;
    B.q = slot.q;
    B.work = slot.work;
    B.tickets = slot.tickets;
    B.partials = slot.partials;
    B.results = slot.results_host;
    B.done = slot.done_host;
    return B;
}

int graph_blocks(rmpc_ctx *ctx, const rmpc_launch_config &cfg)
{
    const int per_cu = cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : rmpc::batch_blocks_per_cu(cfg.lookahead);
    return per_cu * ctx->cu_count;
}

}  // namespace

rmpc_status slot_graph(rmpc_ctx *ctx, LaunchSlot &slot, const rmpc_launch_config &cfg)
{
    const int gblocks = graph_blocks(ctx, cfg);
    if (slot.graph && slot.graph_blocks == gblocks && slot.graph_lookahead == cfg.lookahead) return RMPC_OK;
    // the grid is fixed (resident blocks) and the per-batch data sit in device memory, so one
    // captured launch serves every batch of this slot
    if (slot.graph) { RMPC_HIP(hipGraphExecDestroy(slot.graph)); slot.graph = nullptr; }
    hipStream_t s = slot.stream;
    hipGraph_t g;
    RMPC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hipError_t le = rmpc::launch_batch(slot_args(slot), gblocks, cfg.lookahead, s);
    const hipError_t ce = hipStreamEndCapture(s, &g);
    if (le != hipSuccess) return fail(RMPC_E_HIP, std::string("batch capture: ") + hipGetErrorString(le));
    if (ce != hipSuccess) return fail(RMPC_E_HIP, std::string("batch capture: ") + hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&slot.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(RMPC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    slot.graph_blocks = gblocks;
    slot.graph_lookahead = cfg.lookahead;
    return RMPC_OK;
}

rmpc_status slot_launch(rmpc_ctx *ctx, LaunchSlot &slot, int nq, int n_tiles,
                        const rmpc_launch_config &cfg, hipEvent_t after, uint64_t *seq_out)
{
    const uint64_t seq = ++slot.seq;
    slot.hdr_host->n_queries = nq;
    slot.hdr_host->n_tiles = n_tiles;
    slot.hdr_host->seq = seq;
    const int blocks = std::max(1, std::min(graph_blocks(ctx, cfg), n_tiles));
    const rmpc::BatchArgs B = slot_args(slot);
    hipStream_t s = slot.stream;
    if (cfg.use_graph) {
        if (rmpc_status st = slot_graph(ctx, slot, cfg)) return st;
    }
    if (after) RMPC_HIP(hipStreamWaitEvent(s, after, 0));
    // header and descriptors in one copy
    RMPC_HIP(hipMemcpyAsync(slot.hdr, slot.hdr_host, kDescHead + sizeof(rmpc::BatchQuery) * (size_t)nq,
                            hipMemcpyHostToDevice, s));
    if (cfg.use_graph) {
        RMPC_HIP(hipGraphLaunch(slot.graph, s));
    } else {
        RMPC_HIP(rmpc::launch_batch(B, blocks, cfg.lookahead, s));
    }
    *seq_out = seq;
    return RMPC_OK;
}

namespace {

// The batch path's slot, created on first use with the largest capacities.
rmpc_status batch_prepare(rmpc_ctx *ctx)
{
    if (ctx->batch.stream) return RMPC_OK;
    if (!ctx->ev_dep) RMPC_HIP(hipEventCreateWithFlags(&ctx->ev_dep, hipEventDisableTiming));
    rmpc_status st = slot_create(ctx, ctx->batch, rmpc::kBatchMaxQueries, rmpc::kBatchMaxTiles);
    if (st) slot_destroy(ctx, ctx->batch);
    return st;
}

// One blocking launch over the descriptors in ctx->batch.q_host[0 .. nq).
rmpc_status batch_launch(rmpc_ctx *ctx, int nq, int n_tiles, const rmpc_launch_config &cfg,
                         hipStream_t user, rmpc_result *out)
{
    LaunchSlot &slot = ctx->batch;
    // the launch runs on the slot's own stream, after the caller's stream's work
    RMPC_HIP(hipEventRecord(ctx->ev_dep, user));
    uint64_t seq = 0;
    if (rmpc_status st = slot_launch(ctx, slot, nq, n_tiles, cfg, ctx->ev_dep, &seq)) return st;
    if (rmpc_status st = wait_done(slot.done_host, slot.stream, seq)) return st;
    std::memcpy(out, slot.results_host, sizeof(rmpc_result) * (size_t)nq);
    // the caller's later work may reuse the point buffers: order it after this launch
    RMPC_HIP(hipEventRecord(slot.ev, slot.stream));
    RMPC_HIP(hipStreamWaitEvent(user, slot.ev, 0));
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
    LaunchSlot &slot = ctx->batch;
    int k0 = 0;
    while (k0 < n) {
        int nq = 0, tiles = 0;
        while (k0 + nq < n && nq < slot.max_queries && tiles + all[(size_t)(k0 + nq)].n_tiles <= slot.max_tiles) {
            rmpc::BatchQuery &Q = slot.q_host[nq];
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
}  // namespace rmpc_host

using namespace rmpc_host;

extern "C" {

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

}  // extern "C"
