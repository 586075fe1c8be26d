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

#include "rmpc_host.h"

namespace rmpc_host {

constexpr size_t kMinArena = 16u << 20;
constexpr int kMaxDim = 4096;
constexpr int32_t kMaxSparseBlocks = 1 << 22;   // slot * 512 + voxel fits int32

thread_local std::string g_last_error;

rmpc_status fail(rmpc_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

DeviceGuard::DeviceGuard(int dev)
{
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
}

DeviceGuard::~DeviceGuard()
{
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

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
void ray_list(const rmpc_ctx *ctx, int32_t n, const rmpc::RayRec **list, int32_t *list_len)
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

bool grid_coords(const rmpc_map_desc &d, const double x[3], float g[3])
{
    const int32_t n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        g[a] = (float)((x[a] - d.origin_m[a]) / d.voxel_m);
        if (!(g[a] >= 0.0f) || !(g[a] < (float)n[a])) return false;
    }
    return true;
}

bool sparse_position_ok(const rmpc_map_desc &d, const double x[3], double tmax)
{
    const double reach = (double)(1 << 23) - 16.0;
    for (int a = 0; a < 3; ++a) {
        const float g = (float)((x[a] - d.origin_m[a]) / d.voxel_m);
        if (!(std::fabs((double)g) + tmax < reach)) return false;
    }
    return true;
}

// A map query on a sparse map: the world has no edge, so the start only has to keep every
// voxel a ray can reach within the block coordinate range; segments per ray from the sparse
// launch configuration.
rmpc_status setup_sparse_query(rmpc_ctx *ctx, const MapEntry &me, const double x[3], int32_t n_rays,
                               const rmpc_params *params, const rmpc_launch_config &cfg, rmpc::RayArgs &A)
{
    std::memset(&A, 0, sizeof A);
    if (params->subvoxel && me.desc.dtype == RMPC_OCC_U8)
        return fail(RMPC_E_INVALID, "subvoxel distances need a TSDF map (float32 or float16)");
    const double tmax = params->max_range_m / me.desc.voxel_m;
    // every voxel within tmax of the start keeps |coordinate| < 2^23 (block coordinates in 21 bits)
    const double reach = (double)(1 << 23) - 16.0;
    if (!(tmax < reach)) return fail(RMPC_E_INVALID, "max_range_m spans too many voxels for a sparse map");
    if (!sparse_position_ok(me.desc, x, tmax))
        return fail(RMPC_E_OUT_OF_BOUNDS, "position too far from the sparse map's origin");
    uint32_t start_flags = 0;
    for (int a = 0; a < 3; ++a) {
        const float g = (float)((x[a] - me.desc.origin_m[a]) / me.desc.voxel_m);
        A.g[a] = g;
        A.v0[a] = (int32_t)std::floor(g);
        const double fr = (double)g - std::floor((double)g);
        if (fr < 1e-5 || 1.0 - fr < 1e-5) start_flags |= RMPC_RAY_START_FACE;
    }
    ray_list(ctx, n_rays, &A.rays, &A.n_list);
    A.sparse = 1;
    A.sp = me.sview;
    A.subvoxel = params->subvoxel != 0;
    A.n_rays = n_rays;
    A.start_flags = start_flags;
    A.tmax_lo = (float)(tmax * (1.0 - 1e-6) - 2e-5);
    A.tmax_hi = (float)(tmax * (1.0 + 1e-6) + 2e-5);
    A.tmax_v = tmax;
    A.segments = segments_for(n_rays, tmax, cfg.lane_target_log2);
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
    return RMPC_OK;
}

// Validates the query state and fills the geometry part of RayArgs.
rmpc_status setup_query(rmpc_ctx *ctx, int32_t map_id, const double x[3], int32_t n_rays,
                        const rmpc_params *params, const rmpc_launch_config &cfg, rmpc::RayArgs &A,
                        const rmpc_launch_config *sparse_cfg)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (!finite3(x)) return fail(RMPC_E_INVALID, "position is NULL or not finite");
    if (n_rays < 1 || n_rays > RMPC_MAX_RAYS) return fail(RMPC_E_INVALID, "n_rays out of [1, 65536]");
    if (rmpc_status st = check_params(params)) return st;
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    const MapEntry &me = it->second;
    if (me.sparse) return setup_sparse_query(ctx, me, x, n_rays, params, sparse_cfg ? *sparse_cfg : cfg, A);
    const int32_t n[3] = {me.desc.nx, me.desc.ny, me.desc.nz};
    std::memset(&A, 0, sizeof A);
    uint32_t start_flags = 0;
    float gc[3];
    if (!grid_coords(me.desc, x, gc)) return fail(RMPC_E_OUT_OF_BOUNDS, "position outside the grid");
    for (int a = 0; a < 3; ++a) {
        const float g = gc[a];
        A.g[a] = g;
        A.v0[a] = (int32_t)std::floor(g);
        const double fr = (double)g - std::floor((double)g);
        if (fr < 1e-5 || 1.0 - fr < 1e-5) start_flags |= RMPC_RAY_START_FACE;
    }
    if (params->subvoxel && me.desc.dtype == RMPC_OCC_U8)
        return fail(RMPC_E_INVALID, "subvoxel distances need a TSDF map (float32 or float16)");
    ray_list(ctx, n_rays, &A.rays, &A.n_list);
    A.map = me.view;
    A.subvoxel = params->subvoxel != 0;
    A.n_rays = n_rays;
    // below 2^31 for every accepted grid (rmpc_map_upload refuses larger ones)
    A.lin0 = (int32_t)((int64_t)A.v0[0] + (int64_t)n[0] * ((int64_t)A.v0[1] + (int64_t)n[1] * A.v0[2]));
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
    return RMPC_OK;
}

// Wait for a query's result: spin on the completion word the kernel sets after writing the
// result (a few microseconds sooner than a stream synchronisation).  The stream is checked for
// errors only once the wait has lasted kStreamCheck, and then once per kStreamCheck (measured:
// with a stream query every 1,024 spins a query whose kernel takes 20 us returned after 40 us;
// with none in its first millisecond, after 25 us).
rmpc_status wait_done(const uint64_t *done, hipStream_t s, uint64_t seq)
{
    using Clock = std::chrono::steady_clock;
    const auto t0 = Clock::now();
    auto next_check = t0 + kStreamCheck;
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(done, __ATOMIC_ACQUIRE) == seq) return RMPC_OK;
        if ((it & 255) == 0 && Clock::now() >= next_check) {
            next_check = Clock::now() + kStreamCheck;
            if (Clock::now() - t0 > std::chrono::seconds(60))
                return fail(RMPC_E_HIP, "query kernel did not finish within 60 s");
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (__atomic_load_n(done, __ATOMIC_ACQUIRE) == seq) return RMPC_OK;
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


// Validates a dense map's descriptor and lays it out: the grid, then one summary element per
// whole 8^3 cell and one per whole 2^3 brick, each at an offset rounded up to 256 elements.
// Linear voxel indices must fit int32 (the per-ray debug output and the query's start index are
// int32), and every element offset uint32.
rmpc_status dense_layout(const rmpc_map_desc &d, rmpc::MapView &v, uint64_t &n_all)
{
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || d.nx > kMaxDim || d.ny > kMaxDim || d.nz > kMaxDim)
        return fail(RMPC_E_INVALID, "grid dimensions out of [1, 4096]");
    if (d.dtype != RMPC_TSDF_F32 && d.dtype != RMPC_TSDF_F16 && d.dtype != RMPC_OCC_U8)
        return fail(RMPC_E_INVALID, "unknown dtype");
    if (!(d.voxel_m > 0) || !std::isfinite(d.voxel_m) || !finite3(d.origin_m))
        return fail(RMPC_E_INVALID, "voxel size or origin invalid");
    const uint64_t n_log = (uint64_t)d.nx * d.ny * d.nz;
    if (n_log >= (1ull << 31)) return fail(RMPC_E_INVALID, "grid has 2^31 voxels or more (linear indices are int32)");
    std::memset(&v, 0, sizeof v);
    v.nx = d.nx; v.ny = d.ny; v.nz = d.nz; v.dtype = d.dtype;
    v.ncx = d.nx >> rmpc::kCellLog2;
    v.ncy = d.ny >> rmpc::kCellLog2;
    v.ncz = d.nz >> rmpc::kCellLog2;
    v.nbx = d.nx >> rmpc::kBrickLog2;
    v.nby = d.ny >> rmpc::kBrickLog2;
    v.nbz = d.nz >> rmpc::kBrickLog2;
    const uint64_t cell_base = (n_log + 255) / 256 * 256;
    const uint64_t brick_base = (cell_base + (uint64_t)v.ncx * v.ncy * v.ncz + 255) / 256 * 256;
    n_all = brick_base + (uint64_t)v.nbx * v.nby * v.nbz;
    if (n_all >= (1ull << 32)) return fail(RMPC_E_INVALID, "grid too large for 32-bit voxel offsets");
    v.cell_base = (uint32_t)cell_base;
    v.brick_base = (uint32_t)brick_base;
    return RMPC_OK;
}

// Validates a scan query and fills everything of ScanArgs but its reduction slots.
rmpc_status setup_scan(const float *points_dev, int32_t n_points, const double v[3], const rmpc_params *params,
                       rmpc::ScanArgs &A)
{
    if (n_points < 0 || n_points > kMaxScanPoints) return fail(RMPC_E_INVALID, "n_points out of [0, 2^24]");
    if (n_points > 0 && !points_dev) return fail(RMPC_E_INVALID, "points_dev is NULL");
    if (!finite3(v)) return fail(RMPC_E_INVALID, "velocity is NULL or not finite");
    if (rmpc_status st = check_params(params)) return st;
    std::memset(&A, 0, sizeof A);
    A.points = points_dev;
    A.n_points = n_points;
    A.min_range2 = params->min_range_m * params->min_range_m;
    for (int a = 0; a < 3; ++a) A.vel64[a] = v[a];
    A.radius64 = params->radius;
    A.pol = policy_f(params, v);
    A.rank_tol = params->rank_tol;
    return RMPC_OK;
}

}  // namespace rmpc_host

using namespace rmpc_host;

extern "C" {

const char *rmpc_last_error(void) { return g_last_error.c_str(); }

rmpc_status rmpc_create(int device, void *arena_dev, size_t arena_bytes, rmpc_ctx **out)
{
    if (!out || !arena_dev) return fail(RMPC_E_INVALID, "NULL argument");
    if (arena_bytes < kMinArena) return fail(RMPC_E_INVALID, "arena smaller than 16 MiB");
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
    // sparse walks have no brick level and each block step probes the hash table, so slow rays
    // are longer and more lanes per ray pay; block rounds of 4 steps waste fewer table loads and
    // registers (a 160 m world at 65,536 rays, 4 lanes per ray: lookahead 4 134 us, 8 182 us,
    // 16 236 us; lookahead 8: 8 lanes per ray 186 us, 16 lanes 242 us)
    c->cfg[RMPC_CONFIG_SPARSE] = rmpc_launch_config{4, 18, 0, 0};
    c->ev_dep = nullptr;
    c->server = nullptr;
    c->cu_count = 0;
    c->profiling = false;
    c->ev0 = c->ev1 = nullptr;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    c->result_host = nullptr;
    c->done_host = nullptr;
    c->seq = 0;
    // every failure below ends here: work already queued on the null stream may still write
    // into the caller's arena, so it is waited for before the pinned buffers and the context go
    auto abandon = [c](rmpc_status st, const std::string &msg) {
        (void)hipStreamSynchronize(nullptr);
        if (c->result_host) (void)hipHostFree(c->result_host);
        if (c->done_host) (void)hipHostFree(c->done_host);
        delete c;
        return fail(st, msg);
    };
    if (hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->cu_count < 1)
        return abandon(RMPC_E_HIP, "cannot read the device's compute-unit count");
    size_t o_dirs, o_part, o_ticket, o_order, o_counts, o_tmp;
    if (!c->alloc.alloc(sizeof(float) * 3 * RMPC_MAX_RAYS, &o_dirs) ||
        !c->alloc.alloc(sizeof(int32_t) * RMPC_MAX_RAYS, &o_order) ||
        !c->alloc.alloc(sizeof(int32_t) * RMPC_MAX_RAYS, &o_tmp) ||
        !c->alloc.alloc(sizeof(int32_t) * 1024, &o_counts) ||
        !c->alloc.alloc(sizeof(float) * rmpc::kMaxPartialSlots * rmpc::kPartialWords, &o_part) ||
        !c->alloc.alloc(256, &o_ticket))
        return abandon(RMPC_E_NOMEM, "arena too small for the context tables");
    c->dirs = reinterpret_cast<float *>(c->arena + o_dirs);
    c->order = reinterpret_cast<int32_t *>(c->arena + o_order);
    c->counts = reinterpret_cast<int32_t *>(c->arena + o_counts);
    c->list_tmp = reinterpret_cast<int32_t *>(c->arena + o_tmp);
    c->partials = reinterpret_cast<float *>(c->arena + o_part);
    c->ticket = reinterpret_cast<uint32_t *>(c->arena + o_ticket);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c->result_host), sizeof(rmpc_result),
                                 hipHostMallocCoherent);
    if (e != hipSuccess) {
        c->result_host = nullptr;
        return abandon(RMPC_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    std::memset(c->result_host, 0, sizeof(rmpc_result));
    e = hipHostMalloc(reinterpret_cast<void **>(&c->done_host), 64, hipHostMallocCoherent);
    if (e != hipSuccess) {
        c->done_host = nullptr;
        return abandon(RMPC_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *c->done_host = 0;
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
        size_t off;
        if (!c->alloc.alloc(sizeof(rmpc::RayRec) * (size_t)n, &off))
            return abandon(RMPC_E_NOMEM, "arena too small for the ray lists");
        rmpc::RayRec *list = reinterpret_cast<rmpc::RayRec *>(c->arena + off);
        const int32_t *idx = c->order;
        if (n < RMPC_MAX_RAYS) {
            rmpc::CompactArgs ca{c->order, RMPC_MAX_RAYS, n, c->counts, c->list_tmp};
            e = rmpc::launch_compact(ca, nullptr);
            idx = c->list_tmp;
        }
        rmpc::GatherArgs ga{idx, n, c->dirs, RMPC_MAX_RAYS, list};
        if (e == hipSuccess) e = rmpc::launch_gather(ga, nullptr);
        c->ladder_lists.push_back(list);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return abandon(RMPC_E_HIP, std::string("context setup: ") + hipGetErrorString(e));
    *out = c;
    return RMPC_OK;
}

rmpc_status rmpc_destroy(rmpc_ctx *ctx)
{
    if (!ctx) return RMPC_OK;
    DeviceGuard dg(ctx->device);
    server_destroy(ctx);
    (void)hipDeviceSynchronize();
    slot_destroy(ctx, ctx->batch);
    for (hipStream_t st : ctx->stream_pool) (void)hipStreamDestroy(st);
    (void)hipHostFree(ctx->result_host);
    (void)hipHostFree(ctx->done_host);
    if (ctx->ev_dep) (void)hipEventDestroy(ctx->ev_dep);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return RMPC_OK;
}

rmpc_status rmpc_map_footprint(const rmpc_map_desc *desc, size_t *bytes)
{
    if (!desc || !bytes) return fail(RMPC_E_INVALID, "NULL argument");
    rmpc::MapView v;
    uint64_t n_all;
    if (rmpc_status st = dense_layout(*desc, v, n_all)) return st;
    *bytes = (size_t)(n_all * elem_bytes(desc->dtype));
    return RMPC_OK;
}

rmpc_status rmpc_map_upload(rmpc_ctx *ctx, const rmpc_map_desc *desc, const void *voxels,
                            int voxels_on_device, void *hip_stream, int32_t *map_id_out)
{
    if (!ctx || !desc || !voxels || !map_id_out) return fail(RMPC_E_INVALID, "NULL argument");
    if (ctx->server) return fail(RMPC_E_INVALID, "maps cannot change while the server runs");
    rmpc::MapView v;
    uint64_t n_all;
    if (rmpc_status st = dense_layout(*desc, v, n_all)) return st;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const uint64_t n_log = (uint64_t)desc->nx * desc->ny * desc->nz;
    const size_t eb = elem_bytes(desc->dtype);
    size_t off;
    if (!ctx->alloc.alloc(n_all * eb, &off)) return fail(RMPC_E_NOMEM, "arena full (map)");
    v.data = ctx->arena + off;
    // the grid is stored as given (x-fastest); the cell and brick summaries follow it
    hipError_t e = hipMemcpyAsync(ctx->arena + off, voxels, n_log * eb,
                                  voxels_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = rmpc::launch_map_summaries(rmpc::SummaryArgs{v}, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        ctx->alloc.release(off);
        return fail(RMPC_E_HIP, std::string("map upload: ") + hipGetErrorString(e));
    }
    const int32_t id = ctx->next_map_id++;
    MapEntry me;
    me.desc = *desc;
    me.view = v;
    me.off = off;
    ctx->maps[id] = me;
    *map_id_out = id;
    return RMPC_OK;
}

constexpr uint64_t kTableSlack = 16;       // block-table entries per stored block, at least

rmpc_status rmpc_sparse_map_upload(rmpc_ctx *ctx, const rmpc_sparse_desc *desc, const int32_t *block_coords_host,
                                   const void *values, int values_on_device, void *hip_stream, int32_t *map_id_out)
{
    if (!ctx || !desc || !block_coords_host || !values || !map_id_out) return fail(RMPC_E_INVALID, "NULL argument");
    if (ctx->server) return fail(RMPC_E_INVALID, "maps cannot change while the server runs");
    const int32_t n = desc->n_blocks;
    if (n < 1 || n > kMaxSparseBlocks) return fail(RMPC_E_INVALID, "n_blocks out of [1, 2^22]");
    if (desc->dtype != RMPC_TSDF_F32 && desc->dtype != RMPC_TSDF_F16 && desc->dtype != RMPC_OCC_U8)
        return fail(RMPC_E_INVALID, "unknown dtype");
    if (!(desc->voxel_m > 0) || !std::isfinite(desc->voxel_m) || !finite3(desc->origin_m))
        return fail(RMPC_E_INVALID, "voxel size or origin invalid");
    // the field outside the stored blocks, as a stored value of the map's type reads back
    double free_value = 0.0;
    if (desc->dtype == RMPC_TSDF_F32) free_value = (double)(float)desc->free_value;
    if (desc->dtype == RMPC_TSDF_F16) free_value = (double)(_Float16)desc->free_value;
    if (desc->dtype != RMPC_OCC_U8 && !(free_value > 0.0 && std::isfinite(free_value)))
        return fail(RMPC_E_INVALID, "free_value must be positive and finite in the map's storage type");
    // the table: a power of two of at least kTableSlack times the blocks, filled on the host by
    // linear probing.  Most lookups are of blocks that are not stored; at a load factor of 1/2
    // nearly half of them met another key at their first entry and probed on (a further
    // dependent load, and the end of a block round), at 1/16 few do
    uint64_t cap64 = 1024;
    while (cap64 < kTableSlack * (uint64_t)n) cap64 *= 2u;
    if (cap64 > (1ull << 31)) return fail(RMPC_E_INVALID, "too many blocks for the block table");
    const uint32_t cap = (uint32_t)cap64;
    std::vector<rmpc::HashEntry> table(cap, rmpc::HashEntry{rmpc::kEmptyKey, -1, 0u});
    const uint32_t mask = cap - 1u;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t *c = block_coords_host + 3 * (size_t)k;
        for (int a = 0; a < 3; ++a)
            if (c[a] < -rmpc::kBlockCoordBias || c[a] >= rmpc::kBlockCoordBias)
                return fail(RMPC_E_INVALID, "block " + std::to_string(k) + ": coordinate out of [-2^20, 2^20)");
        const uint64_t key = rmpc::block_key(c[0], c[1], c[2]);
        uint32_t i = rmpc::block_hash(key, mask);
        while (table[i].key != rmpc::kEmptyKey) {
            if (table[i].key == key) return fail(RMPC_E_INVALID, "block " + std::to_string(k) + ": listed twice");
            i = (i + 1u) & mask;
        }
        table[i] = rmpc::HashEntry{key, k, 0u};
    }
    const size_t eb = elem_bytes(desc->dtype);
    size_t o_table, o_occ, o_vals;
    if (!ctx->alloc.alloc(sizeof(rmpc::HashEntry) * (size_t)cap, &o_table))
        return fail(RMPC_E_NOMEM, "arena full (sparse map table)");
    if (!ctx->alloc.alloc(sizeof(uint64_t) * 8 * (size_t)n, &o_occ)) {
        ctx->alloc.release(o_table);
        return fail(RMPC_E_NOMEM, "arena full (sparse map occupancy)");
    }
    if (!ctx->alloc.alloc(eb * rmpc::kBlockVoxels * (size_t)n, &o_vals)) {
        ctx->alloc.release(o_table);
        ctx->alloc.release(o_occ);
        return fail(RMPC_E_NOMEM, "arena full (sparse map values)");
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rmpc::HashEntry *table_dev = reinterpret_cast<rmpc::HashEntry *>(ctx->arena + o_table);
    rmpc::SparseView v;
    std::memset(&v, 0, sizeof v);
    v.table = table_dev;
    v.table_mask = mask;
    v.n_slots = n;
    v.occ = reinterpret_cast<const uint64_t *>(ctx->arena + o_occ);
    v.values = ctx->arena + o_vals;
    v.dtype = desc->dtype;
    v.free_value = free_value;
    hipError_t e = hipMemcpyAsync(table_dev, table.data(), sizeof(rmpc::HashEntry) * (size_t)cap,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->arena + o_vals, values, eb * rmpc::kBlockVoxels * (size_t)n,
                           values_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = rmpc::launch_sparse_masks(v, table_dev, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        ctx->alloc.release(o_table);
        ctx->alloc.release(o_occ);
        ctx->alloc.release(o_vals);
        return fail(RMPC_E_HIP, std::string("sparse map upload: ") + hipGetErrorString(e));
    }
    MapEntry me;
    std::memset(&me.desc, 0, sizeof me.desc);
    me.desc.dtype = desc->dtype;
    me.desc.voxel_m = desc->voxel_m;
    for (int a = 0; a < 3; ++a) me.desc.origin_m[a] = desc->origin_m[a];
    std::memset(&me.view, 0, sizeof me.view);
    me.off = o_table;
    me.sparse = true;
    me.sview = v;
    me.more = {o_occ, o_vals};
    const int32_t id = ctx->next_map_id++;
    ctx->maps[id] = me;
    *map_id_out = id;
    return RMPC_OK;
}

rmpc_status rmpc_map_release(rmpc_ctx *ctx, int32_t map_id)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (ctx->server) return fail(RMPC_E_INVALID, "maps cannot change while the server runs");
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    DeviceGuard dg(ctx->device);
    RMPC_HIP(hipDeviceSynchronize());
    ctx->alloc.release(it->second.off);
    for (size_t o : it->second.more) ctx->alloc.release(o);
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
    if (rmpc_status st = setup_query(ctx, map_id, x, n_rays, params, ctx->cfg[RMPC_CONFIG_QUERY], A,
                                     &ctx->cfg[RMPC_CONFIG_SPARSE]))
        return st;
    A.seq = ++ctx->seq;
    A.pol = policy_f(params, v);
    for (int a = 0; a < 3; ++a) A.vel64[a] = v[a];
    if (A.sparse) RMPC_HIP(rmpc::launch_sparse(A, s, false, ctx->profiling ? ctx->ev0 : nullptr, ctx->ev1));
    else RMPC_HIP(rmpc::launch_raycast(A, s, false, ctx->profiling ? ctx->ev0 : nullptr, ctx->ev1));
    if (rmpc_status st = wait_done(ctx->done_host, s, A.seq)) return st;
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
    if (rmpc_status st = setup_query(ctx, map_id, x, n_rays, params, ctx->cfg[RMPC_CONFIG_QUERY], A,
                                     &ctx->cfg[RMPC_CONFIG_SPARSE]))
        return st;
    A.seq = ++ctx->seq;
    A.dbg_hit = hit_lin_dev;
    A.dbg_dist = dist_dev;
    A.dbg_flags = flags_dev;
    A.dbg_visits = visits_dev;
    if (A.sparse) RMPC_HIP(rmpc::launch_sparse(A, s, true));
    else RMPC_HIP(rmpc::launch_raycast(A, s, true));
    RMPC_HIP(hipStreamSynchronize(s));
    return RMPC_OK;
}

rmpc_status rmpc_scan_query(rmpc_ctx *ctx, const float *points_dev, int32_t n_points,
                            const double v[3], const rmpc_params *params, void *hip_stream,
                            rmpc_result *out)
{
    if (!ctx || !out) return fail(RMPC_E_INVALID, "NULL argument");
    rmpc::ScanArgs A;
    if (rmpc_status st = setup_scan(points_dev, n_points, v, params, A)) return st;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    A.partials = ctx->partials;
    A.ticket = ctx->ticket;
    A.result = ctx->result_host;
    A.done = ctx->done_host;
    A.seq = ++ctx->seq;
    RMPC_HIP(rmpc::launch_scan(A, s, ctx->profiling ? ctx->ev0 : nullptr, ctx->ev1));
    if (rmpc_status st = wait_done(ctx->done_host, s, A.seq)) return st;
    std::memcpy(out, ctx->result_host, sizeof(rmpc_result));
    if (ctx->profiling) RMPC_HIP(hipEventSynchronize(ctx->ev1));
    return account_profile(ctx);
}


rmpc_status rmpc_config_set(rmpc_ctx *ctx, int32_t which, const rmpc_launch_config *cfg)
{
    if (!ctx) return fail(RMPC_E_INVALID, "ctx is NULL");
    if (which != RMPC_CONFIG_QUERY && which != RMPC_CONFIG_BATCH && which != RMPC_CONFIG_SPARSE)
        return fail(RMPC_E_INVALID, "unknown config");
    if (rmpc_status st = check_config(cfg)) return st;
    ctx->cfg[which] = *cfg;
    return RMPC_OK;
}

rmpc_status rmpc_config_get(rmpc_ctx *ctx, int32_t which, rmpc_launch_config *cfg)
{
    if (!ctx || !cfg) return fail(RMPC_E_INVALID, "NULL argument");
    if (which != RMPC_CONFIG_QUERY && which != RMPC_CONFIG_BATCH && which != RMPC_CONFIG_SPARSE)
        return fail(RMPC_E_INVALID, "unknown config");
    *cfg = ctx->cfg[which];
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

rmpc_status rmpc_edt(rmpc_ctx *ctx, int32_t map_id, int32_t *sqdist_dev, void *hip_stream)
{
    if (!ctx || !sqdist_dev) return fail(RMPC_E_INVALID, "NULL argument");
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    if (it->second.sparse) return fail(RMPC_E_INVALID, "the distance transform needs a dense map");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RMPC_HIP(rmpc::launch_edt(it->second.view, sqdist_dev, s));
    RMPC_HIP(hipStreamSynchronize(s));
    return RMPC_OK;
}

rmpc_status rmpc_esdf_query(rmpc_ctx *ctx, int32_t map_id, const int32_t *sqdist_dev, const double x[3],
                            const double v[3], const rmpc_params *params, void *hip_stream, rmpc_result *out)
{
    if (!ctx || !sqdist_dev || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (!finite3(x) || !finite3(v)) return fail(RMPC_E_INVALID, "state is NULL or not finite");
    if (rmpc_status st = check_params(params)) return st;
    auto it = ctx->maps.find(map_id);
    if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, "unknown map id");
    if (it->second.sparse) return fail(RMPC_E_INVALID, "the ESDF policy needs a dense map");
    const rmpc_map_desc &d = it->second.desc;
    float g[3];
    if (!grid_coords(d, x, g)) return fail(RMPC_E_OUT_OF_BOUNDS, "position outside the grid");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rmpc::EsdfArgs A;
    std::memset(&A, 0, sizeof A);
    A.sq = sqdist_dev;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    for (int a = 0; a < 3; ++a) {
        A.v0[a] = (int32_t)std::floor(g[a]);
        A.vel[a] = v[a];
    }
    A.h = d.voxel_m;
    A.c = params->c;
    A.eta_rep = params->eta_rep;
    A.nu_rep = params->nu_rep;
    A.eta_damp = params->eta_damp;
    A.nu_damp = params->nu_damp;
    A.radius = params->radius;
    A.eps = params->eps;
    A.rank_tol = params->rank_tol;
    // the result goes through the context's partial-sum buffer (a query's scratch, idle here)
    A.out = reinterpret_cast<rmpc_result *>(ctx->partials);
    RMPC_HIP(rmpc::launch_esdf(A, s));
    RMPC_HIP(hipMemcpyAsync(out, A.out, sizeof(rmpc_result), hipMemcpyDeviceToHost, s));
    RMPC_HIP(hipStreamSynchronize(s));
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
