// rmpc_host.h -- host-side internals shared by the C-ABI translation units: the context,
// the arena sub-allocator, resident maps, launch slots of the batched kernel, and helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "rmpcast.h"
#include "rmpc_kernels.h"
#include "rmpc_sched.h"

namespace rmpc_host {

// Records the calling thread's error message and returns st.
rmpc_status fail(rmpc_status st, const std::string &msg);
extern thread_local std::string g_last_error;

#define RMPC_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::rmpc_host::fail(RMPC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

using rmpc_sched::Arena;
using rmpc_sched::kAlign;

struct MapEntry {
    rmpc_map_desc desc;          // sparse maps: nx = ny = nz = 0
    rmpc::MapView view;          // dense maps
    size_t off;                  // first arena allocation (dense: the grid; sparse: the table)
    bool sparse = false;
    rmpc::SparseView sview;      // sparse maps
    std::vector<size_t> more;    // further arena allocations of a sparse map
};

// Everything one launch of the persistent batch kernel needs, on its own stream: device
// descriptors, tickets and partials, pinned staging for the descriptors, pinned results and
// completion word, and an optional captured graph of the launch.
struct LaunchSlot {
    int max_queries = 0, max_tiles = 0;
    rmpc::BatchHeader *hdr = nullptr;        // device
    rmpc::BatchQuery *q = nullptr;           // device
    uint32_t *work = nullptr;                // device
    uint32_t *tickets = nullptr;             // device
    float *partials = nullptr;               // device
    rmpc::BatchHeader *hdr_host = nullptr;   // pinned: the header, then (256 bytes on) q_host,
    rmpc::BatchQuery *q_host = nullptr;      //   as hdr and q lie on the device (one copy)
    rmpc_result *results_host = nullptr;     // pinned, written by the kernel
    uint64_t *done_host = nullptr;           // pinned completion word
    uint64_t seq = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_blocks = 0, graph_lookahead = 0;
    std::vector<size_t> arena_offsets;
};

// Runs a call with the context's device current, restoring the caller's afterwards.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

struct ServerState;

}  // namespace rmpc_host

struct rmpc_ctx {
    int device;
    uint8_t *arena;
    size_t arena_bytes;
    rmpc_host::Arena alloc;
    float *dirs;            // structure of arrays, RMPC_MAX_RAYS per component
    int32_t *order;         // all Halton indices in direction-coherent (Hilbert) order
    int32_t *counts;        // compaction scratch
    int32_t *list_tmp;      // compaction output before the gather into ray records
    // ordered ray lists for a ladder of list sizes (all built at creation): a query with N
    // rays walks the list of the smallest size >= N and skips entries >= N
    std::vector<int32_t> ladder;            // ascending sizes, last = RMPC_MAX_RAYS
    std::vector<const rmpc::RayRec *> ladder_lists;
    float *partials;
    uint32_t *ticket;
    rmpc_result *result_host;   // pinned, written by the kernels
    uint64_t *done_host;        // pinned completion word (sequence number of the last result)
    uint64_t seq;
    std::map<int32_t, rmpc_host::MapEntry> maps;
    int32_t next_map_id;
    rmpc_launch_config cfg[3];  // RMPC_CONFIG_QUERY, RMPC_CONFIG_BATCH, RMPC_CONFIG_SPARSE
    int cu_count;
    rmpc_host::LaunchSlot batch;          // rmpc_query_batch (allocated on first use)
    // streams of destroyed launch slots, kept for the next slots: a server that is stopped and
    // started again reuses them (creating streams again and again made a later server's first
    // copies under load wait ~8 ms for the runtime)
    std::vector<hipStream_t> stream_pool;
    hipEvent_t ev_dep;
    rmpc_host::ServerState *server;       // serving loop (rmpc_server_start)
    // kernel timing (rmpc_set_profiling)
    bool profiling;
    hipEvent_t ev0, ev1;
    double prof_ms;
    int64_t prof_n;
};

namespace rmpc_host {

bool finite3(const double *p);
rmpc_status check_params(const rmpc_params *p);
rmpc_status check_config(const rmpc_launch_config *c);
rmpc::PolicyF policy_f(const rmpc_params *p, const double v[3]);
// Grid coordinates of a world position, (x - origin) / voxel rounded to float32 per axis;
// false when one falls outside [0, n) (or is NaN).  The test every map query applies.
bool grid_coords(const rmpc_map_desc &d, const double x[3], float g[3]);
// Validate a map query and fill the geometry and policy-independent part of RayArgs; a query
// on a sparse map takes its segmentation from sparse_cfg when given, else from cfg.
rmpc_status setup_query(rmpc_ctx *ctx, int32_t map_id, const double x[3], int32_t n_rays,
                        const rmpc_params *params, const rmpc_launch_config &cfg, rmpc::RayArgs &A,
                        const rmpc_launch_config *sparse_cfg = nullptr);
// Whether a query at x on a sparse map keeps every voxel within tmax (voxel units) of its start
// inside the block coordinate range (|index| < 2^23 - 16), the test every sparse query applies.
bool sparse_position_ok(const rmpc_map_desc &d, const double x[3], double tmax);
// Largest scan query (points).
constexpr int32_t kMaxScanPoints = 1 << 24;
// Validate a scan query and fill ScanArgs except partials, ticket, result, done and seq.
rmpc_status setup_scan(const float *points_dev, int32_t n_points, const double v[3], const rmpc_params *params,
                       rmpc::ScanArgs &A);
// Spin until *done == seq (the kernel's publication), checking the stream for errors once the
// wait has lasted kStreamCheck, and once per kStreamCheck after that.
constexpr std::chrono::microseconds kStreamCheck(1000);
rmpc_status wait_done(const uint64_t *done, hipStream_t s, uint64_t seq);

// Launch slots of the batch kernel.
rmpc_status slot_create(rmpc_ctx *ctx, LaunchSlot &slot, int max_queries, int max_tiles);
void slot_destroy(rmpc_ctx *ctx, LaunchSlot &slot);
// Validate query k and fill its descriptor (tiles not yet placed).
rmpc_status batch_describe(rmpc_ctx *ctx, const rmpc_query_desc &d, int k, const rmpc_params *mp,
                           const rmpc_params *sp, const rmpc_launch_config &cfg, rmpc::BatchQuery &Q);
// Capture (or re-capture after a change of grid or lookahead) the slot's launch as a graph.
rmpc_status slot_graph(rmpc_ctx *ctx, LaunchSlot &slot, const rmpc_launch_config &cfg);
// Copy slot.q_host[0..nq) to the device and launch on the slot's stream after `after` (an
// event already recorded, or null).  Returns the launch's sequence number; non-blocking.
rmpc_status slot_launch(rmpc_ctx *ctx, LaunchSlot &slot, int nq, int n_tiles,
                        const rmpc_launch_config &cfg, hipEvent_t after, uint64_t *seq_out);

void server_destroy(rmpc_ctx *ctx);

}  // namespace rmpc_host
