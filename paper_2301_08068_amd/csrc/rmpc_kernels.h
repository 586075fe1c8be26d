// rmpc_kernels.h -- plain-data launch arguments shared by the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmpcast.h"

namespace rmpc {

// Steps (voxels or free cells) planned per lane and round of a single query by default
// (4, 8 or 16 are compiled; measured fastest for one 65536-ray query on gfx950).
constexpr int kLookahead = 8;

// Threads per block of the query kernels (one tile = this many lanes).
constexpr int kBlockThreads = 256;

// Block-partial slots of one reduction (one per block of a launch).
constexpr int kMaxPartialSlots = 4096;

// Words of one block partial in device memory: 18 floats + 4 integers, padded.
constexpr int kPartialWords = 32;

// Blocks of one scan query (each block's ticket costs a release/acquire, so the points are
// looped over instead of adding blocks).
constexpr int kScanMaxBlocks = 128;
constexpr int kScanBatch = 8;                // scan points a thread loads before it evaluates them

// A resident map: the voxel grid x-fastest (element offset x + nx (y + ny z)), then, at
// element offset cell_base, one summary element per cell of 8 x 8 x 8 voxels, also x-fastest:
// "occupied" when any voxel of the cell is, "free" when none is.  Only whole cells inside the
// grid have a summary (ncx = nx / 8 etc.); the walk skips free cells whole.
struct MapView {
    const void *data;
    int32_t nx, ny, nz, dtype;
    uint32_t cell_base;          // element offset of the cell summaries
    int32_t ncx, ncy, ncz;       // whole cells along each axis
    uint32_t brick_base;         // element offset of the brick summaries
    int32_t nbx, nby, nbz;       // whole bricks along each axis
};

// log2 of the edge, in voxels, of a summary cell and of a summary brick.
constexpr int kCellLog2 = 3;
constexpr int kBrickLog2 = 1;

// A sparse map: 8 x 8 x 8-voxel blocks stored where the world has content (every other voxel
// is free), found through an open-addressed hash table from block coordinates to slots.
constexpr int kBlockLog2 = 3;
constexpr int kBlockVoxels = 512;
// Block coordinates are signed 21-bit integers (|voxel coordinate| < 2^23 voxels).
constexpr int kBlockCoordBits = 21;
constexpr int32_t kBlockCoordBias = 1 << (kBlockCoordBits - 1);
constexpr uint64_t kEmptyKey = ~0ull;

// One table entry (16 bytes, one load): the packed block coordinates, the block's slot and
// whether any of its voxels is occupied.
struct alignas(16) HashEntry {
    uint64_t key;
    int32_t slot;
    uint32_t occupied;
};

// Key of block (bx, by, bz): the three biased 21-bit coordinates, x lowest.  Valid keys have
// bit 63 clear, so they never equal kEmptyKey.
__host__ __device__ inline uint64_t block_key(int32_t bx, int32_t by, int32_t bz)
{
    return (uint64_t)(uint32_t)(bx + kBlockCoordBias) | ((uint64_t)(uint32_t)(by + kBlockCoordBias) << 21) |
           ((uint64_t)(uint32_t)(bz + kBlockCoordBias) << 42);
}

// First table index of a key: the 64-bit finaliser of MurmurHash3 (fmix64), masked.
__host__ __device__ inline uint32_t block_hash(uint64_t k, uint32_t mask)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

struct SparseView {
    const HashEntry *table;      // table_mask + 1 entries (a power of two, at least twice the blocks)
    uint32_t table_mask;
    int32_t n_slots;
    const uint64_t *occ;         // per slot 8 words: word z holds bit x + 8 y of the block's layer z
    const void *values;          // per slot 512 elements, x fastest within the block
    int32_t dtype;
    int32_t pad;
    double free_value;           // TSDF maps: the field's value outside the stored blocks
};

// Policy constants in float32 (reciprocals precomputed on the host).
struct PolicyF {
    float vx, vy, vz;            // robot velocity
    float c, eta_rep, inv_nu_rep, eta_damp, inv_nu_damp, radius, inv_radius, eps;
};

// One entry of an ordered ray list: the float32 direction of Halton ray i and i itself, so
// that a lane gets its ray with one 16-byte load.
struct alignas(16) RayRec {
    float x, y, z;
    int32_t i;
};

// Everything one map query needs.
struct RayArgs {
    MapView map;                 // dense maps
    SparseView sp;               // sparse maps
    int32_t sparse;
    const RayRec *rays;          // ordered ray list; entries with i >= n_rays are skipped
    int32_t n_list;              // length of `rays` (>= n_rays)
    int32_t n_rays;
    float g[3];                  // start in grid units, float32((x - origin) / h)
    int32_t v0[3];               // start voxel floor(g)
    int32_t lin0;                // its logical index
    uint32_t start_flags;        // RMPC_RAY_START_FACE when g is within 1e-5 of a face
    float tmax_lo, tmax_hi;      // float32 guard band around max_range / h
    double tmax_v;               // parameter span split into segments: min(max_range / h, grid diagonal)
    int32_t segments;            // segments per ray (1, 2, 4, 8 or 16): a tile holds kBlock / segments rays
    int32_t lookahead;           // steps planned per round (4, 8 or 16)
    double max_range, h;
    int32_t subvoxel;            // non-zero: refine hit distances on the interpolated TSDF
    double vel64[3];             // velocity, float64 (for the exact contribution count)
    double radius64;
    PolicyF pol;
    double rank_tol;
    float *partials;             // per-block partial sums
    uint32_t *ticket;            // arrival counter, zero between launches
    rmpc_result *result;         // written by the last block
    uint64_t *done;              // host-visible completion word, set to seq after the result
    uint64_t seq;
    // debug outputs (trace kernel only)
    int32_t *dbg_hit;
    double *dbg_dist;
    uint8_t *dbg_flags;
    int32_t *dbg_visits;
};

// LiDAR scan query.
struct ScanArgs {
    const float *points;         // n x 3 float32
    int32_t n_points;
    double min_range2;           // squared minimum range, float64
    double vel64[3];
    double radius64;
    PolicyF pol;
    double rank_tol;
    float *partials;
    uint32_t *ticket;
    rmpc_result *result;         // host (pinned) or device memory
    uint64_t *done;              // host-visible completion word, or null (result left on the stream)
    uint64_t seq;
};

// One query of a batched launch.
struct BatchQuery {
    int32_t kind;                // 0: map query (ray), 1: scan query (scan)
    int32_t tile_begin;          // first tile of this query in the batch
    int32_t n_tiles;             // 256-lane tiles of this query
    int32_t pad;
    union {
        RayArgs ray;
        ScanArgs scan;
    };
};

// Per-launch header of a batch, in device memory (so a captured launch can be replayed).
struct BatchHeader {
    int32_t n_queries;
    int32_t n_tiles;
    uint64_t seq;
};

// Launch arguments of the persistent batch kernel (pointers only).
struct BatchArgs {
    const BatchHeader *hdr;
    const BatchQuery *__restrict__ q;
    uint32_t *work;              // [0] next tile, [1] blocks exited, [2] queries finished
    uint32_t *tickets;           // one per query
    float *partials;             // tile rows of all queries
    rmpc_result *results;        // one per query (pinned host memory)
    uint64_t *done;              // completion word, set to hdr->seq when all queries are done
};

constexpr int kBatchMaxQueries = 4096;
constexpr int kBatchMaxTiles = 262144;

struct DirsArgs {
    float *out;                  // structure of arrays with stride n
    int32_t n;
};

// Keep, in order, the entries of `order` (a permutation of 0..n_all-1) that are < n.
struct CompactArgs {
    const int32_t *order;
    int32_t n_all;
    int32_t n;
    int32_t *counts;             // n_all / 1024 per-chunk counts (scratch)
    int32_t *out;                // n entries
};

// out[k] = {dirs[idx[k]] (x, y, z from a structure of arrays with stride `stride`), idx[k]}.
struct GatherArgs {
    const int32_t *idx;
    int32_t n;
    const float *dirs;
    int32_t stride;
    RayRec *out;
};

struct SummaryArgs {
    MapView map;                 // grid in place; summaries are written at cell_base
};

int ray_grid_blocks(int n_rays);
int scan_grid_blocks(int n_points);
// When ev0/ev1 are non-null the kernel is launched with hipExtLaunchKernelGGL so the two
// events carry the dispatch's own start and end timestamps.
hipError_t launch_raycast(const RayArgs &a, hipStream_t s, bool debug, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
hipError_t launch_scan(const ScanArgs &a, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
hipError_t launch_directions(const DirsArgs &a, hipStream_t s);
hipError_t launch_map_summaries(const SummaryArgs &a, hipStream_t s);
hipError_t launch_compact(const CompactArgs &a, hipStream_t s);
hipError_t launch_gather(const GatherArgs &a, hipStream_t s);
// Exact squared Euclidean distance transform of the map's occupancy into out (x fastest).
hipError_t launch_edt(const MapView &m, int32_t *out, hipStream_t s);

// The single-lookup ESDF policy at one position.
struct EsdfArgs {
    const int32_t *sq;           // squared distance transform, x fastest
    int32_t nx, ny, nz;
    int32_t v0[3];               // the position's voxel
    double h;
    double vel[3];
    double c, eta_rep, nu_rep, eta_damp, nu_damp, radius, eps, rank_tol;
    rmpc_result *out;            // device memory
};
hipError_t launch_esdf(const EsdfArgs &a, hipStream_t s);
// One map query on a sparse map (debug: per-ray outputs instead of the policy).
hipError_t launch_sparse(const RayArgs &a, hipStream_t s, bool debug, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// Occupancy masks of n sparse blocks from their values, and the tables' occupied flags.
hipError_t launch_sparse_masks(const SparseView &v, HashEntry *table, hipStream_t s);
// Persistent fused batch: `blocks` resident blocks pull tiles from a counter.
hipError_t launch_batch(const BatchArgs &a, int blocks, int lookahead, hipStream_t s);
// Resident blocks per CU of the batch kernel for a lookahead.
int batch_blocks_per_cu(int lookahead);

}  // namespace rmpc
