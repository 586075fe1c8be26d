// rmpc_sparse.h -- the walk over a sparse block map (Sec. III-E/F: the map is a GPU hash of
// 8^3-voxel blocks allocated where the world has content; every voxel outside an allocated
// block is free, and the world has no edge), shared by the single-query kernel (sparse.hip)
// and the batch kernel (raycast.hip).
//
// S adjacent lanes walk the S segments of one ray (as in the dense kernel: segment k starts
// at the voxel that holds the float64-located boundary near k max_range / S and ends at the
// next one; the lowest segment with a hit owns the ray) with the exact 3-D DDA of the dense
// kernels (float32 crossing parameters, float64 decisions inside the guard band, the hit
// distance from the entered face in float64), at two levels:
//   block level: the walk steps block by block (block faces are voxel faces, so it enters the
//     blocks the voxel walk enters, in the same order).  A round plans K block steps and issues
//     the K hash-table loads at once; the first planned block that is allocated and holds an
//     occupied voxel is entered at its entry voxel (found as for a dense cell).
//   voxel level: inside a block the walk tests the block's 512-bit occupancy mask, held in
//     registers, so a voxel step reads no memory; leaving the block it looks the next block up
//     and goes back to the block level when that block is free.
// Near max_range the current free block is finished at the voxel level, so the last voxel and
// the range decision are those of the voxel walk.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"
#include "rmpc_walk.h"

namespace rmpc {

namespace {

constexpr int kLayers = 8;                      // occupancy words per block (one per z layer)

// A table entry in registers (plain words: HIP's vector types keep arrays of them in private
// memory).
struct Entry {
    uint64_t key;
    uint32_t slot, occ;
};

__device__ __forceinline__ Entry load_entry(const HashEntry *t, uint32_t i)
{
    const uint4 q = reinterpret_cast<const uint4 *>(t)[i];
    Entry e;
    e.key = (uint64_t)q.x | ((uint64_t)q.y << 32);
    e.slot = q.z;
    e.occ = q.w;
    return e;
}

// Slot and occupied flag of block (bx, by, bz) by linear probing from its first entry e0 (at
// index i0, already loaded); slot -1 when the block is not allocated.  The table always has
// empty entries, so the probe ends; the bound only guards against a damaged table.
__device__ __forceinline__ void probe_from(const SparseView &S, uint64_t key, uint32_t i0, Entry e0, int &slot,
                                           bool &occ)
{
    uint32_t i = i0;
    Entry e = e0;
    for (uint32_t n = 0; n <= S.table_mask; ++n) {
        const uint64_t k = e.key;
        if (k == key) {
            slot = (int)e.slot;
            occ = e.occ != 0u;
            return;
        }
        if (k == kEmptyKey) break;
        i = (i + 1u) & S.table_mask;
        e = load_entry(S.table, i);
    }
    slot = -1;
    occ = false;
}

__device__ __forceinline__ void lookup(const SparseView &S, int bx, int by, int bz, int &slot, bool &occ)
{
    const uint64_t key = block_key(bx, by, bz);
    const uint32_t i = block_hash(key, S.table_mask);
    probe_from(S, key, i, load_entry(S.table, i), slot, occ);
}

// The 8 occupancy words of a slot (zeros for slot < 0).
__device__ __forceinline__ void load_mask(const SparseView &S, int slot, uint64_t (&m)[kLayers])
{
    if (slot < 0) {
#pragma unroll
        for (int k = 0; k < kLayers; ++k) m[k] = 0;
        return;
    }
    const uint4 *p = reinterpret_cast<const uint4 *>(S.occ + (size_t)slot * kLayers);
#pragma unroll
    for (int k = 0; k < kLayers / 2; ++k) {
        const uint4 q = p[k];
        m[2 * k] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        m[2 * k + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
    }
}

// Word of layer z (0..7) by selects between values: a select between the array's elements
// would be folded into an indexed load and keep the array in private memory.
__device__ __forceinline__ uint64_t layer_word_v(uint64_t m0, uint64_t m1, uint64_t m2, uint64_t m3, uint64_t m4,
                                                 uint64_t m5, uint64_t m6, uint64_t m7, int z)
{
    const uint64_t lo = (z & 2) ? ((z & 1) ? m3 : m2) : ((z & 1) ? m1 : m0);
    const uint64_t hi = (z & 2) ? ((z & 1) ? m7 : m6) : ((z & 1) ? m5 : m4);
    return (z & 4) ? hi : lo;
}

__device__ __forceinline__ uint64_t layer_word(const uint64_t (&m)[kLayers], int z)
{
    return layer_word_v(m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], z);
}

// One of three values by axis index (values, never fields: a select between fields would
// keep the struct in private memory).
__device__ __forceinline__ float pick3(int a, float x, float y, float z)
{
    return a == 0 ? x : (a == 1 ? y : z);
}

__device__ __forceinline__ bool mask_bit(uint64_t layer, int x, int y)
{
    return (layer >> (x + 8 * y)) & 1ull;
}

// Coordinate (at level lg) of the element whose face ahead, in direction-signed form, is sB.
// Axes with r = 0 keep the form of a downward axis (sB = -B, B = u * 2^lg).
__device__ __forceinline__ int elem_of(float sB, float r, int lg)
{
    const int B = r > 0.0f ? (int)sB : -(int)sB;
    return (B >> lg) - (r > 0.0f ? 1 : 0);           // B is a multiple of 2^lg: exact floor division
}

struct SWalk {
    float Bx, By, Bz;                 // faces ahead at the current level, direction-signed
    float Tx, Ty, Tz;                 // their float32 crossing parameters
    bool blk;                         // block level (else voxel level)
    int cbx, cby, cbz;                // the current block
    int slot;                         // voxel level: its slot (-1: not allocated)
    uint64_t m[kLayers];              // voxel level: the current block's occupancy
    bool pending;                     // voxel level: the current voxel is still to be tested
    int ent_a;                        // axis across which the current voxel (voxel level) or
                                      // block (block level) was entered; -1: the start
    bool anchored;                    // block level: the walk entered the current block at the
    int ax, ay, az;                   //   voxel level, at voxel (ax, ay, az)
    bool settled;                     // finishing at the voxel level near max_range
    bool tie, rtie;                   // near-ties at decisions taken, near-tie with max_range
    float t_hi;                       // the segment stops once the next crossing exceeds this
    float t_lo;                       // crossings at or beyond this get the float64 range test
    bool last;                        // the segment ending at max_range
    bool done;                        // the segment's walk is over
    bool ended, hit;                  // the ray's walk ends in this segment (hit or max_range)
    int fx, fy, fz;                   // last voxel entered (the hit voxel on a hit)
};

// Start walking at element (ux, uy, uz) of level lg (0: voxel, kBlockLog2: block).
__device__ __forceinline__ void s_enter(SWalk &w, const RayF &R, int lg, int ux, int uy, int uz)
{
    const int E = 1 << lg;
    const int px = R.rx > 0.0f, py = R.ry > 0.0f, pz = R.rz > 0.0f;
    const int bx = (ux + px) * E, by = (uy + py) * E, bz = (uz + pz) * E;
    w.Bx = (float)(px ? bx : -bx);
    w.By = (float)(py ? by : -by);
    w.Bz = (float)(pz ? bz : -bz);
    w.Tx = R.rx != 0.0f ? (w.Bx - R.gsx) * R.arx : kInf;
    w.Ty = R.ry != 0.0f ? (w.By - R.gsy) * R.ary : kInf;
    w.Tz = R.rz != 0.0f ? (w.Bz - R.gsz) * R.arz : kInf;
    w.blk = lg != 0;
}

// Entry voxel of block (cx, cy, cz) entered across its face on axis a.
__device__ __forceinline__ void block_entry(const RayArgs &A, const RayF &R, int a, int cx, int cy, int cz, int &vx,
                                            int &vy, int &vz, bool &tie)
{
    entry_voxel(A, R, kBlockLog2, a, cx, cy, cz, vx, vy, vz, tie);
}

// Axis of the nearest crossing (the lowest axis on an exact tie), in float64 when the two
// nearest float32 crossings lie within the guard band.
__device__ __forceinline__ int step_axis64(const RayF &R, float Bx, float By, float Bz, float Tx, float Ty, float Tz,
                                           bool &tie)
{
    const float t1 = __builtin_amdgcn_fmed3f(Tx, fminf(Ty, Tz), -kInf);
    const float t2 = __builtin_amdgcn_fmed3f(Tx, Ty, Tz);
    if (t2 - t1 >= 2e-5f + 1e-6f * t2) return Tx == t1 ? 0 : (Ty == t1 ? 1 : 2);
    const double X = R.rx != 0.0f ? face64(R.rx > 0.0f ? (int)Bx : -(int)Bx, R.gx, R.rx) : __builtin_huge_val();
    const double Y = R.ry != 0.0f ? face64(R.ry > 0.0f ? (int)By : -(int)By, R.gy, R.ry) : __builtin_huge_val();
    const double Z = R.rz != 0.0f ? face64(R.rz > 0.0f ? (int)Bz : -(int)Bz, R.gz, R.rz) : __builtin_huge_val();
    int a = 0;
    double m1 = X;
    if (Y < m1) { a = 1; m1 = Y; }
    if (Z < m1) { a = 2; m1 = Z; }
    tie = tie || (a != 0 && X - m1 < 1e-5) || (a != 1 && Y - m1 < 1e-5) || (a != 2 && Z - m1 < 1e-5);
    return a;
}

// Continue at the voxel level in block (cx, cy, cz) at voxel (vx, vy, vz), entered across axis a
// (-1: the start); the block's occupancy is m.  `pending`: the voxel is still to be tested.
__device__ __forceinline__ void to_voxel_level(SWalk &w, const RayF &R, int cx, int cy, int cz, int slot, int vx,
                                               int vy, int vz, int a, bool pending)
{
    s_enter(w, R, 0, vx, vy, vz);
    w.cbx = cx; w.cby = cy; w.cbz = cz;
    w.slot = slot;
    w.ent_a = a;
    w.pending = pending;
}

// Voxel-level walk from the current voxel: tests the block's occupancy bits until a hit, the
// end of the segment or range, or a block face; a crossed face's block is looked up, and the
// walk goes on at the block level (a free block, not settled) or in that block's voxels.
__device__ __forceinline__ void voxel_run(const RayArgs &A, SWalk &w, const RayF &R)
{
    const SparseView &S = A.sp;
    int vx = elem_of(w.Bx, R.rx, 0), vy = elem_of(w.By, R.ry, 0), vz = elem_of(w.Bz, R.rz, 0);
    uint64_t layer = layer_word(w.m, vz & 7);
    if (w.pending) {
        w.pending = false;
        if (mask_bit(layer, vx & 7, vy & 7)) {
            w.hit = w.ended = w.done = true;
            w.fx = vx; w.fy = vy; w.fz = vz;
            return;
        }
    }
    const int sx = R.rx > 0.0f ? 1 : -1, sy = R.ry > 0.0f ? 1 : -1, sz = R.rz > 0.0f ? 1 : -1;
    const float t_lo = w.t_lo, t_hi = w.t_hi;
    // every step moves one face ahead, so the nearest crossing passes t_hi within
    // 2 (t_hi + 8) steps; the bound only guards the loop
    const int max_steps = 2 * (int)t_hi + 64;
    bool crossed = false;
    for (int it = 0; it < max_steps; ++it) {
        int a = step_axis64(R, w.Bx, w.By, w.Bz, w.Tx, w.Ty, w.Tz, w.tie);
        const float ta = pick3(a, w.Tx, w.Ty, w.Tz);
        if (ta > t_hi || ta >= t_lo) {
            // past the segment's end, or (the last segment) near max_range
            bool stop = ta > t_hi;
            if (!stop) {
                // range test (closed interval) in float64 inside the guard band
                const float sB = pick3(a, w.Bx, w.By, w.Bz);
                const float ga = pick3(a, R.gx, R.gy, R.gz);
                const float ra = pick3(a, R.rx, R.ry, R.rz);
                const double dist = face64(ra > 0.0f ? (int)sB : -(int)sB, ga, ra) * A.h;
                stop = dist > A.max_range;
                if (fabs(dist - A.max_range) < 1e-5 * A.h) w.rtie = true;
            }
            if (stop) {
                w.done = true;
                w.ended = w.last;
                w.fx = vx; w.fy = vy; w.fz = vz;
                return;
            }
        }
        // take the step, with selects rather than branches (a wave's lanes step along different
        // axes); the face crossed is a block face when its coordinate is a multiple of 8
        const bool bx = a == 0, by = a == 1, bz = !bx && !by;
        const float Ba = bx ? w.Bx : (by ? w.By : w.Bz);
        const float rA = bx ? R.rx : (by ? R.ry : R.rz);
        const int face = rA > 0.0f ? (int)Ba : -(int)Ba;
        w.Bx = bx ? w.Bx + 1.0f : w.Bx;
        w.By = by ? w.By + 1.0f : w.By;
        w.Bz = bz ? w.Bz + 1.0f : w.Bz;
        w.Tx = bx ? (w.Bx - R.gsx) * R.arx : w.Tx;
        w.Ty = by ? (w.By - R.gsy) * R.ary : w.Ty;
        w.Tz = bz ? (w.Bz - R.gsz) * R.arz : w.Tz;
        vx += bx ? sx : 0;
        vy += by ? sy : 0;
        vz += bz ? sz : 0;
        w.ent_a = a;
        if ((face & 7) == 0) {
            crossed = true;
            break;
        }
        layer = bz ? layer_word(w.m, vz & 7) : layer;
        if (mask_bit(layer, vx & 7, vy & 7)) {
            w.hit = w.ended = w.done = true;
            w.fx = vx; w.fy = vy; w.fz = vz;
            return;
        }
    }
    if (!crossed) {
        w.done = true;                // not reached: the range ends the walk first
        w.ended = w.last;
        w.fx = vx; w.fy = vy; w.fz = vz;
        return;
    }
    // into the neighbouring block along the last step's axis.  Looked up here, after the step
    // loop, so that the lanes of a wave that cross block faces wait for their table and mask
    // loads together rather than one crossing at a time.
    const int a = w.ent_a;
    const int cx = w.cbx + (a == 0 ? sx : 0), cy = w.cby + (a == 1 ? sy : 0), cz = w.cbz + (a == 2 ? sz : 0);
    int slot;
    bool occ;
    lookup(S, cx, cy, cz, slot, occ);
    w.cbx = cx; w.cby = cy; w.cbz = cz;
    if (!occ && !w.settled) {
        // a free block: on at the block level, anchored at its entry voxel
        s_enter(w, R, kBlockLog2, cx, cy, cz);
        w.anchored = true;
        w.ax = vx; w.ay = vy; w.az = vz;
        return;
    }
    w.slot = slot;
    load_mask(S, occ ? slot : -1, w.m);
    w.pending = true;                 // the next run tests the voxel entered
}

// The current free block's voxels, from the voxel the walk entered it at, to the end of the
// range: the block level stops short of max_range.
__device__ __forceinline__ void settle(const RayArgs &A, SWalk &w, const RayF &R)
{
    int vx, vy, vz;
    if (w.anchored) {
        vx = w.ax; vy = w.ay; vz = w.az;
    } else {
        block_entry(A, R, w.ent_a, w.cbx, w.cby, w.cbz, vx, vy, vz, w.tie);
    }
    w.settled = true;
#pragma unroll
    for (int k = 0; k < kLayers; ++k) w.m[k] = 0;
    to_voxel_level(w, R, w.cbx, w.cby, w.cbz, -1, vx, vy, vz, w.ent_a, false);
}

// Enter block (cx, cy, cz), known to hold an occupied voxel, across axis a: at its entry voxel.
__device__ __forceinline__ void descend(const RayArgs &A, SWalk &w, const RayF &R, int cx, int cy, int cz, int a,
                                        int slot)
{
    int vx, vy, vz;
    block_entry(A, R, a, cx, cy, cz, vx, vy, vz, w.tie);
    load_mask(A.sp, slot, w.m);
    to_voxel_level(w, R, cx, cy, cz, slot, vx, vy, vz, a, true);
}

// Plan K block steps, issue their table loads, and act on the first block that holds an
// occupied voxel (or whose key needs further probing).  Steps whose decision needs float64, or
// whose crossing reaches the range band, end the plan.
template <int K>
__device__ __forceinline__ void block_round(const RayArgs &A, SWalk &w, const RayF &R)
{
    const SparseView &S = A.sp;
    const float gsx = R.gsx, gsy = R.gsy, gsz = R.gsz, arx = R.arx, ary = R.ary, arz = R.arz;
    const float L = (float)(1 << kBlockLog2);
    const int sx = R.rx > 0.0f ? 1 : -1, sy = R.ry > 0.0f ? 1 : -1, sz = R.rz > 0.0f ? 1 : -1;
    const float t_lo = w.t_lo, t_hi = w.t_hi;
    const float t_stop = fminf(t_lo, next_up(t_hi));      // a step is planned iff its crossing is below
    float Bx = w.Bx, By = w.By, Bz = w.Bz, Tx = w.Tx, Ty = w.Ty, Tz = w.Tz;
    int cx = w.cbx, cy = w.cby, cz = w.cbz;
    Entry e[K];
    uint32_t mx = 0, my = 0;
    int nplan = 0;
    bool going = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float t1 = __builtin_amdgcn_fmed3f(Tx, fminf(Ty, Tz), -kInf);
        const float t2 = __builtin_amdgcn_fmed3f(Tx, Ty, Tz);
        const bool bx = Tx == t1, by = !bx & (Ty == t1), bz = !bx & !by;
        going = going & (t1 < t_stop) & (t2 - t1 >= 2e-5f + 1e-6f * t2);
        Bx = bx ? Bx + L : Bx;
        By = by ? By + L : By;
        Bz = bz ? Bz + L : Bz;
        Tx = bx ? (Bx - gsx) * arx : Tx;
        Ty = by ? (By - gsy) * ary : Ty;
        Tz = bz ? (Bz - gsz) * arz : Tz;
        cx += bx ? sx : 0;
        cy += by ? sy : 0;
        cz += bz ? sz : 0;
        const uint32_t idx = block_hash(block_key(cx, cy, cz), S.table_mask);
        e[k] = load_entry(S.table, going ? idx : 0u);
        mx |= bx ? 1u << k : 0u;
        my |= by ? 1u << k : 0u;
        nplan += going ? 1 : 0;
        in_vgpr(mx);
        in_vgpr(my);
        in_vgpr(nplan);
    }
    // the block after step k, from the start and the steps' axes
    const int c0x = w.cbx, c0y = w.cby, c0z = w.cbz;
    uint32_t stopm = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t upto = (2u << k) - 1u;
        const int nx = __builtin_popcount(mx & upto), ny = __builtin_popcount(my & upto), nz = k + 1 - nx - ny;
        const uint64_t key = block_key(c0x + sx * nx, c0y + sy * ny, c0z + sz * nz);
        const uint64_t ek = e[k].key;
        const bool allocated_occ = ek == key && e[k].occ != 0u;
        const bool collide = ek != key && ek != kEmptyKey;     // another key: probe further
        stopm |= (allocated_occ || collide) ? 1u << k : 0u;
    }
    stopm &= (1u << nplan) - 1u;
    const int j = stopm ? __builtin_ctz(stopm) : (nplan == K ? K - 1 : nplan - 1);
    // continue from the position after step j (j = -1: the round's start)
    {
        const uint32_t upto = j >= 0 ? (2u << j) - 1u : 0u;
        const int nx = __builtin_popcount(mx & upto), ny = __builtin_popcount(my & upto);
        const int nz = (j + 1) - nx - ny;
        Bx = w.Bx + L * (float)nx;
        By = w.By + L * (float)ny;
        Bz = w.Bz + L * (float)nz;
        Tx = R.rx != 0.0f ? (Bx - gsx) * arx : kInf;
        Ty = R.ry != 0.0f ? (By - gsy) * ary : kInf;
        Tz = R.rz != 0.0f ? (Bz - gsz) * arz : kInf;
        cx = c0x + sx * nx;
        cy = c0y + sy * ny;
        cz = c0z + sz * nz;
    }
    if (j >= 0) {
        w.Bx = Bx; w.By = By; w.Bz = Bz; w.Tx = Tx; w.Ty = Ty; w.Tz = Tz;
        w.cbx = cx; w.cby = cy; w.cbz = cz;
        w.ent_a = ((mx >> j) & 1u) ? 0 : (((my >> j) & 1u) ? 1 : 2);
        w.anchored = false;
    }
    if (stopm) {
        // block j holds an occupied voxel, or its key probes on (entry j picked by selects, not
        // by indexing the register array)
        Entry ej = e[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            ej.key = k == j ? e[k].key : ej.key;
            ej.slot = k == j ? e[k].slot : ej.slot;
            ej.occ = k == j ? e[k].occ : ej.occ;
        }
        int slot = (int)ej.slot;
        bool occ = ej.occ != 0u;
        const uint64_t key = block_key(cx, cy, cz);
        if (ej.key != key) {
            const uint32_t i0 = block_hash(key, S.table_mask);
            probe_from(S, key, i0, ej, slot, occ);
        }
        if (occ) descend(A, w, R, cx, cy, cz, w.ent_a, slot);
        return;
    }
    if (nplan == K) return;
    // the plan ended at step nplan: the range band, the segment's end, or a near-tie
    const float t1 = __builtin_amdgcn_fmed3f(Tx, fminf(Ty, Tz), -kInf);
    if (t1 >= t_lo) {
        settle(A, w, R);
        return;
    }
    if (t1 > t_hi) {
        // the segment ends inside this free block: nothing before its end is occupied
        w.done = true;
        return;
    }
    bool tie = false;
    const int a = step_axis64(R, Bx, By, Bz, Tx, Ty, Tz, tie);
    const float ta = pick3(a, Tx, Ty, Tz);
    if (ta >= t_lo) {
        // the step the float64 decision takes reaches the range band
        settle(A, w, R);
        return;
    }
    if (ta > t_hi) {
        w.done = true;
        return;
    }
    w.tie = w.tie || tie;
    if (a == 0) { w.Bx = Bx + L; w.Tx = (w.Bx - gsx) * arx; w.cbx = cx + sx; }
    if (a == 1) { w.By = By + L; w.Ty = (w.By - gsy) * ary; w.cby = cy + sy; }
    if (a == 2) { w.Bz = Bz + L; w.Tz = (w.Bz - gsz) * arz; w.cbz = cz + sz; }
    w.ent_a = a;
    w.anchored = false;
    int slot;
    bool occ;
    lookup(S, w.cbx, w.cby, w.cbz, slot, occ);
    if (occ) descend(A, w, R, w.cbx, w.cby, w.cbz, a, slot);
}

// Per-ray outcome of a group of S lanes (valid in the lane that reports the ray: its hit
// segment, else segment 0), and each lane's share of the visit count.
struct SOut {
    bool report;
    bool hit;
    double d;
    uint32_t flags;
    int visits_lane;                  // the ray's visits in the lane whose segment ended it, else 0
    int hit_slot, hit_local;          // debug
};

// Set up segment seg of S of a ray: its start voxel (and block), its end, and its start level.
// Returns false for an empty segment.  The start block (slot0, whether it holds an occupied
// voxel, its occupancy m0) is shared by every segment 0.
__device__ __forceinline__ bool sparse_segment(const RayArgs &A, bool valid, int seg, int S, const RayF &R, int slot0,
                                               bool occ0, const uint64_t (&m0)[kLayers], SWalk &w)
{
    const float rx = R.rx, ry = R.ry, rz = R.rz;
    const double tmax = A.tmax_v;
    bool active = valid;
    // segment start: the start voxel, or the voxel that holds the boundary near seg tmax / S
    int ux = A.v0[0], uy = A.v0[1], uz = A.v0[2];
    if (seg != 0) {
        bool ok;
        seg_boundary(tmax * seg / S, R.gx, R.gy, R.gz, rx, ry, rz, ux, uy, uz, ok);
        if (!ok) {
            active = false;                               // an empty segment
            ux = A.v0[0]; uy = A.v0[1]; uz = A.v0[2];
        }
    }
    // segment end: the next boundary that exists, else max_range
    w.last = true;
    w.t_hi = A.tmax_hi;
    w.t_lo = A.tmax_lo;
    for (int e = seg + 1; e < S && w.last; ++e) {
        int bx, by, bz;
        bool ok;
        const double te = seg_boundary(tmax * e / S, R.gx, R.gy, R.gz, rx, ry, rz, bx, by, bz, ok);
        if (ok) {
            w.last = false;
            w.t_hi = (float)te;       // no crossing lies within the segment margin of te
            w.t_lo = kInf;
        }
    }
    // the start block: a later segment looks its own up (its start voxel was tested by the
    // segment before, so it is not tested again)
    int slot = slot0;
    bool occ = occ0;
    uint64_t m[kLayers];
#pragma unroll
    for (int k = 0; k < kLayers; ++k) m[k] = m0[k];
    const int b0x = ux >> kBlockLog2, b0y = uy >> kBlockLog2, b0z = uz >> kBlockLog2;
    if (seg != 0) {
        lookup(A.sp, b0x, b0y, b0z, slot, occ);
        load_mask(A.sp, occ ? slot : -1, m);
    }
    w.tie = w.rtie = false;
    w.done = !active;
    w.ended = w.hit = false;
    w.settled = false;
    w.anchored = true;
    w.ax = ux; w.ay = uy; w.az = uz;
    w.fx = ux; w.fy = uy; w.fz = uz;
    w.cbx = b0x; w.cby = b0y; w.cbz = b0z;
    w.ent_a = -1;
    w.slot = occ ? slot : -1;
    w.pending = false;
#pragma unroll
    for (int k = 0; k < kLayers; ++k) w.m[k] = m[k];
    if (occ) s_enter(w, R, 0, ux, uy, uz);
    else s_enter(w, R, kBlockLog2, b0x, b0y, b0z);
    return active;
}

// Walk segment seg of S of one ray and combine the segments of the ray (the group of S
// adjacent lanes); every lane of the wave must call this.
template <int K>
__device__ __forceinline__ SOut sparse_trace(const RayArgs &A, bool valid, int seg, int S, float rx, float ry, float rz,
                                             int slot0, bool occ0, const uint64_t (&m0)[kLayers])
{
    const RayF R = make_ray(A, rx, ry, rz);
    SWalk w;
    bool active = sparse_segment(A, valid, seg, S, R, slot0, occ0, m0, w);
    const int lane = threadIdx.x & (kWave - 1);
    const int base = lane & ~(S - 1);
    const uint64_t seg_bits = (1ull << S) - 1ull;        // S <= 16
    const uint64_t lower = ((1ull << seg) - 1ull) << base;
    for (;;) {
        const uint64_t hm = __ballot(w.hit);
        if (hm & lower) active = false;                  // a lower segment already hit
        if (!__any(active)) break;
        if (active) {
            if (w.blk) block_round<K>(A, w, R);
            else voxel_run(A, w, R);
            active = !w.done;
        }
    }
    // combine the group: the lowest segment with a hit owns the ray; the lowest segment whose
    // walk ended holds the ray's last voxel
    const uint64_t gh = (__ballot(w.hit) >> base) & seg_bits;
    const int h = gh ? __ffsll((unsigned long long)gh) - 1 : S;
    const uint64_t ge = (__ballot(valid && w.ended) >> base) & seg_bits;
    const int t = ge ? __ffsll((unsigned long long)ge) - 1 : S;
    const bool keep = valid && seg <= h;
    const uint64_t tm = (__ballot(keep && w.tie) >> base) & seg_bits;
    const uint64_t rm = (__ballot(keep && w.rtie) >> base) & seg_bits;
    SOut o;
    o.report = valid && seg == (h < S ? h : 0);
    o.hit = w.hit && seg == h;
    o.visits_lane = valid && seg == t ? 1 + abs(w.fx - A.v0[0]) + abs(w.fy - A.v0[1]) + abs(w.fz - A.v0[2]) : 0;
    double d = __builtin_huge_val();
    if (o.hit) {
        const int a = w.ent_a;
        d = (a == 0 ? entry64(w.fx, R.gx, R.rx) : (a == 1 ? entry64(w.fy, R.gy, R.ry) : entry64(w.fz, R.gz, R.rz))) * A.h;
    }
    o.d = d;
    o.flags = A.start_flags | (tm ? kRayTie : 0u) | (rm ? kRayRangeTie : 0u);
    o.hit_slot = o.hit ? w.slot : -1;
    o.hit_local = (w.fx & 7) + 8 * (w.fy & 7) + 64 * (w.fz & 7);
    return o;
}

// The value of voxel (i, j, k) of a sparse TSDF map as a field reader: the stored value in its
// block, or free_value outside every stored block (no edge, no clamping).
template <int DT>
struct SparseField {
    SparseView S;                     // a copy (see DenseField)
    __device__ __forceinline__ double operator()(int i, int j, int k) const
    {
        int slot;
        bool occ;
        lookup(S, i >> kBlockLog2, j >> kBlockLog2, k >> kBlockLog2, slot, occ);
        if (slot < 0) return S.free_value;
        const uint32_t local = (uint32_t)(i & 7) + 8u * (uint32_t)(j & 7) + 64u * (uint32_t)(k & 7);
        const typename Voxel<DT>::T v =
            static_cast<const typename Voxel<DT>::T *>(S.values)[(size_t)slot * kBlockVoxels + local];
        if constexpr (DT == RMPC_TSDF_F32) return (double)v;
        else return (double)__builtin_bit_cast(_Float16, v);
    }
};

// Which hit distance a sparse kernel reports: kSvNone the walk's, kSvF32 / kSvF16 the sub-voxel
// distance on a float32 / float16 map.  A template parameter, so that kernels without the
// refinement carry none of its registers.
constexpr int kSvNone = 0, kSvF32 = 1, kSvF16 = 2;

template <int SV>
__device__ __forceinline__ double sparse_distance(const RayArgs &A, float rx, float ry, float rz, double d)
{
    if constexpr (SV == kSvF32) return subvoxel_at(A, SparseField<RMPC_TSDF_F32>{A.sp}, rx, ry, rz, d);
    else if constexpr (SV == kSvF16) return subvoxel_at(A, SparseField<RMPC_TSDF_F16>{A.sp}, rx, ry, rz, d);
    else return d;
}

// The start block, shared by every lane: its slot, whether it holds an occupied voxel, its
// occupancy, and whether the start voxel itself is occupied.
__device__ __forceinline__ bool start_block(const RayArgs &A, int &slot0, bool &occ0, uint64_t (&m0)[kLayers])
{
    lookup(A.sp, A.v0[0] >> kBlockLog2, A.v0[1] >> kBlockLog2, A.v0[2] >> kBlockLog2, slot0, occ0);
    load_mask(A.sp, occ0 ? slot0 : -1, m0);
    return occ0 && mask_bit(layer_word(m0, A.v0[2] & 7), A.v0[0] & 7, A.v0[1] & 7);
}

// One 256-lane tile of a query on a sparse map (lane -> ray position and segment, as for dense
// maps), accumulated and reduced into the query's slots F; every lane of the block calls this.
// SV: the hit distance (see sparse_distance).
template <int K, int SV>
__device__ __forceinline__ void sparse_tile(const RayArgs &A, int tile, int n_tiles, const FinishSlots &F, float *lds)
{
    int slot0;
    bool occ0;
    uint64_t m0[kLayers];
    const bool in_coll = start_block(A, slot0, occ0, m0);
    const int S = A.segments;
    const int p = tile * kBlock + threadIdx.x;
    const int j = p < A.n_list * S ? p / S : 0;
    const int seg = p & (S - 1);
    const float4 rr = load_ray(A.rays, j);
    const bool valid = p < A.n_list * S && __float_as_int(rr.w) < A.n_rays;
    Acc acc;
    acc.zero();
    if (in_coll) {
        if (valid && seg == 0) {
            acc.visits = 1;
            acc.n_hit = 1;
            acc.n_contrib = contributes(A, rr.x, rr.y, rr.z, 0.0);
            policy_accumulate(A.pol, rr.x, rr.y, rr.z, 0.0f, acc);
        }
    } else {
        const SOut o = sparse_trace<K>(A, valid, seg, S, rr.x, rr.y, rr.z, slot0, occ0, m0);
        acc.visits = o.visits_lane;
        if (o.report) {
            acc.n_tie = (o.flags & kRayTie) != 0;
            if (o.hit) {
                const double d = sparse_distance<SV>(A, rr.x, rr.y, rr.z, o.d);
                acc.n_hit = 1;
                acc.n_contrib = contributes(A, rr.x, rr.y, rr.z, d);
                policy_accumulate(A.pol, rr.x, rr.y, rr.z, (float)d, acc);
            }
        }
    }
    grid_finish(acc, tile, n_tiles, F, A.rank_tol, A.n_rays, in_coll ? RMPC_Q_IN_COLLISION : 0u, lds);
}

}  // namespace

}  // namespace rmpc
