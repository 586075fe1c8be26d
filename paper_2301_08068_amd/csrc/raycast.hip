// raycast.hip -- the fused raycast-and-policy kernel (Sec. III-E, III-F) and its debug twin.
//
// One lane owns one ray at a time.  It walks the voxel grid with a 3-D DDA (Amanatides &
// Woo) from the float32 start g along the float32 Halton direction r, planning K voxel
// visits ahead (the visited addresses do not depend on the loaded values, so K loads are
// in flight per lane), stops at the first occupied voxel, evaluates the obstacle policy of
// Sec. III-C in registers and adds it to compensated float32 sums.  The grid-wide sum is
// resolved in float64 by the last block to finish.
//
// Exactness: face crossings are compared in float32 as T = (B - g) / r with B the integer
// boundary (never accumulated).  When the two nearest crossings lie within a guard band
// that bounds the float32 error, or the range test is that close, the decision is redone
// in float64 from the same formula, so every traversal decision -- including which axis
// steps at an exact tie (the lowest index) -- and the hit distance d = T h are the float64
// values of the definition.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"

namespace rmpc {

namespace {

constexpr float kInf = __builtin_huge_valf();

// Float64 crossing parameter of the next face along one axis (r != 0).
__device__ __forceinline__ double cross64(int v, float g, float r)
{
    const double B = r > 0.0f ? (double)(v + 1) : (double)v;
    return (B - (double)g) / (double)r;
}

// The start voxel is occupied: every ray hits at distance 0 (same address for all lanes).
template <int DT>
__device__ __forceinline__ bool start_occupied(const RayArgs &A)
{
    using VT = typename Voxel<DT>::T;
    const VT *vox = static_cast<const VT *>(A.map.data);
    const uint32_t a = addr_x(A.map, A.v0[0]) + addr_y(A.map, A.v0[1]) + addr_z(A.map, A.v0[2]);
    return Voxel<DT>::occ(vox[a]);
}

struct TraceOut {
    double d;          // metres, +inf on a miss
    int32_t hit_lin;   // logical index (debug builds), -1 on a miss
    uint32_t flags;
    int32_t visits;
    bool hit;
};

// Walk one ray.  K voxel visits are planned per round; DEBUG also reports the hit voxel.
template <int DT, int K, bool DEBUG>
__device__ __forceinline__ TraceOut trace_ray(const RayArgs &A, float rx, float ry, float rz)
{
    using VT = typename Voxel<DT>::T;
    const MapView &m = A.map;
    const VT *vox = static_cast<const VT *>(m.data);
    TraceOut o;
    o.flags = A.start_flags;
    o.hit_lin = -1;
    o.d = __builtin_huge_val();
    o.hit = false;
    o.visits = 1;

    int vx = A.v0[0], vy = A.v0[1], vz = A.v0[2];
    const float gx = A.g[0], gy = A.g[1], gz = A.g[2];
    const float irx = rx != 0.0f ? 1.0f / rx : kInf;
    const float iry = ry != 0.0f ? 1.0f / ry : kInf;
    const float irz = rz != 0.0f ? 1.0f / rz : kInf;
    const int px = rx > 0.0f, py = ry > 0.0f, pz = rz > 0.0f;     // face offset of the next boundary
    const int sx = px ? 1 : -1, sy = py ? 1 : -1, sz = pz ? 1 : -1;
    float Tx = rx != 0.0f ? ((float)(vx + px) - gx) * irx : kInf;
    float Ty = ry != 0.0f ? ((float)(vy + py) - gy) * iry : kInf;
    float Tz = rz != 0.0f ? ((float)(vz + pz) - gz) * irz : kInf;
    uint32_t ax = addr_x(m, vx), ay = addr_y(m, vy), az = addr_z(m, vz);

    int step = 0;                 // iterations done (one per face crossing)
    int tie_at = 1 << 30;         // first iteration with a near-tie
    int rtie_at = 1 << 30;        // first iteration with a range near-tie
    bool done = false;

    while (!done) {
        uint32_t addr[K];
        int info[K];              // axis in bits 0..1, coordinate along it above
        int hx[K], hy[K], hz[K];  // full coordinates (debug only)
        int nplan = 0;
        bool ended = false;       // a range/grid termination inside this round
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!ended) {
                // nearest crossing, lowest axis on exact ties
                int a = 0;
                float t1 = Tx;
                if (Ty < t1) { a = 1; t1 = Ty; }
                if (Tz < t1) { a = 2; t1 = Tz; }
                const float t2 = a == 0 ? fminf(Ty, Tz) : (a == 1 ? fminf(Tx, Tz) : fminf(Tx, Ty));
                if (t2 - t1 < 2e-5f + 1e-6f * t2) {
                    // decide in float64 exactly as the definition does
                    const double X = rx != 0.0f ? cross64(vx, gx, rx) : __builtin_huge_val();
                    const double Y = ry != 0.0f ? cross64(vy, gy, ry) : __builtin_huge_val();
                    const double Z = rz != 0.0f ? cross64(vz, gz, rz) : __builtin_huge_val();
                    a = 0;
                    double m1 = X;
                    if (Y < m1) { a = 1; m1 = Y; }
                    if (Z < m1) { a = 2; m1 = Z; }
                    const bool tie = (a != 0 && X - m1 < 1e-5) || (a != 1 && Y - m1 < 1e-5) ||
                                     (a != 2 && Z - m1 < 1e-5);
                    if (tie && tie_at > step + k) tie_at = step + k;
                    t1 = a == 0 ? Tx : (a == 1 ? Ty : Tz);
                }
                // range test (closed interval), float64 inside the guard band
                bool beyond = t1 > A.tmax_hi;
                if (!beyond && t1 >= A.tmax_lo) {
                    const double T64 = a == 0 ? cross64(vx, gx, rx)
                                     : (a == 1 ? cross64(vy, gy, ry) : cross64(vz, gz, rz));
                    const double dist = T64 * A.h;
                    beyond = dist > A.max_range;
                    if (fabs(dist - A.max_range) < 1e-5 * A.h && rtie_at > step + k) rtie_at = step + k;
                }
                if (beyond) {
                    ended = true;
                } else {
                    int coord;
                    if (a == 0) {
                        vx += sx; coord = vx;
                        Tx = ((float)(vx + px) - gx) * irx;
                        ax = addr_x(m, vx);
                    } else if (a == 1) {
                        vy += sy; coord = vy;
                        Ty = ((float)(vy + py) - gy) * iry;
                        ay = addr_y(m, vy);
                    } else {
                        vz += sz; coord = vz;
                        Tz = ((float)(vz + pz) - gz) * irz;
                        az = addr_z(m, vz);
                    }
                    if ((unsigned)vx >= (unsigned)m.nx || (unsigned)vy >= (unsigned)m.ny ||
                        (unsigned)vz >= (unsigned)m.nz) {
                        ended = true;                        // left the grid: a miss
                    } else {
                        addr[k] = ax + ay + az;
                        info[k] = a | (coord << 2);
                        if (DEBUG) { hx[k] = vx; hy[k] = vy; hz[k] = vz; }
                        nplan = k + 1;
                    }
                }
            }
        }
        VT val[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k < nplan) val[k] = vox[addr[k]];
        int hk = -1;
#pragma unroll
        for (int k = K - 1; k >= 0; --k)
            if (k < nplan && Voxel<DT>::occ(val[k])) hk = k;
        if (hk >= 0) {
            int inf = 0, cx = 0, cy = 0, cz = 0;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == hk) {
                    inf = info[k];
                    if (DEBUG) { cx = hx[k]; cy = hy[k]; cz = hz[k]; }
                }
            const int a = inf & 3, c = inf >> 2;
            // the face entered: lower face when moving up, upper face when moving down
            double T64;
            if (a == 0) T64 = cross64(c - sx, gx, rx);
            else if (a == 1) T64 = cross64(c - sy, gy, ry);
            else T64 = cross64(c - sz, gz, rz);
            o.d = T64 * A.h;
            o.hit = true;
            o.visits += hk + 1;
            if (DEBUG) o.hit_lin = cx + m.nx * (cy + m.ny * cz);
            if (tie_at <= step + hk) o.flags |= kRayTie;
            if (rtie_at <= step + hk) o.flags |= kRayRangeTie;
            done = true;
        } else {
            o.visits += nplan;
            step += nplan;
            if (ended) {
                // the iteration that ended the ray is number `step` (0-based)
                if (tie_at <= step) o.flags |= kRayTie;
                if (rtie_at <= step) o.flags |= kRayRangeTie;
                done = true;
            }
        }
    }
    return o;
}

// The obstacle policy of one hit ray (Sec. III-C, Eqs. 4-9), float32, folded into the
// rank-one form  A_i = a r r^T,  b_i = -a |r|^2 phi r  with
//   p = max(0, xdot . r)^2,  q = eta_damp p / (d/nu_damp + eps)        (|f_damp| / |r|)
//   sigma = q / (q|r| + c log(1 + exp(-2 c q|r|)))                      (s(f_damp) = -sigma r)
//   a = w_r(d) sigma^2,  phi = eta_rep exp(-d/nu_rep) + q,  w_r(d) = (1 - d/r)^2 on [0, r].
__device__ __forceinline__ void policy_accumulate(const PolicyF &P, float rx, float ry, float rz,
                                                  float d, Acc &acc)
{
    const float vr = P.vx * rx + P.vy * ry + P.vz * rz;
    const float pp = vr > 0.0f ? vr * vr : 0.0f;
    const float q = P.eta_damp * pp / (d * P.inv_nu_damp + P.eps);
    const float rn2 = rx * rx + ry * ry + rz * rz;
    const float mq = q * sqrtf(rn2);
    const float sigma = q / (mq + P.c * log1pf(expf(-2.0f * P.c * mq)));
    const float wl = 1.0f - d * P.inv_radius;
    const float w = d <= P.radius ? wl * wl : 0.0f;
    const float a = w * sigma * sigma;
    const float phi = P.eta_rep * expf(-d * P.inv_nu_rep) + q;
    const float bb = -a * rn2 * phi;
    csum_add(acc.s[0], acc.c[0], a * rx * rx);
    csum_add(acc.s[1], acc.c[1], a * rx * ry);
    csum_add(acc.s[2], acc.c[2], a * rx * rz);
    csum_add(acc.s[3], acc.c[3], a * ry * ry);
    csum_add(acc.s[4], acc.c[4], a * ry * rz);
    csum_add(acc.s[5], acc.c[5], a * rz * rz);
    csum_add(acc.s[6], acc.c[6], bb * rx);
    csum_add(acc.s[7], acc.c[7], bb * ry);
    csum_add(acc.s[8], acc.c[8], bb * rz);
}

// Exact "non-zero metric" predicate in float64: d < radius and xdot . r > 0, with the dot
// product evaluated left to right without fused multiply-adds.
__device__ __forceinline__ int contributes(const RayArgs &A, float rx, float ry, float rz, double d)
{
#pragma clang fp contract(off)
    const double vn = (A.vel64[0] * (double)rx + A.vel64[1] * (double)ry) + A.vel64[2] * (double)rz;
    return d < A.radius64 && vn > 0.0;
}

template <int DT, int K>
__global__ void __launch_bounds__(kBlock) raycast_rmp_kernel(RayArgs A)
{
    __shared__ float lds[kWavesPerBlock * kPartialWords];
    Acc acc;
    acc.zero();
    const bool in_coll = start_occupied<DT>(A);
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < A.n_rays; i += stride) {
        const float rx = A.dirs[i], ry = A.dirs[i + A.dir_stride], rz = A.dirs[i + 2 * A.dir_stride];
        double d;
        bool hit;
        uint32_t fl;
        int vis;
        if (in_coll) {
            d = 0.0; hit = true; fl = kRayInCollision; vis = 1;
        } else {
            const TraceOut t = trace_ray<DT, K, false>(A, rx, ry, rz);
            d = t.d; hit = t.hit; fl = t.flags; vis = t.visits;
        }
        acc.visits += vis;
        acc.n_tie += (fl & kRayTie) != 0;
        if (hit) {
            acc.n_hit += 1;
            acc.n_contrib += contributes(A, rx, ry, rz, d);
            policy_accumulate(A.pol, rx, ry, rz, (float)d, acc);
        }
    }
    grid_finish(acc, A.partials, A.ticket, A.rank_tol, A.n_rays,
                in_coll ? RMPC_Q_IN_COLLISION : 0u, A.result, lds);
}

template <int DT, int K>
__global__ void __launch_bounds__(kBlock) trace_debug_kernel(RayArgs A)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.n_rays) return;
    const float rx = A.dirs[i], ry = A.dirs[i + A.dir_stride], rz = A.dirs[i + 2 * A.dir_stride];
    TraceOut t;
    if (start_occupied<DT>(A)) {
        t.d = 0.0; t.hit = true; t.flags = kRayInCollision; t.visits = 1; t.hit_lin = A.lin0;
    } else {
        t = trace_ray<DT, K, true>(A, rx, ry, rz);
    }
    A.dbg_hit[i] = t.hit ? t.hit_lin : -1;
    A.dbg_dist[i] = t.d;
    A.dbg_flags[i] = (uint8_t)t.flags;
    if (A.dbg_visits) A.dbg_visits[i] = t.visits;
}

// LiDAR scan policy (Sec. III-G): point p gives direction p/|p| and distance |p|.
// Non-finite points and points closer than min_range are skipped.
__global__ void __launch_bounds__(kBlock) scan_rmp_kernel(ScanArgs A)
{
    __shared__ float lds[kWavesPerBlock * kPartialWords];
    Acc acc;
    acc.zero();
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < A.n_points; i += stride) {
        const float px = A.points[3 * (size_t)i], py = A.points[3 * (size_t)i + 1],
                    pz = A.points[3 * (size_t)i + 2];
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
        double n2, vp;
        {
#pragma clang fp contract(off)
            n2 = ((double)px * (double)px + (double)py * (double)py) + (double)pz * (double)pz;
            vp = (A.vel64[0] * (double)px + A.vel64[1] * (double)py) + A.vel64[2] * (double)pz;
        }
        if (!(n2 >= A.min_range2)) continue;
        const double d64 = sqrt(n2);
        const float inv = (float)(1.0 / d64);
        acc.n_hit += 1;
        acc.n_contrib += d64 < A.radius64 && vp > 0.0;
        policy_accumulate(A.pol, px * inv, py * inv, pz * inv, (float)d64, acc);
    }
    grid_finish(acc, A.partials, A.ticket, A.rank_tol, A.n_points, 0u, A.result, lds);
}

template <int DT>
hipError_t launch_dt(const RayArgs &A, int grid, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 blk(kBlock);
    if (debug) {
        const dim3 g((A.n_rays + kBlock - 1) / kBlock);
        if (e0) hipExtLaunchKernelGGL(trace_debug_kernel<DT, kLookahead>, g, blk, 0, s, e0, e1, 0, A);
        else trace_debug_kernel<DT, kLookahead><<<g, blk, 0, s>>>(A);
    } else {
        if (e0) hipExtLaunchKernelGGL(raycast_rmp_kernel<DT, kLookahead>, dim3(grid), blk, 0, s, e0, e1, 0, A);
        else raycast_rmp_kernel<DT, kLookahead><<<grid, blk, 0, s>>>(A);
    }
    return hipGetLastError();
}

}  // namespace

int ray_grid_blocks(int n_rays)
{
    int b = (n_rays + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b);
}

int scan_grid_blocks(int n_points)
{
    int b = (n_points + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

hipError_t launch_scan(const ScanArgs &A, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 g(scan_grid_blocks(A.n_points)), blk(kBlock);
    if (e0) hipExtLaunchKernelGGL(scan_rmp_kernel, g, blk, 0, s, e0, e1, 0, A);
    else scan_rmp_kernel<<<g, blk, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t launch_raycast(const RayArgs &A, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    const int grid = ray_grid_blocks(A.n_rays);
    switch (A.map.dtype) {
    case RMPC_TSDF_F32: return launch_dt<RMPC_TSDF_F32>(A, grid, s, debug, e0, e1);
    case RMPC_TSDF_F16: return launch_dt<RMPC_TSDF_F16>(A, grid, s, debug, e0, e1);
    default: return launch_dt<RMPC_OCC_U8>(A, grid, s, debug, e0, e1);
    }
}

}  // namespace rmpc
