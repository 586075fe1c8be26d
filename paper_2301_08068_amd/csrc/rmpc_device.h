// rmpc_device.h -- device-side building blocks shared by the library's HIP kernels:
// map addressing and occupancy, compensated float32 sums, wave/block reductions and the
// float64 3x3 resolve.  gfx950 only (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmpcast.h"
#include "rmpc_kernels.h"

namespace rmpc {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // threads per block of the ray kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPartialWords = 32;           // one block partial: 18 floats + 4 ints, padded
constexpr int kMaxBlocks = kMaxPartialSlots;

// Per-ray debug flags (same bit values as the public RMPC_RAY_*).
constexpr uint32_t kRayTie = RMPC_RAY_TIE;
constexpr uint32_t kRayRangeTie = RMPC_RAY_RANGE_TIE;
constexpr uint32_t kRayStartFace = RMPC_RAY_START_FACE;
constexpr uint32_t kRayInCollision = RMPC_RAY_IN_COLLISION;

__device__ __forceinline__ uint32_t addr_x(const MapView &m, int x)
{
    return ((uint32_t)(x >> m.lbx) << (m.lbx + m.lby + m.lbz)) + (uint32_t)(x & ((1 << m.lbx) - 1));
}
__device__ __forceinline__ uint32_t addr_y(const MapView &m, int y)
{
    return (uint32_t)(y >> m.lby) * ((uint32_t)m.nbx << (m.lbx + m.lby + m.lbz)) +
           ((uint32_t)(y & ((1 << m.lby) - 1)) << m.lbx);
}
__device__ __forceinline__ uint32_t addr_z(const MapView &m, int z)
{
    return (uint32_t)(z >> m.lbz) * ((uint32_t)(m.nbx * m.nby) << (m.lbx + m.lby + m.lbz)) +
           ((uint32_t)(z & ((1 << m.lbz) - 1)) << (m.lbx + m.lby));
}

// Occupancy of a stored value: TSDF <= 0 (NaN is free), occupancy byte != 0.
template <int DT> struct Voxel;
template <> struct Voxel<RMPC_TSDF_F32> {
    using T = float;
    static __device__ __forceinline__ bool occ(float v) { return v <= 0.0f; }
};
template <> struct Voxel<RMPC_TSDF_F16> {
    using T = uint16_t;
    // binary16 <= 0: +-0, or sign set and not NaN
    static __device__ __forceinline__ bool occ(uint16_t b)
    {
        uint32_t mag = b & 0x7fffu;
        return mag == 0u || ((b & 0x8000u) && mag <= 0x7c00u);
    }
};
template <> struct Voxel<RMPC_OCC_U8> {
    using T = uint8_t;
    static __device__ __forceinline__ bool occ(uint8_t v) { return v != 0; }
};

// ------------------------------------------------------------------------------------
// compensated float32 sums (error-free TwoSum; the compensations are kept to the end)
// ------------------------------------------------------------------------------------

__device__ __forceinline__ void csum_add(float &s, float &c, float x)
{
#pragma clang fp contract(off)
    float t = s + x;
    float bp = t - s;
    float err = (s - (t - bp)) + (x - bp);
    s = t;
    c += err;
}

__device__ __forceinline__ void csum_merge(float &s, float &c, float s2, float c2)
{
#pragma clang fp contract(off)
    float t = s + s2;
    float bp = t - s;
    float err = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = (c + c2) + err;
}

// The quantities one query reduces: the 6 unique entries of sum A_i, the 3 of sum b_i
// (each as a compensated pair) and four integer counters.
struct Acc {
    float s[9], c[9];
    int32_t n_hit, n_contrib, n_tie, visits;

    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k < 9; ++k) { s[k] = 0.0f; c[k] = 0.0f; }
        n_hit = n_contrib = n_tie = visits = 0;
    }
    __device__ __forceinline__ void merge(const Acc &o)
    {
#pragma unroll
        for (int k = 0; k < 9; ++k) csum_merge(s[k], c[k], o.s[k], o.c[k]);
        n_hit += o.n_hit; n_contrib += o.n_contrib; n_tie += o.n_tie; visits += o.visits;
    }
};

// Butterfly reduction across the 64 lanes; every lane ends with the same total, combined
// in a fixed pattern (so the result does not depend on timing).
__device__ __forceinline__ void wave_reduce(Acc &a)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        Acc o;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            o.s[k] = __shfl_xor(a.s[k], off, kWave);
            o.c[k] = __shfl_xor(a.c[k], off, kWave);
        }
        o.n_hit = __shfl_xor(a.n_hit, off, kWave);
        o.n_contrib = __shfl_xor(a.n_contrib, off, kWave);
        o.n_tie = __shfl_xor(a.n_tie, off, kWave);
        o.visits = __shfl_xor(a.visits, off, kWave);
        // lower lane first so both partners form the identical sum
        if (threadIdx.x & off) {
            Acc lo = o;
            lo.merge(a);
            a = lo;
        } else {
            a.merge(o);
        }
    }
}

// Block reduction: waves reduce, then wave totals are merged in wave order by thread 0.
// Returns the total in thread 0.  `lds` holds kWavesPerBlock * kPartialWords words.
__device__ __forceinline__ void block_reduce(Acc &a, float *lds)
{
    wave_reduce(a);
    const int wid = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        float *p = lds + wid * kPartialWords;
#pragma unroll
        for (int k = 0; k < 9; ++k) { p[k] = a.s[k]; p[9 + k] = a.c[k]; }
        int32_t *q = reinterpret_cast<int32_t *>(p + 18);
        q[0] = a.n_hit; q[1] = a.n_contrib; q[2] = a.n_tie; q[3] = a.visits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWavesPerBlock; ++w) {
            const float *p = lds + w * kPartialWords;
            Acc o;
#pragma unroll
            for (int k = 0; k < 9; ++k) { o.s[k] = p[k]; o.c[k] = p[9 + k]; }
            const int32_t *q = reinterpret_cast<const int32_t *>(p + 18);
            o.n_hit = q[0]; o.n_contrib = q[1]; o.n_tie = q[2]; o.visits = q[3];
            a.merge(o);
        }
    }
}

__device__ __forceinline__ void store_partial(float *dst, const Acc &a)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) { dst[k] = a.s[k]; dst[9 + k] = a.c[k]; }
    int32_t *q = reinterpret_cast<int32_t *>(dst + 18);
    q[0] = a.n_hit; q[1] = a.n_contrib; q[2] = a.n_tie; q[3] = a.visits;
}

__device__ __forceinline__ void load_partial(const float *src, Acc &a)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) { a.s[k] = src[k]; a.c[k] = src[9 + k]; }
    const int32_t *q = reinterpret_cast<const int32_t *>(src + 18);
    a.n_hit = q[0]; a.n_contrib = q[1]; a.n_tie = q[2]; a.visits = q[3];
}

// ------------------------------------------------------------------------------------
// float64 resolve: f = S^+ b  (Eq. 1 with the pseudo-inverse cut rank_tol * lambda_max)
// ------------------------------------------------------------------------------------

// One Jacobi rotation in the (P, Q) plane that annihilates S[P][Q]; V accumulates the
// eigenvectors as columns.  Compile-time indices keep everything in registers.
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&S)[3][3], double (&V)[3][3])
{
    const double spq = S[P][Q];
    if (spq == 0.0) return;
    const double theta = (S[Q][Q] - S[P][P]) / (2.0 * spq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0);
    const double s = t * c;
    constexpr int R = 3 - P - Q;                 // the untouched index
    const double spp = S[P][P], sqq = S[Q][Q], srp = S[R][P], srq = S[R][Q];
    S[P][P] = spp - t * spq;
    S[Q][Q] = sqq + t * spq;
    S[P][Q] = S[Q][P] = 0.0;
    S[R][P] = S[P][R] = c * srp - s * srq;
    S[R][Q] = S[Q][R] = s * srp + c * srq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][P], vkq = V[k][Q];
        V[k][P] = c * vkp - s * vkq;
        V[k][Q] = s * vkp + c * vkq;
    }
}

// Resolve a symmetric PSD 3x3 metric sum: eigenvalues (ascending), rank, ILL flag and f.
__device__ inline void resolve3(const double (&Sin)[3][3], const double (&b)[3], double rank_tol,
                                double (&f)[3], double (&lam)[3], int32_t &rank, uint32_t &flags)
{
    double S[3][3], V[3][3];
    double frob2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            S[i][j] = Sin[i][j];
            V[i][j] = i == j ? 1.0 : 0.0;
            frob2 += S[i][j] * S[i][j];
        }
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off2 = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
        if (off2 <= 1e-30 * frob2) break;
        jacobi_rotate<0, 1>(S, V);
        jacobi_rotate<0, 2>(S, V);
        jacobi_rotate<1, 2>(S, V);
    }
    // sort eigenpairs ascending (a 3-element network on indices)
    int i0 = 0, i1 = 1, i2 = 2;
    double d0 = S[0][0], d1 = S[1][1], d2 = S[2][2];
    if (d1 < d0) { double t = d0; d0 = d1; d1 = t; int u = i0; i0 = i1; i1 = u; }
    if (d2 < d1) { double t = d1; d1 = d2; d2 = t; int u = i1; i1 = i2; i2 = u; }
    if (d1 < d0) { double t = d0; d0 = d1; d1 = t; int u = i0; i0 = i1; i1 = u; }
    lam[0] = d0; lam[1] = d1; lam[2] = d2;
    const int idx[3] = {i0, i1, i2};
    f[0] = f[1] = f[2] = 0.0;
    rank = 0;
    if (!(d2 > 0.0)) return;
    const double tau = rank_tol * d2;
    double lmin_kept = d2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double l = lam[j];
        if (l >= 0.1 * tau && l <= 10.0 * tau) flags |= RMPC_Q_ILL;
        if (!(l > tau)) continue;
        ++rank;
        lmin_kept = fmin(lmin_kept, l);
        const int col = idx[j];
        double q0, q1, q2;
        // column `col` of V without dynamic register indexing
        q0 = col == 0 ? V[0][0] : (col == 1 ? V[0][1] : V[0][2]);
        q1 = col == 0 ? V[1][0] : (col == 1 ? V[1][1] : V[1][2]);
        q2 = col == 0 ? V[2][0] : (col == 1 ? V[2][1] : V[2][2]);
        const double qb = (q0 * b[0] + q1 * b[1] + q2 * b[2]) / l;
        f[0] += q0 * qb; f[1] += q1 * qb; f[2] += q2 * qb;
    }
    if (d2 / lmin_kept > 1e3) flags |= RMPC_Q_ILL;
}

// Turn a reduced accumulator into the public result (run by one thread).
__device__ inline void finalize_result(const Acc &a, double rank_tol, int32_t n_rays,
                                       uint32_t extra_flags, rmpc_result *out)
{
    double sv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) sv[k] = (double)a.s[k] + (double)a.c[k];
    // unique entries: 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz, then b x, y, z
    const double S[3][3] = {{sv[0], sv[1], sv[2]}, {sv[1], sv[3], sv[4]}, {sv[2], sv[4], sv[5]}};
    const double b[3] = {sv[6], sv[7], sv[8]};
    double f[3], lam[3];
    int32_t rank = 0;
    uint32_t flags = extra_flags;
    resolve3(S, b, rank_tol, f, lam, rank, flags);
    if (a.n_tie > 0) flags |= RMPC_Q_TIE;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out->f[i] = f[i];
        out->b[i] = b[i];
        out->lambda[i] = lam[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) out->A[3 * i + j] = S[i][j];
    }
    out->rank = rank;
    out->n_hit = a.n_hit;
    out->n_contrib = a.n_contrib;
    out->n_tie = a.n_tie;
    out->flags = flags;
    out->n_rays = n_rays;
    out->visits = a.visits;
}

// Grid-level finish: every block stores its partial; the last block to arrive (ticket)
// merges all partials in block order and resolves.  Deterministic for a fixed grid.
__device__ inline void grid_finish(Acc &a, float *partials, uint32_t *ticket, double rank_tol,
                                   int32_t n_rays, uint32_t extra_flags, rmpc_result *out,
                                   float *lds)
{
    __shared__ int is_last;
    block_reduce(a, lds);
    if (threadIdx.x == 0) {
        store_partial(partials + (size_t)blockIdx.x * kPartialWords, a);
        __threadfence();
        const uint32_t prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        is_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    Acc t;
    t.zero();
    for (uint32_t blk = threadIdx.x; blk < gridDim.x; blk += kBlock) {
        Acc o;
        load_partial(partials + (size_t)blk * kPartialWords, o);
        t.merge(o);
    }
    __syncthreads();                       // lds reuse
    block_reduce(t, lds);
    if (threadIdx.x == 0) {
        finalize_result(t, rank_tol, n_rays, extra_flags, out);
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace rmpc
