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
constexpr int kMaxBlocks = kMaxPartialSlots;

// Per-ray debug flags (same bit values as the public RMPC_RAY_*).
constexpr uint32_t kRayTie = RMPC_RAY_TIE;
constexpr uint32_t kRayRangeTie = RMPC_RAY_RANGE_TIE;
constexpr uint32_t kRayStartFace = RMPC_RAY_START_FACE;
constexpr uint32_t kRayInCollision = RMPC_RAY_IN_COLLISION;

// Occupancy of a stored value: TSDF <= 0 (NaN is free), occupancy byte != 0.
template <int DT> struct Voxel;
template <> struct Voxel<RMPC_TSDF_F32> {
    using T = float;
    static __device__ __forceinline__ bool occ(float v) { return v <= 0.0f; }
};
template <> struct Voxel<RMPC_TSDF_F16> {
    using T = uint16_t;
    // binary16 <= 0 as one half-precision comparison (NaN compares false: free)
    static __device__ __forceinline__ bool occ(uint16_t b)
    {
        return __builtin_bit_cast(_Float16, b) <= (_Float16)0.0f;
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

// ------------------------------------------------------------------------------------
// block and grid reductions of Acc
//
// A block writes one row per thread to LDS.  Nine groups of 16 lanes (threads 0..143) merge
// one compensated pair each and four groups in the last wave (threads 192..255) add one
// integer counter each, so no wave mixes the two kinds.  Lane q of a group merges rows q,
// q+16, ... in row order (all 16 loaded first), and the 16 lanes combine with a butterfly
// that always puts the lower lane first.  (A pairwise tree over the 16 rows was no faster.)  Every step has a fixed order, so results do not
// depend on timing.
// ------------------------------------------------------------------------------------

constexpr int kRowWords = 23;                 // odd row stride: conflict-free column reads
constexpr int kColLanes = 16;
constexpr int kPairLanes = 9 * kColLanes;     // threads merging the compensated pairs
constexpr int kIntLane0 = kBlock - 4 * kColLanes;   // first thread adding the counters
constexpr int kReduceLdsWords = kBlock * kRowWords;
static_assert(kPairLanes <= kIntLane0 && kIntLane0 % kWave == 0, "pair and counter lanes share a wave");

__device__ __forceinline__ void row_store(float *row, const Acc &a)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) { row[k] = a.s[k]; row[9 + k] = a.c[k]; }
    int32_t *q = reinterpret_cast<int32_t *>(row + 18);
    q[0] = a.n_hit; q[1] = a.n_contrib; q[2] = a.n_tie; q[3] = a.visits;
}

// Butterfly over the 16 lanes of a pair group; the lower lane's value is always the left
// operand of the merge.
__device__ __forceinline__ void pair_butterfly(int t, float &s, float &c)
{
#pragma unroll
    for (int off = 1; off < kColLanes; off <<= 1) {
        const float s2 = __shfl_xor(s, off, kWave);
        const float c2 = __shfl_xor(c, off, kWave);
        const bool upper = (t & off) != 0;
        float ls = upper ? s2 : s, lc = upper ? c2 : c;
        csum_merge(ls, lc, upper ? s : s2, upper ? c : c2);
        s = ls;
        c = lc;
    }
}

__device__ __forceinline__ int32_t int_butterfly(int32_t v)
{
#pragma unroll
    for (int off = 1; off < kColLanes; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// The thread index through an empty asm statement.  The reductions' LDS addresses and lane
// masks depend on it alone, and in a kernel that loops over tiles the compiler would otherwise
// compute them once before the loop and keep them in registers through every walk.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// The block total, written to out[] in partial layout (9 sums, 9 compensations, 4 counters).
__device__ __forceinline__ void block_reduce_store(const Acc &a, float *lds, float *out)
{
    const int t = opaque_tid(), q = t % kColLanes;
    row_store(lds + t * kRowWords, a);
    __syncthreads();
    if (t < kPairLanes) {
        const int col = t / kColLanes;
        float vs[kBlock / kColLanes], vc[kBlock / kColLanes];
#pragma unroll
        for (int u = 0; u < kBlock / kColLanes; ++u) {
            vs[u] = lds[(q + u * kColLanes) * kRowWords + col];
            vc[u] = lds[(q + u * kColLanes) * kRowWords + 9 + col];
        }
        float s = vs[0], c = vc[0];
#pragma unroll
        for (int u = 1; u < kBlock / kColLanes; ++u) csum_merge(s, c, vs[u], vc[u]);
        pair_butterfly(t, s, c);
        if (q == 0) { out[col] = s; out[9 + col] = c; }
    } else if (t >= kIntLane0) {
        const int col = (t - kIntLane0) / kColLanes;
        const int32_t *rows = reinterpret_cast<const int32_t *>(lds);
        int32_t v = 0;
#pragma unroll
        for (int u = 0; u < kBlock / kColLanes; ++u) v += rows[(q + u * kColLanes) * kRowWords + 18 + col];
        v = int_butterfly(v);
        if (q == 0) reinterpret_cast<int32_t *>(out)[18 + col] = v;
    }
}

// ------------------------------------------------------------------------------------
// float64 resolve: f = S^+ b  (Eq. 1 with the pseudo-inverse cut rank_tol * lambda_max)
// ------------------------------------------------------------------------------------

// Reciprocal and reciprocal square root from the hardware estimates plus two Newton steps
// (relative error near 1 ulp; a Jacobi rotation only needs c^2 + s^2 = 1 to that level).
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ double rsqrt64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x * r, r, 1.5);
    return r * fma(-0.5 * x * r, r, 1.5);
}

// One Jacobi rotation in the (P, Q) plane that annihilates S[P][Q]; V accumulates the
// eigenvectors as columns.  Compile-time indices keep everything in registers.
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&S)[3][3], double (&V)[3][3])
{
    const double spq = S[P][Q];
    if (spq == 0.0) return;
    const double theta = (S[Q][Q] - S[P][P]) * (0.5 * rcp64(spq));
    const double at = fabs(theta);
    // t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), the smaller root of t^2 + 2 t theta = 1
    double t;
    if (at > 1e100) {
        t = 0.5 * rcp64(theta);
    } else {
        const double y = fma(at, at, 1.0);
        t = rcp64(at + y * rsqrt64(y));
        t = theta < 0.0 ? -t : t;
    }
    const double c = rsqrt64(fma(t, t, 1.0));
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

// Eigenvalues of a symmetric 3x3 matrix, ascending, from the trigonometric solution of its
// characteristic cubic: with q = tr S / 3, p^2 = |S - q I|_F^2 / 6 and B = (S - q I) / p, the
// eigenvalues are q + 2 p cos(phi + 2 pi k / 3), phi = acos(det B / 2) / 3.  Each is within a
// few units of rounding of |S| of the exact value.  False for a diagonal matrix.
__device__ inline bool sym3_eigvals(const double (&S)[3][3], double (&lam)[3])
{
    const double p1 = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    if (p1 == 0.0) return false;
    const double q = (S[0][0] + S[1][1] + S[2][2]) * (1.0 / 3.0);
    const double d0 = S[0][0] - q, d1 = S[1][1] - q, d2 = S[2][2] - q;
    const double p = sqrt((d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1) * (1.0 / 6.0));
    const double ip = 1.0 / p;
    const double b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip;
    const double b01 = S[0][1] * ip, b02 = S[0][2] * ip, b12 = S[1][2] * ip;
    const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    const double phi = acos(r) * (1.0 / 3.0);
    lam[2] = q + 2.0 * p * cos(phi);
    lam[0] = q + 2.0 * p * cos(phi + 2.0943951023931957);          // + 2 pi / 3
    lam[1] = 3.0 * q - lam[0] - lam[2];
    return true;
}

// Resolve a symmetric PSD 3x3 metric sum: eigenvalues (ascending), rank, ILL flag and f.
// A sum whose smallest eigenvalue lies clearly above the ILL band and whose condition number
// lies clearly below the ILL limit (both by a relative margin of 1e-9, far above the closed
// form's error) has full rank and no ILL flag: there f = S^-1 b by the adjugate, which is the
// pseudo-inverse; every other sum takes the cyclic Jacobi path below.
__device__ inline void resolve3(const double (&Sin)[3][3], const double (&b)[3], double rank_tol,
                                double (&f)[3], double (&lam)[3], int32_t &rank, uint32_t &flags)
{
    {
        double l[3];
        if (sym3_eigvals(Sin, l) && l[2] > 0.0 && l[0] > 10.0 * (rank_tol * l[2]) * (1.0 + 1e-9) &&
            l[2] < 1e3 * (1.0 - 1e-9) * l[0]) {
            const double(&A)[3][3] = Sin;
            // cofactors (symmetric for a symmetric matrix, so the adjugate is the same matrix)
            const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
            const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
            const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
            const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
            const double c12 = A[0][1] * A[2][0] - A[0][0] * A[2][1];
            const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
            const double id = 1.0 / (A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02);
            f[0] = (c00 * b[0] + c01 * b[1] + c02 * b[2]) * id;
            f[1] = (c01 * b[0] + c11 * b[1] + c12 * b[2]) * id;
            f[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * id;
            lam[0] = l[0]; lam[1] = l[1]; lam[2] = l[2];
            rank = 3;
            return;
        }
    }
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

// A row in partial layout (16-byte aligned: rows are 128 bytes apart) as six 16-byte loads.
__device__ __forceinline__ void acc_from_partial(const float *p, Acc &a)
{
    const float4 *q4 = reinterpret_cast<const float4 *>(p);
    float w[24];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float4 v = q4[k];
        w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) { a.s[k] = w[k]; a.c[k] = w[9 + k]; }
    a.n_hit = __float_as_int(w[18]); a.n_contrib = __float_as_int(w[19]);
    a.n_tie = __float_as_int(w[20]); a.visits = __float_as_int(w[21]);
}

// Where one reduction keeps its state: tile rows (one per tile), a ticket, the result slot,
// and the completion publication.  A batch shares `finished` (queries done so far) among its
// queries and publishes once, when the last one is done.
struct FinishSlots {
    float *tile_rows;
    uint32_t *tickets;
    rmpc_result *out;
    uint32_t *finished;          // null for a single query
    int32_t n_queries;
    uint64_t *done;              // null: nothing is published
    uint64_t seq;
};

// Grid reduction: every block stores its total in its row and takes a ticket; the last block
// merges all rows -- thread t takes rows t, t + 256, ... in that order, then the block tree
// merges the threads -- so the result depends on the rows and their count only, never on the
// order in which blocks finish.  It resolves, writes the result and publishes.
__device__ inline void grid_finish(const Acc &a, int b, int nb, const FinishSlots &F,
                                   double rank_tol, int32_t n_rays, uint32_t extra_flags, float *lds)
{
    __shared__ int last;
    __shared__ __align__(16) float tot[kPartialWords];
    block_reduce_store(a, lds, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        // one thread stores the block's row (the 22 words and 2 of padding) and takes the ticket
        // with release order only: the release writes this XCD's L2 back so that the last
        // block, on any XCD, reads the row; an acquire here would invalidate the L2 that the
        // blocks still walking on this XCD read the map through
        float4 *dst = reinterpret_cast<float4 *>(F.tile_rows + (size_t)b * kPartialWords);
        const float4 *src = reinterpret_cast<const float4 *>(tot);
#pragma unroll
        for (int k = 0; k < 6; ++k) dst[k] = src[k];
        const uint32_t prev = __hip_atomic_fetch_add(F.tickets, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == (uint32_t)(nb - 1);
    }
    __syncthreads();
    if (!last) return;
    // the last block acquires every block's row
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    Acc m;
    m.zero();
    for (int r0 = opaque_tid(); r0 < nb; r0 += 2 * kBlock) {
        // two rows per pass, both loaded before either is merged
        Acc r1, r2;
        acc_from_partial(F.tile_rows + (size_t)r0 * kPartialWords, r1);
        const int s2 = r0 + kBlock;
        if (s2 < nb) acc_from_partial(F.tile_rows + (size_t)s2 * kPartialWords, r2);
        else r2.zero();
        m.merge(r1);
        if (s2 < nb) m.merge(r2);
    }
    __syncthreads();                         // lds and tot are reused
    block_reduce_store(m, lds, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc total;
        acc_from_partial(tot, total);
        __hip_atomic_store(F.tickets, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        finalize_result(total, rank_tol, n_rays, extra_flags, F.out);
        bool publish = true;
        if (F.finished) {
            // system scope: every query's result reaches the host before the publication
            const uint32_t prev = __hip_atomic_fetch_add(F.finished, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_SYSTEM);
            publish = prev == (uint32_t)(F.n_queries - 1);
            if (publish) __hip_atomic_store(F.finished, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // publish: the results are visible to the host before the sequence number (no word to
        // publish to: the result stays in device memory, ordered by the stream)
        if (publish && F.done) __hip_atomic_store(F.done, F.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace rmpc
