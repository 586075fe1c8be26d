// edt.hip -- exact Euclidean distance transform of a resident map's occupancy, the distance
// field behind the single-lookup ESDF policy of Sec. III-D: for every voxel the squared
// centre-to-centre distance, in voxels, to the nearest occupied voxel.  The squared distance
// separates over the axes, so three passes: the squared distance to the nearest occupied voxel
// of each x row, then min over j of g_j + (i - j)^2 along y and along z.  Integer arithmetic.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"

namespace rmpc {

namespace {

constexpr int32_t kFar = 1 << 30;   // larger than any squared distance of an allowed grid

// The x pass: one wave per row of at most 64 chunks of 64 voxels (rows of up to 4,096, the
// largest extent a map may have).  The row is read once, four chunks' loads in flight: per
// chunk a ballot marks the occupied voxels and lane c keeps chunk c's mask.  Scans over the
// lanes give each chunk the last occupied voxel before it and the first after it.  Then per
// chunk the nearest occupied voxel at or left of each voxel is the highest set bit up to it
// (else the one before the chunk), at or right of it the lowest set bit from it on (else the
// one after), and the row's value, written once, is the square of the nearer of the two, kFar
// when the row has none.
template <int DT>
__global__ void __launch_bounds__(256) edt_rows_kernel(MapView m, int32_t *g)
{
    constexpr int32_t kNone = 0x7fffffff;                 // no occupied voxel after
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (int64_t)m.ny * m.nz) return;             // the same for the whole wave
    using T = typename Voxel<DT>::T;
    const T *data = static_cast<const T *>(m.data);
    const int lane = threadIdx.x & 63;
    const int32_t nx = m.nx;
    const int nch = (nx + 63) >> 6;
    const int64_t base = row * nx;
    uint64_t mine = 0;                                    // lane c: the mask of chunk c
    for (int c0 = 0; c0 < nch; c0 += 4) {
        bool o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t i = ((c0 + u) << 6) + lane;
            o[u] = i < nx && Voxel<DT>::occ(data[base + i]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t mask = __ballot(o[u]);
            mine = lane == c0 + u ? mask : mine;
        }
    }
    // inclusive prefix max of the chunks' last occupied index, suffix min of their first
    int32_t before = mine ? (lane << 6) + 63 - __clzll(mine) : -1;
    int32_t after = mine ? (lane << 6) + __ffsll((unsigned long long)mine) - 1 : kNone;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t b = __shfl_up(before, o, 64), a = __shfl_down(after, o, 64);
        if (lane >= o) before = max(before, b);
        if (lane + o < 64) after = min(after, a);
    }
    // exclusive: chunks strictly before / after lane's chunk
    int32_t lc_all = __shfl_up(before, 1, 64), rc_all = __shfl_down(after, 1, 64);
    if (lane == 0) lc_all = -1;
    if (lane == 63) rc_all = kNone;
    for (int c = 0; c < nch; ++c) {
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)mine, c);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(mine >> 32), c);
        const uint64_t mask = (uint64_t)lo | ((uint64_t)hi << 32);
        const int32_t lc = __builtin_amdgcn_readlane(lc_all, c), rc = __builtin_amdgcn_readlane(rc_all, c);
        const int32_t i = (c << 6) + lane;
        const uint64_t upto = lane == 63 ? mask : mask & ((2ull << lane) - 1ull);
        const uint64_t from = mask & (~0ull << lane);
        const int32_t left = upto ? (c << 6) + 63 - __clzll(upto) : lc;
        const int32_t right = from ? (c << 6) + __ffsll((unsigned long long)from) - 1 : rc;
        if (i < nx) {
            int32_t d = kFar;
            if (left >= 0) d = i - left;
            if (right != kNone && right - i < d) d = right - i;
            g[base + i] = d >= kFar ? kFar : d * d;
        }
    }
}

// min over j of line[j] + (i - j)^2 for element i of a line of len values (each in [0, kFar]),
// from best = line[i], going outward four distances per pass (eight LDS reads in flight; two
// per pass took 2 % longer) until d^2 reaches best.  Indices
// are clamped at the line's ends instead of tested: a clamped candidate line[0] + d^2 (or
// line[len - 1] + d^2) is no better than the same element's own candidate at its true
// distance, which the search reaches first or which cannot beat best; candidates past the
// stopping distance cannot beat best either, so the result is the exact minimum.  kFar + d^2
// stays below 2^31 for lines of at most 2^15 - 4 elements (lines here have at most 8,190).
__device__ __forceinline__ int32_t line_min(const int32_t *line, int32_t len, int32_t i, int32_t best)
{
    const int32_t last = len - 1;
    int32_t d = 1, dd = 1;                                // dd = d^2
    while (d < len && dd < best) {
        // (d + 1)^2, (d + 2)^2, (d + 3)^2 from d^2
        const int32_t dd1 = dd + 2 * d + 1, dd2 = dd1 + 2 * d + 3, dd3 = dd2 + 2 * d + 5;
        const int32_t a0 = line[max(i - d, 0)], b0 = line[min(i + d, last)];
        const int32_t a1 = line[max(i - d - 1, 0)], b1 = line[min(i + d + 1, last)];
        const int32_t a2 = line[max(i - d - 2, 0)], b2 = line[min(i + d + 2, last)];
        const int32_t a3 = line[max(i - d - 3, 0)], b3 = line[min(i + d + 3, last)];
        best = min(best, min(a0, b0) + dd);
        best = min(best, min(a1, b1) + dd1);
        best = min(best, min(a2, b2) + dd2);
        best = min(best, min(a3, b3) + dd3);
        dd = dd3 + 2 * d + 7;                             // (d + 4)^2
        d += 4;
    }
    return best;
}

// The y and z passes: one block per group of up to 2^wlog neighbouring lines (consecutive x at
// one z for the y pass, at one y for the z pass), each of len elements `stride` apart.  Global
// loads and stores go element by element across the group's lines, so that a wave covers runs
// of consecutive x, eight per thread in flight; in LDS each line is contiguous (rows of len + 1
// words: the transposing writes and reads hit distinct banks), and the search runs along a line
// in consecutive lanes, whose distances are alike.  Every element takes min over j of
// line_j + (i - j)^2, searching outward from j = i and stopping once (i - j)^2 alone reaches the
// best value found (every line_j is >= 0, so no farther j can be smaller): the same minimum as
// the full scan.  A line with nothing finite keeps "far" without a search; the last pass writes
// -1 there (a grid without occupied voxels).
__global__ void __launch_bounds__(256) edt_lines_kernel(int32_t *g, int32_t len, int64_t stride, int32_t nx,
                                                        int32_t groups_x, int wlog, int64_t plane, int y_pass,
                                                        int last_pass)
{
    constexpr int kUnroll = 8;
    extern __shared__ int32_t lds[];                      // in[W][len + 1], res[W][len + 1], found[W]
    const int W = 1 << wlog;
    const int row = len + 1;
    int32_t *res = lds + (size_t)W * row;
    int32_t *found = res + (size_t)W * row;
    const int64_t q = blockIdx.x / groups_x;              // z (y pass) or y (z pass)
    const int32_t x0 = (int32_t)(blockIdx.x % groups_x) * W;
    const int64_t base = x0 + (y_pass ? plane * q : (int64_t)nx * q);
    const int nw = min(W, nx - x0);                       // lines of this group inside the grid
    const int n = len * W;
    if ((int)threadIdx.x < W) found[threadIdx.x] = 0;
    __syncthreads();
    for (int i0 = threadIdx.x; i0 < n; i0 += kUnroll * 256) {
        int32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int idx = i0 + u * 256;
            const int w = idx & (W - 1), i = idx >> wlog;
            v[u] = idx < n && w < nw ? g[base + w + (int64_t)i * stride] : kFar;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int idx = i0 + u * 256;
            const int w = idx & (W - 1), i = idx >> wlog;
            if (idx < n) {
                lds[w * row + i] = v[u];
                if (v[u] < kFar) found[w] = 1;            // every writer stores the same value
            }
        }
    }
    __syncthreads();
    // line w, element i of the thread's first item; later items are 256 further in (w, i) order
    int w = threadIdx.x / len, i = threadIdx.x - w * len;
    for (; w < nw; ) {
        const int32_t *line = lds + w * row;
        int32_t best = line[i];
        if (found[w]) best = line_min(line, len, i, best);
        res[w * row + i] = last_pass && best >= kFar ? -1 : best;
        i += 256;
        if (i >= len) {
            const int k = i / len;
            w += k;
            i -= k * len;
        }
    }
    __syncthreads();
    for (int i0 = threadIdx.x; i0 < n; i0 += kUnroll * 256) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int idx = i0 + u * 256;
            const int ww = idx & (W - 1), ii = idx >> wlog;
            if (idx < n && ww < nw) g[base + ww + (int64_t)ii * stride] = res[ww * row + ii];
        }
    }
}

// LDS a group of 2^wlog lines of len elements may take (both copies and the flags).  The y pass
// takes at most 13 KiB, so that many blocks share a CU for the latency of the searches' LDS
// reads (4 lines per group at the paper map's 400-voxel lines: 1.3 % faster than 8, while 2 lost
// 21 %); the z pass, whose elements lie a whole plane apart, at most 26 KiB, so that a group's
// loads and stores cover longer runs of consecutive x (8 lines at 400: 2.8 % faster than 4 over
// the transform, 16 slower).  A single line may take up to 64 KiB.
constexpr size_t kGroupLdsY = 13 * 1024;
constexpr size_t kGroupLdsZ = 26 * 1024;
constexpr size_t kLinesLds = 64 * 1024;

size_t lines_lds(int32_t len, int wlog)
{
    return (2 * ((size_t)len + 1) + 1) * ((size_t)1 << wlog) * sizeof(int32_t);
}

// The widest group (at most 64 lines) that fits cap bytes.
int lines_wlog(int32_t len, size_t cap)
{
    int wlog = 6;
    while (wlog > 0 && lines_lds(len, wlog) > cap) --wlog;
    return wlog;
}

hipError_t launch_lines(int32_t *g, int32_t len, int64_t stride, int32_t nx, int64_t other, int64_t plane,
                        int y_pass, int last_pass, hipStream_t s)
{
    const int wlog = lines_wlog(len, y_pass ? kGroupLdsY : kGroupLdsZ);
    const int32_t groups_x = (nx + (1 << wlog) - 1) >> wlog;
    const size_t lds = lines_lds(len, wlog);
    if (lds > kLinesLds) return hipErrorInvalidValue;     // a line longer than 8,190 voxels (uploads take 4,096)
    edt_lines_kernel<<<(unsigned)(other * groups_x), 256, lds, s>>>(g, len, stride, nx, groups_x, wlog, plane, y_pass,
                                                                    last_pass);
    return hipGetLastError();
}

template <int DT>
hipError_t launch_edt_dt(const MapView &m, int32_t *out, hipStream_t s)
{
    const int64_t rows = (int64_t)m.ny * m.nz, plane = (int64_t)m.nx * m.ny;
    edt_rows_kernel<DT><<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(m, out);
    if (hipError_t e = hipGetLastError()) return e;
    // y: lines (x, z), elements nx apart; z: lines (x, y), elements nx ny apart
    if (hipError_t e = launch_lines(out, m.ny, m.nx, m.nx, m.nz, plane, 1, 0, s)) return e;
    return launch_lines(out, m.nz, plane, m.nx, m.ny, plane, 0, 1, s);
}

// Distance in metres at voxel (i, j, k), indices clamped into the grid; -1 when the grid has
// no occupied voxel.
__device__ double esdf_at(const EsdfArgs &A, int i, int j, int k)
{
    i = i < 0 ? 0 : (i >= A.nx ? A.nx - 1 : i);
    j = j < 0 ? 0 : (j >= A.ny ? A.ny - 1 : j);
    k = k < 0 ? 0 : (k >= A.nz ? A.nz - 1 : k);
    const int32_t q = A.sq[(int64_t)i + (int64_t)A.nx * ((int64_t)j + (int64_t)A.ny * k)];
    return q < 0 ? -1.0 : A.h * sqrt((double)q);
}

// Single-lookup ESDF policy (Sec. III-D): the distance of the position's voxel, its gradient by
// central differences over the six neighbours (divided by 2h), the obstacle direction
// r = -grad / |grad|, one obstacle policy (Eqs. 4-9) for (r, d) in float64, resolved.  Nothing
// occupied or a zero gradient: all sums zero.  One thread.
__global__ void esdf_policy_kernel(EsdfArgs A)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    rmpc_result r = {};
    r.n_rays = 1;
    const int c0 = A.v0[0], c1 = A.v0[1], c2 = A.v0[2];
    const double d = esdf_at(A, c0, c1, c2);
    double S[3][3] = {}, b[3] = {}, f[3] = {}, lam[3] = {};
    int32_t rank = 0;
    uint32_t flags = d == 0.0 ? RMPC_Q_IN_COLLISION : 0u;
    double grad[3] = {0.0, 0.0, 0.0};
    if (d >= 0.0) {
        grad[0] = (esdf_at(A, c0 + 1, c1, c2) - esdf_at(A, c0 - 1, c1, c2)) / (2.0 * A.h);
        grad[1] = (esdf_at(A, c0, c1 + 1, c2) - esdf_at(A, c0, c1 - 1, c2)) / (2.0 * A.h);
        grad[2] = (esdf_at(A, c0, c1, c2 + 1) - esdf_at(A, c0, c1, c2 - 1)) / (2.0 * A.h);
    }
    const double gn = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    if (d >= 0.0 && gn > 0.0) {
        const double rh[3] = {-grad[0] / gn, -grad[1] / gn, -grad[2] / gn};
        const double n[3] = {-rh[0], -rh[1], -rh[2]};            // away from the obstacle
        const double erep = A.eta_rep * exp(-d / A.nu_rep);
        const double vn = -(A.vel[0] * n[0] + A.vel[1] * n[1] + A.vel[2] * n[2]);
        const double mx = vn > 0.0 ? vn : 0.0;
        const double kd = A.eta_damp / (d / A.nu_damp + A.eps);
        double fd[3], fo[3];
        for (int a = 0; a < 3; ++a) {
            fd[a] = kd * (mx * mx * n[a]);
            fo[a] = erep * n[a] + fd[a];
        }
        const double nf = sqrt(fd[0] * fd[0] + fd[1] * fd[1] + fd[2] * fd[2]);
        const double den = nf + A.c * log1p(exp(-2.0 * A.c * nf));
        const double w = d > A.radius ? 0.0 : d * d / (A.radius * A.radius) - 2.0 * d / A.radius + 1.0;
        double sv[3];
        for (int a = 0; a < 3; ++a) sv[a] = fd[a] / den;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S[i][j] = w * sv[i] * sv[j];
        for (int i = 0; i < 3; ++i) b[i] = S[i][0] * fo[0] + S[i][1] * fo[1] + S[i][2] * fo[2];
        r.n_hit = 1;
        r.n_contrib = d < A.radius && (A.vel[0] * rh[0] + A.vel[1] * rh[1] + A.vel[2] * rh[2]) > 0.0;
        resolve3(S, b, A.rank_tol, f, lam, rank, flags);
    }
    for (int i = 0; i < 3; ++i) {
        r.f[i] = f[i];
        r.b[i] = b[i];
        r.lambda[i] = lam[i];
        for (int j = 0; j < 3; ++j) r.A[3 * i + j] = S[i][j];
    }
    r.rank = rank;
    r.flags = flags;
    *A.out = r;
}

}  // namespace

hipError_t launch_esdf(const EsdfArgs &a, hipStream_t s)
{
    esdf_policy_kernel<<<1, 64, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_edt(const MapView &m, int32_t *out, hipStream_t s)
{
    switch (m.dtype) {
    case RMPC_TSDF_F32: return launch_edt_dt<RMPC_TSDF_F32>(m, out, s);
    case RMPC_TSDF_F16: return launch_edt_dt<RMPC_TSDF_F16>(m, out, s);
    default: return launch_edt_dt<RMPC_OCC_U8>(m, out, s);
    }
}

}  // namespace rmpc
