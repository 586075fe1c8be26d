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

// The x pass: one wave per row.  Per chunk of 64 voxels a ballot marks the occupied ones; the
// nearest occupied voxel at or left of each lane is the highest set bit up to the lane (else
// the last one of earlier chunks), found in a forward sweep over the chunks, and the nearest
// at or right of it the lowest set bit from the lane on, in a backward sweep.  The row's
// value is the square of the nearer of the two, kFar when the row has none.
template <int DT>
__global__ void __launch_bounds__(256) edt_rows_kernel(MapView m, int32_t *g)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (int64_t)m.ny * m.nz) return;             // the same for the whole wave
    using T = typename Voxel<DT>::T;
    const T *data = static_cast<const T *>(m.data);
    const int lane = threadIdx.x & 63;
    const int32_t nx = m.nx;
    const int64_t base = row * nx;
    int32_t carry = -1;                                   // last occupied index of earlier chunks
    for (int32_t c0 = 0; c0 < nx; c0 += 64) {
        const int32_t i = c0 + lane;
        const uint64_t mask = __ballot(i < nx && Voxel<DT>::occ(data[base + i]));
        const uint64_t upto = lane == 63 ? mask : mask & ((2ull << lane) - 1ull);
        if (i < nx) g[base + i] = upto ? c0 + 63 - __clzll(upto) : carry;
        if (mask) carry = c0 + 63 - __clzll(mask);
    }
    carry = -1;                                           // first occupied index of later chunks
    for (int32_t c0 = ((nx - 1) / 64) * 64; c0 >= 0; c0 -= 64) {
        const int32_t i = c0 + lane;
        const uint64_t mask = __ballot(i < nx && Voxel<DT>::occ(data[base + i]));
        const uint64_t from = mask & (~0ull << lane);
        const int32_t right = from ? c0 + __ffsll((unsigned long long)from) - 1 : carry;
        if (i < nx) {
            const int32_t left = g[base + i];
            int32_t d = kFar;
            if (left >= 0) d = i - left;
            if (right >= 0 && right - i < d) d = right - i;
            g[base + i] = d >= kFar ? kFar : d * d;
        }
        if (mask) carry = c0 + __ffsll((unsigned long long)mask) - 1;
    }
}

// The y and z passes: one block per line of len elements, `stride` apart; line l starts at
// (l % nx) + nx ny (l / nx) for y and at l for z.  The line is staged in LDS and every element
// takes min over j of line_j + (i - j)^2, searching outward from j = i and stopping once
// (i - j)^2 alone reaches the best value found (every line_j is >= 0, so no farther j can be
// smaller): the same minimum as the full scan.  The last pass writes -1 where nothing was found
// (a grid without occupied voxels).
__global__ void __launch_bounds__(256) edt_lines_kernel(int32_t *g, int32_t len, int64_t stride, int32_t nx,
                                                        int64_t plane, int y_pass, int last_pass)
{
    extern __shared__ int32_t line[];
    const int64_t l = blockIdx.x;
    const int64_t base = y_pass ? (l % nx) + plane * (l / nx) : l;
    int found = 0;
    for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
        const int32_t v = g[base + i * stride];
        line[i] = v;
        found |= v < kFar;
    }
    // a line with nothing finite stays "far" (the search below would scan all of it per element)
    if (!__syncthreads_or(found)) {
        for (int32_t i = threadIdx.x; i < len; i += blockDim.x) g[base + i * stride] = last_pass ? -1 : kFar;
        return;
    }
    for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
        int32_t best = line[i];
        for (int32_t d = 1; d < len && d * d < best; ++d) {
            const int32_t lo = i - d, hi = i + d;
            if (lo >= 0 && line[lo] < kFar && line[lo] + d * d < best) best = line[lo] + d * d;
            if (hi < len && line[hi] < kFar && line[hi] + d * d < best) best = line[hi] + d * d;
        }
        g[base + i * stride] = last_pass && best >= kFar ? -1 : best;
    }
}

template <int DT>
hipError_t launch_edt_dt(const MapView &m, int32_t *out, hipStream_t s)
{
    const int64_t rows = (int64_t)m.ny * m.nz, plane = (int64_t)m.nx * m.ny;
    edt_rows_kernel<DT><<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(m, out);
    edt_lines_kernel<<<(unsigned)((int64_t)m.nx * m.nz), 256, sizeof(int32_t) * (size_t)m.ny, s>>>(
        out, m.ny, m.nx, m.nx, plane, 1, 0);
    edt_lines_kernel<<<(unsigned)plane, 256, sizeof(int32_t) * (size_t)m.nz, s>>>(out, m.nz, plane, m.nx, plane, 0,
                                                                                1);
    return hipGetLastError();
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
