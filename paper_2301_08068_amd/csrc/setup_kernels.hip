// setup_kernels.hip -- one-time device work: the Halton ray-direction table, the ordered ray
// lists and the free-cell summaries of an uploaded voxel grid.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"

namespace rmpc {

namespace {

// Radical inverse (van der Corput) of i in base b: the base-b digits of i, mirrored about
// the radix point, formed as an exact integer ratio num / b^k and rounded once.
__device__ double radical_inverse(uint32_t i, uint32_t b)
{
    uint64_t num = 0, den = 1;
    while (i != 0) {
        num = num * b + i % b;
        den *= b;
        i /= b;
    }
    return (double)num / (double)den;
}

// Ray i of the 2-D Halton set (Sec. III-E, Eq. 10): polar angle from base 2, azimuth from
// base 3.  cos(phi) = 1 - 2 H(i,2), sin(phi) = sqrt(1 - cos^2 phi), theta = 2 pi H(i,3);
// float64 throughout, each component rounded to float32 once.
__global__ void directions_kernel(DirsArgs A)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const double u = radical_inverse((uint32_t)i, 2);
    const double w = radical_inverse((uint32_t)i, 3);
    const double z = 1.0 - 2.0 * u;
    const double rho = sqrt(fmax(0.0, 1.0 - z * z));
    double s, c;
    sincospi(2.0 * w, &s, &c);
    A.out[i] = (float)(rho * c);
    A.out[i + A.n] = (float)(rho * s);
    A.out[i + 2 * A.n] = (float)z;
}

// Summary of each whole block of (2^LG)^3 voxels: "occupied" if any voxel in it is, stored
// at base + bx + nbx * (by + nby * bz).
template <int DT, int LG>
__global__ void summary_kernel(MapView m, uint32_t base, int nbx, int nby, int nbz, typename Voxel<DT>::T occ_val,
                               typename Voxel<DT>::T free_val)
{
    using T = typename Voxel<DT>::T;
    constexpr int E = 1 << LG;
    const int n_blocks = nbx * nby * nbz;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_blocks) return;
    const int cx = c % nbx, cy = (c / nbx) % nby, cz = c / (nbx * nby);
    T *data = static_cast<T *>(const_cast<void *>(m.data));
    bool any = false;
    for (int k = 0; k < E * E * E && !any; ++k) {
        const int x = (cx << LG) + (k % E), y = (cy << LG) + ((k / E) % E), z = (cz << LG) + k / (E * E);
        any = Voxel<DT>::occ(data[(uint32_t)x + (uint32_t)m.nx * ((uint32_t)y + (uint32_t)m.ny * (uint32_t)z)]);
    }
    data[base + (uint32_t)c] = any ? occ_val : free_val;
}

template <int DT, int LG>
void launch_summary(const MapView &m, uint32_t base, int nbx, int nby, int nbz, typename Voxel<DT>::T occ_val,
                    typename Voxel<DT>::T free_val, hipStream_t s)
{
    const int n = nbx * nby * nbz;
    if (n > 0) summary_kernel<DT, LG><<<(n + 255) / 256, 256, 0, s>>>(m, base, nbx, nby, nbz, occ_val, free_val);
}

template <int DT>
void launch_summaries(const MapView &m, typename Voxel<DT>::T occ_val, typename Voxel<DT>::T free_val, hipStream_t s)
{
    launch_summary<DT, kCellLog2>(m, m.cell_base, m.ncx, m.ncy, m.ncz, occ_val, free_val, s);
    launch_summary<DT, kBrickLog2>(m, m.brick_base, m.nbx, m.nby, m.nbz, occ_val, free_val, s);
}

// Chunk-wise count of entries < n (one 1024-entry chunk per block).
__global__ void __launch_bounds__(1024) compact_count_kernel(CompactArgs A)
{
    __shared__ int wsum[16];
    const int j = blockIdx.x * 1024 + threadIdx.x;
    const bool keep = j < A.n_all && A.order[j] < A.n;
    const uint64_t m = __ballot(keep);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        A.counts[blockIdx.x] = t;
    }
}

// Stable scatter of the kept entries: chunk offset from the counts of earlier chunks,
// wave offset from earlier waves, lane offset from the ballot.
__global__ void __launch_bounds__(1024) compact_scatter_kernel(CompactArgs A)
{
    __shared__ int wsum[16];
    __shared__ int base;
    const int j = blockIdx.x * 1024 + threadIdx.x;
    const bool keep = j < A.n_all && A.order[j] < A.n;
    const uint64_t m = __ballot(keep);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = __popcll(m);
    if (threadIdx.x == 0) {
        int t = 0;
        for (int b = 0; b < (int)blockIdx.x; ++b) t += A.counts[b];
        base = t;
    }
    __syncthreads();
    int off = base;
    for (int u = 0; u < w; ++u) off += wsum[u];
    off += __popcll(m & ((1ull << lane) - 1ull));
    if (keep) A.out[off] = A.order[j];
}

__global__ void __launch_bounds__(256) gather_kernel(GatherArgs A)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= A.n) return;
    const int32_t i = A.idx[k];
    A.out[k] = RayRec{A.dirs[i], A.dirs[i + A.stride], A.dirs[i + 2 * A.stride], i};
}

}  // namespace

hipError_t launch_gather(const GatherArgs &a, hipStream_t s)
{
    gather_kernel<<<(a.n + 255) / 256, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs &a, hipStream_t s)
{
    const int blocks = (a.n_all + 1023) / 1024;
    compact_count_kernel<<<blocks, 1024, 0, s>>>(a);
    compact_scatter_kernel<<<blocks, 1024, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_directions(const DirsArgs &a, hipStream_t s)
{
    directions_kernel<<<(a.n + 255) / 256, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_map_summaries(const SummaryArgs &a, hipStream_t s)
{
    switch (a.map.dtype) {
    case RMPC_TSDF_F32: launch_summaries<RMPC_TSDF_F32>(a.map, -1.0f, 1.0f, s); break;
    case RMPC_TSDF_F16: launch_summaries<RMPC_TSDF_F16>(a.map, (uint16_t)0xbc00, (uint16_t)0x3c00, s); break;
    default: launch_summaries<RMPC_OCC_U8>(a.map, (uint8_t)1, (uint8_t)0, s); break;
    }
    return hipGetLastError();
}

}  // namespace rmpc
