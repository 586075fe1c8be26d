// edt.hip -- exact Euclidean distance transform of a resident map's occupancy, the distance
// field behind the single-lookup ESDF policy of Sec. III-D: for every voxel the squared
// centre-to-centre distance, in voxels, to the nearest occupied voxel.  The squared distance
// separates over the axes, so three passes of min over j of g_j + (i - j)^2 along x, then y,
// then z (g starts as 0 on occupied voxels and "far" elsewhere).  All integer arithmetic.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"

namespace rmpc {

namespace {

constexpr int32_t kFar = 1 << 30;   // larger than any squared distance of an allowed grid

// One block per line of len elements, `stride` apart, starting at `base`.  The first pass
// (x rows, contiguous) stages 0 for occupied voxels and kFar for free ones; the others stage
// the previous pass's values.  Every element then takes min over j of line_j + (i - j)^2,
// searching outward from j = i and stopping once (i - j)^2 alone reaches the best value found
// (every line_j is >= 0, so no farther j can be smaller): the same minimum as the full scan.
// The last pass writes -1 where nothing was found (a grid without occupied voxels).
template <int DT, bool FIRST>
__global__ void __launch_bounds__(256) edt_lines_kernel(MapView m, int32_t *g, int32_t len, int64_t stride,
                                                        int pass, int last_pass)
{
    extern __shared__ int32_t line[];
    const int64_t l = blockIdx.x;
    const int64_t nx = m.nx, plane = (int64_t)m.nx * m.ny;
    // pass 0: x rows; pass 1: y lines over (x, z); pass 2: z lines over (x, y)
    const int64_t base = pass == 0 ? l * nx : (pass == 1 ? (l % nx) + plane * (l / nx) : l);
    int found = 0;
    if constexpr (FIRST) {
        using T = typename Voxel<DT>::T;
        const T *data = static_cast<const T *>(m.data);
        for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
            const int32_t v = Voxel<DT>::occ(data[base + i * stride]) ? 0 : kFar;
            line[i] = v;
            found |= v < kFar;
        }
    } else {
        for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
            const int32_t v = g[base + i * stride];
            line[i] = v;
            found |= v < kFar;
        }
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
    const int64_t plane = (int64_t)m.nx * m.ny;
    edt_lines_kernel<DT, true><<<(unsigned)((int64_t)m.ny * m.nz), 256, sizeof(int32_t) * (size_t)m.nx, s>>>(
        m, out, m.nx, 1, 0, 0);
    edt_lines_kernel<DT, false><<<(unsigned)((int64_t)m.nx * m.nz), 256, sizeof(int32_t) * (size_t)m.ny, s>>>(
        m, out, m.ny, m.nx, 1, 0);
    edt_lines_kernel<DT, false><<<(unsigned)plane, 256, sizeof(int32_t) * (size_t)m.nz, s>>>(m, out, m.nz, plane, 2,
                                                                                           1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_edt(const MapView &m, int32_t *out, hipStream_t s)
{
    switch (m.dtype) {
    case RMPC_TSDF_F32: return launch_edt_dt<RMPC_TSDF_F32>(m, out, s);
    case RMPC_TSDF_F16: return launch_edt_dt<RMPC_TSDF_F16>(m, out, s);
    default: return launch_edt_dt<RMPC_OCC_U8>(m, out, s);
    }
}

}  // namespace rmpc
