// sparse.hip -- the raycast-and-policy query on a sparse block map: the single-query and debug
// kernels over the walk of rmpc_sparse.h, and the kernels that build a sparse map's occupancy
// masks and table flags at upload.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"
#include "rmpc_sparse.h"
#include "rmpc_walk.h"

namespace rmpc {

namespace {

template <int K, int SV>
__global__ void __launch_bounds__(kBlock, 2) sparse_rmp_kernel(RayArgs A)
{
    __shared__ float lds[kReduceLdsWords];
    sparse_tile<K, SV>(A, xcd_tile(blockIdx.x, gridDim.x), gridDim.x,
                   single_slots(A.partials, A.ticket, A.result, A.done, A.seq), lds);
}

// Per-ray outputs: the hit as slot * 512 + (x + 8 y + 64 z within the block), -1 on a miss.
template <int K, int SV>
__global__ void __launch_bounds__(kBlock, 2) sparse_trace_kernel(RayArgs A)
{
    int slot0;
    bool occ0;
    uint64_t m0[kLayers];
    const bool in_coll = start_block(A, slot0, occ0, m0);
    const int S = A.segments;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const int j = p < A.n_list * S ? p / S : 0;
    const int seg = p & (S - 1);
    const float4 rr = load_ray(A.rays, j);
    const int i = __float_as_int(rr.w);
    const bool valid = p < A.n_list * S && i < A.n_rays;
    if (in_coll) {
        if (valid && seg == 0) {
            A.dbg_hit[i] = slot0 * kBlockVoxels + (A.v0[0] & 7) + 8 * (A.v0[1] & 7) + 64 * (A.v0[2] & 7);
            A.dbg_dist[i] = 0.0;
            A.dbg_flags[i] = (uint8_t)(A.start_flags | kRayInCollision);
            if (A.dbg_visits) A.dbg_visits[i] = 1;
        }
        return;
    }
    const SOut o = sparse_trace<K>(A, valid, seg, S, rr.x, rr.y, rr.z, slot0, occ0, m0);
    // the ray's visit count is the sum over its group
    int v = o.visits_lane;
    for (int off = 1; off < S; off <<= 1) v += __shfl_xor(v, off, kWave);
    if (o.report) {
        A.dbg_hit[i] = o.hit ? o.hit_slot * kBlockVoxels + o.hit_local : -1;
        A.dbg_dist[i] = o.hit ? sparse_distance<SV>(A, rr.x, rr.y, rr.z, o.d) : o.d;
        A.dbg_flags[i] = (uint8_t)o.flags;
        if (A.dbg_visits) A.dbg_visits[i] = v;
    }
}

// Occupancy words of every slot (thread: one slot's layer) from its stored values.
template <int DT>
__global__ void sparse_mask_kernel(SparseView v, uint64_t *occ)
{
    using T = typename Voxel<DT>::T;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= v.n_slots * kLayers) return;
    const T *vals = static_cast<const T *>(v.values) + (size_t)t * 64;   // layer z of slot t / 8
    uint64_t w = 0;
    for (int k = 0; k < 64; ++k) w |= Voxel<DT>::occ(vals[k]) ? 1ull << k : 0ull;
    occ[t] = w;
}

// Each table entry's occupied flag: whether its slot's occupancy has any bit set.
__global__ void sparse_flag_kernel(SparseView v, HashEntry *table)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > v.table_mask) return;
    HashEntry &e = table[i];
    if (e.key == kEmptyKey || e.slot < 0 || e.slot >= v.n_slots) return;
    uint64_t any = 0;
    for (int k = 0; k < kLayers; ++k) any |= v.occ[(size_t)e.slot * kLayers + k];
    e.occupied = any != 0 ? 1u : 0u;
}

template <int K, int SV>
hipError_t launch_sparse_k(const RayArgs &A, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 g((A.n_list * A.segments + kBlock - 1) / kBlock), blk(kBlock);
    if (debug) {
        sparse_trace_kernel<K, SV><<<g, blk, 0, s>>>(A);
    } else if (e0) {
        hipExtLaunchKernelGGL(sparse_rmp_kernel<K, SV>, g, blk, 0, s, e0, e1, 0, A);
    } else {
        sparse_rmp_kernel<K, SV><<<g, blk, 0, s>>>(A);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_sparse_sv(const RayArgs &A, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    if (!A.subvoxel) return launch_sparse_k<K, kSvNone>(A, s, debug, e0, e1);
    if (A.sp.dtype == RMPC_TSDF_F32) return launch_sparse_k<K, kSvF32>(A, s, debug, e0, e1);
    return launch_sparse_k<K, kSvF16>(A, s, debug, e0, e1);
}

}  // namespace

hipError_t launch_sparse(const RayArgs &A, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    switch (A.lookahead) {
    case 4: return launch_sparse_sv<4>(A, s, debug, e0, e1);
    case 16: return launch_sparse_sv<16>(A, s, debug, e0, e1);
    default: return launch_sparse_sv<8>(A, s, debug, e0, e1);
    }
}

hipError_t launch_sparse_masks(const SparseView &v, HashEntry *table, hipStream_t s)
{
    uint64_t *occ = const_cast<uint64_t *>(v.occ);
    const int n = v.n_slots * kLayers;
    if (n > 0) {
        switch (v.dtype) {
        case RMPC_TSDF_F32: sparse_mask_kernel<RMPC_TSDF_F32><<<(n + 255) / 256, 256, 0, s>>>(v, occ); break;
        case RMPC_TSDF_F16: sparse_mask_kernel<RMPC_TSDF_F16><<<(n + 255) / 256, 256, 0, s>>>(v, occ); break;
        default: sparse_mask_kernel<RMPC_OCC_U8><<<(n + 255) / 256, 256, 0, s>>>(v, occ); break;
        }
    }
    const uint32_t cap = v.table_mask + 1u;
    sparse_flag_kernel<<<(cap + 255) / 256, 256, 0, s>>>(v, table);
    return hipGetLastError();
}

}  // namespace rmpc
