// noalloc.hip -- rmpc_scan_query_noalloc: the LiDAR scan policy (Sec. III-G) for callers that
// cannot allocate memory (code under HIP graph capture, tight control loops).  It needs no
// context, allocates nothing, and keeps its reduction scratch (block partials and the
// arrival ticket) in a fixed device array of this file; the result goes to caller-owned
// device memory in stream order.  The kernel is the one rmpc_scan_query launches.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rmpc_host.h"

namespace {

constexpr int kMaxDevices = 64;
// block partials of the largest scan launch, then the ticket word on its own 256 bytes
constexpr size_t kPartialBytes = (size_t)rmpc::kScanMaxBlocks * rmpc::kPartialWords * sizeof(float);
constexpr size_t kTicketOffset = kPartialBytes;
constexpr size_t kScratchBytes = kPartialBytes + 256;
static_assert(kPartialBytes % 256 == 0, "the ticket starts on a 256-byte boundary");

// Each GPU the library runs on holds its own copy until the process ends.  Host code never
// uses this name as an address: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

std::mutex g_mu;
uint8_t *g_scratch_dev[kMaxDevices];   // device address of `scratch` on each device, or null

// Sets n words at p to zero (a kernel rather than a memset, so that a caller may capture it).
__global__ void clear_words_kernel(uint32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The device address of `scratch` on `device` (current), looked up on first use.
rmpc_status scratch_on(int device, uint8_t **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rmpc_host::fail(RMPC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_dev[device];
    return RMPC_OK;
}

}  // namespace

using namespace rmpc_host;

extern "C" rmpc_status rmpc_scan_query_noalloc(int device, const float *points_dev, int32_t n_points,
                                               const double v[3], const rmpc_params *params, void *hip_stream,
                                               rmpc_result *out_dev)
{
    if (!out_dev) return fail(RMPC_E_INVALID, "out_dev is NULL");
    rmpc::ScanArgs A;
    if (rmpc_status st = setup_scan(points_dev, n_points, v, params, A)) return st;
    const int blocks = rmpc::scan_grid_blocks(n_points);
    if ((size_t)blocks * rmpc::kPartialWords * sizeof(float) > kPartialBytes)
        return fail(RMPC_E_INVALID, "scan launch needs more block partials than the fixed scratch holds");
    int ndev = 0;
    RMPC_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev || device >= kMaxDevices) return fail(RMPC_E_INVALID, "no such device");
    DeviceGuard dg(device);
    uint8_t *base = nullptr;
    if (rmpc_status st = scratch_on(device, &base)) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    A.partials = reinterpret_cast<float *>(base);
    A.ticket = reinterpret_cast<uint32_t *>(base + kTicketOffset);
    A.result = out_dev;
    A.done = nullptr;
    A.seq = 0;
    // the ticket must read zero when the scan kernel starts (the kernel's last block also
    // resets it, but a call must not depend on how an earlier one ended)
    clear_words_kernel<<<1, 64, 0, s>>>(A.ticket, 64);
    RMPC_HIP(hipGetLastError());
    RMPC_HIP(rmpc::launch_scan(A, s));
    return RMPC_OK;
}
