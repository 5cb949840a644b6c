// noalloc.hip -- rpp_backward_noalloc: the backward gradient scatter with
// its staging buffers in a fixed, statically allocated device array instead
// of library-allocated device memory, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The array lives in the code object's device memory: every GPU the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address (it is a host-side stand-in); the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/rpp.h"
#include "device_common.h"

namespace rpp {
void set_last_error_text(const char *msg);
}

namespace {

using rpp::NONE;

// Scratch layout for m <= RPP_NOALLOC_MAX_BARS bars, each region 256-byte
// aligned: birth edges (u64) | death edges (u64) | dL/dbirth (f32) |
// dL/ddeath (f32).
constexpr size_t kEdgeBytes = (size_t)RPP_NOALLOC_MAX_BARS * 8;
constexpr size_t kGradBytes = (size_t)RPP_NOALLOC_MAX_BARS * 4;
constexpr size_t kScratchBytes = 2 * kEdgeBytes + 2 * kGradBytes;
static_assert(kEdgeBytes % 256 == 0 && kGradBytes % 256 == 0, "regions stay 256-byte aligned");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_dev[kMaxDevices];   // each device's address of `scratch`, once looked up

// Gradient of coordinate k of point u: the birth term, then the death term,
// of every bar in bar order -- the order in which rpp_backward lists its
// terms (it leaves out terms with no edge or a zero gradient, which add
// nothing here either), so both sum the same FP64 values in the same order.
__global__ void k_edge_grad_bars(const float *__restrict__ pts, int n, int d,
                                 const uint64_t *__restrict__ be, const uint64_t *__restrict__ de,
                                 const float *__restrict__ gb, const float *__restrict__ gd,
                                 int64_t nbars, float *__restrict__ grad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * d)
        return;
    const int u = (int)(t / d), k = (int)(t % d);
    double acc = 0.0;
    for (int64_t i = 0; i < nbars; ++i) {
        const float b = gb ? gb[i] : 0.0f;
        if (b != 0.0f)
            rpp::edge_grad_add(acc, pts, d, u, k, be[i], b);
        const float e = gd ? gd[i] : 0.0f;
        if (e != 0.0f)
            rpp::edge_grad_add(acc, pts, d, u, k, de[i], e);
    }
    grad[t] = (float)acc;
}

int fail(int code, const char *msg)
{
    rpp::set_last_error_text(msg);
    return code;
}

// Device address of the current device's scratch array, looked up on the
// device's first call (with that device current) and kept.
int scratch_for_current_device(unsigned char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(RPP_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RPP_E_DEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return fail(RPP_E_DEVICE, "hipGetSymbolAddress(scratch) failed");
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_dev[dev]);
    return RPP_OK;
}

}  // namespace

extern "C" int rpp_backward_noalloc(const float *points_dev, int32_t n, int32_t d, int64_t nbars,
                                    const uint64_t *birth_edge, const uint64_t *death_edge,
                                    const float *grad_birth, const float *grad_death,
                                    float *grad_points_dev, void *hip_stream)
{
    if (n < 1 || d < 1 || nbars < 0)
        return fail(RPP_E_INVAL, "need n >= 1, d >= 1, nbars >= 0");
    if (!points_dev || !grad_points_dev)
        return fail(RPP_E_INVAL, "null device pointer");
    if (nbars > 0 && (!birth_edge || !death_edge))
        return fail(RPP_E_INVAL, "edge arrays are NULL");
    if (nbars > RPP_NOALLOC_MAX_BARS)
        return fail(RPP_E_RANGE, "nbars exceeds RPP_NOALLOC_MAX_BARS, the fixed scratch size");
    const uint64_t E = (uint64_t)n * (uint64_t)(n - 1) / 2;
    for (int64_t i = 0; i < nbars; ++i) {
        if (grad_birth && grad_birth[i] != 0.0f && birth_edge[i] != NONE && birth_edge[i] >= E)
            return fail(RPP_E_INVAL, "birth edge index out of range");
        if (grad_death && grad_death[i] != 0.0f && death_edge[i] != NONE && death_edge[i] >= E)
            return fail(RPP_E_INVAL, "death edge index out of range");
    }
    unsigned char *base = nullptr;
    int rc = scratch_for_current_device(&base);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    uint64_t *be = reinterpret_cast<uint64_t *>(base);
    uint64_t *de = reinterpret_cast<uint64_t *>(base + kEdgeBytes);
    float *gb = reinterpret_cast<float *>(base + 2 * kEdgeBytes);
    float *gd = reinterpret_cast<float *>(base + 2 * kEdgeBytes + kGradBytes);
    if (nbars > 0) {
        // every region the kernel reads is written here first, so nothing
        // left by an earlier call is seen
        if (hipMemcpyAsync(be, birth_edge, (size_t)nbars * 8, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(de, death_edge, (size_t)nbars * 8, hipMemcpyHostToDevice, s) !=
                hipSuccess)
            return fail(RPP_E_DEVICE, "copy of the edge arrays failed");
        if (grad_birth && hipMemcpyAsync(gb, grad_birth, (size_t)nbars * 4,
                                         hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(RPP_E_DEVICE, "copy of dL/dbirth failed");
        if (grad_death && hipMemcpyAsync(gd, grad_death, (size_t)nbars * 4,
                                         hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(RPP_E_DEVICE, "copy of dL/ddeath failed");
    }
    const int64_t m = (int64_t)n * d;
    hipLaunchKernelGGL(k_edge_grad_bars, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                       points_dev, (int)n, (int)d, be, de, grad_birth ? gb : nullptr,
                       grad_death ? gd : nullptr, nbars, grad_points_dev);
    if (hipGetLastError() != hipSuccess)
        return fail(RPP_E_DEVICE, "launch of the gradient kernel failed");
    if (hipStreamSynchronize(s) != hipSuccess)
        return fail(RPP_E_DEVICE, "hipStreamSynchronize failed");
    return RPP_OK;
}
