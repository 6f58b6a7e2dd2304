// Read-bandwidth ceilings of the memory hierarchy of the GPU the library runs
// on: the roofs the assignment walk is measured against.  The walk reads its
// posting slices from L2, from the Infinity Cache (the memory-side cache in
// front of HBM) or from HBM, so one plain read kernel is timed with working
// sets that live at each level.
//
//   shared  every workgroup reads the whole buffer (rotated by workgroup), so
//           a buffer of a few MB stays resident in each XCD's L2;
//   split   the workgroups split the buffer and sweep it `passes` times, so a
//           buffer larger than the L2s but smaller than the Infinity Cache is
//           served from the latter, and a buffer of GBs from HBM.
// Loads are 16 bytes per lane, 64 consecutive lanes reading 1 KB, as the
// walk's dense-slab loads do; the number of loads in flight per lane and the
// workgroups per CU are arguments, so a caller can take the best of several.
#include <hip/hip_runtime.h>

#include <cstring>

#include "ivf_internal.h"

namespace ivf {
namespace {

constexpr int kProbeThreads = 256;

// U loads of 16 bytes per lane in flight before any is used.
template <int U>
__global__ __launch_bounds__(kProbeThreads) void k_read(const uint4* __restrict__ buf, int64_t n16,
                                                        int64_t per_wg, int64_t stride,
                                                        int32_t passes, int32_t wrap,
                                                        uint4* __restrict__ sink) {
    const int64_t base = ((int64_t)blockIdx.x * stride) % n16;
    uint32_t acc = 0;
    for (int p = 0; p < passes; ++p) {
        for (int64_t i0 = 0; i0 < per_wg; i0 += U * kProbeThreads) {
            uint4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * kProbeThreads + threadIdx.x;
                v[u] = make_uint4(0u, 0u, 0u, 0u);
                int64_t q = base + i;   // base < n16 and i < per_wg <= n16
                if (q >= n16 && wrap) q -= n16;
                if (i < per_wg && q < n16) v[u] = buf[q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
        }
    }
    // a data-dependent store keeps the loads; it almost never happens
    if (acc == 0x9e3779b9u)
        sink[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = make_uint4(acc, 0u, 0u, 0u);
}

hipError_t launch_read(int unroll, unsigned grid, hipStream_t s, const uint4* b4, int64_t n16,
                       int64_t per_wg, int64_t stride, int32_t passes, int32_t wrap,
                       uint4* sink) {
    switch (unroll) {
        case 4: k_read<4><<<grid, kProbeThreads, 0, s>>>(b4, n16, per_wg, stride, passes, wrap, sink); break;
        case 8: k_read<8><<<grid, kProbeThreads, 0, s>>>(b4, n16, per_wg, stride, passes, wrap, sink); break;
        default: k_read<16><<<grid, kProbeThreads, 0, s>>>(b4, n16, per_wg, stride, passes, wrap, sink); break;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace ivf

using namespace ivf;

extern "C" ivf_status ivf_read_ceiling(const void* buf, int64_t bytes, int32_t mode,
                                       int32_t passes, int32_t unroll, int32_t wgs_per_cu,
                                       void* stream, double* gbps) {
    if (!buf || !gbps || bytes < 16 * 1024 || passes < 1 || (mode != 0 && mode != 1) ||
        (unroll != 4 && unroll != 8 && unroll != 16) || wgs_per_cu < 1 || wgs_per_cu > 32)
        return IVF_ERR_ARG;
    *gbps = 0.0;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return IVF_ERR_HIP;
    const int64_t n16 = bytes / 16;
    const int64_t grid = (int64_t)cus * wgs_per_cu;
    int64_t per_wg, stride;
    double moved;
    if (mode == 0) {
        per_wg = n16;
        // rotation: neighbouring workgroups start on different 128-byte lines
        stride = 4104;
        moved = (double)grid * (double)n16 * 16.0 * passes;
    } else {
        per_wg = (n16 + grid - 1) / grid;
        stride = per_wg;
        moved = (double)n16 * 16.0 * passes;
    }
    uint4* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&sink, (size_t)grid * kProbeThreads * sizeof(uint4));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    if (e == hipSuccess) {
        // split mode: the last workgroups may start past the end; they read nothing
        const int64_t g = (mode == 1) ? (n16 + per_wg - 1) / per_wg : grid;
        const uint4* b4 = reinterpret_cast<const uint4*>(buf);
        const int32_t wrap = mode == 0 ? 1 : 0;
        e = launch_read(unroll, (unsigned)g, s, b4, n16, per_wg, stride, passes, wrap, sink);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_read(unroll, (unsigned)g, s, b4, n16, per_wg, stride,
                                             passes, wrap, sink);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? IVF_ERR_OOM : IVF_ERR_HIP;
    *gbps = ms > 0.f ? moved / (ms * 1e-3) / 1e9 : 0.0;
    return IVF_OK;
}
