// Gather-rate probe: the roofline of the fitness kernel's TSDF reads.
//
// Every lane issues independent 4-byte loads, each from a pseudo-randomly
// chosen 128-byte line of a working set split into 8 regions, one per XCD
// (workgroups are dealt to the XCDs in turn, so workgroup b reads region
// b mod 8 and each XCD's L2 only sees its own region).  That is the access
// pattern of the fitness gathers -- every lane's voxel in its own cache line
// -- without their address arithmetic; the load rate it reaches with a
// region that fits the L2 is the rate the fitness kernel could reach if
// nothing but its gathers cost time.  A region far larger than the L2 gives
// the same figure for reads served by HBM.
#include "common.h"

namespace rose {

constexpr int kProbeLoads = 8;  // independent loads in flight per lane

__global__ __launch_bounds__(256) void k_gather_peak(const float* buf, uint32_t region_lines, uint32_t iters,
                                                    uint32_t seed, float* sink) {
    const uint32_t xcd = blockIdx.x & 7u;
    const float* region = buf + (uint64_t)xcd * region_lines * 32u;
    const uint32_t mask = region_lines - 1u;
    uint32_t x = (blockIdx.x * 256u + threadIdx.x) * 2654435761u ^ seed;
    float acc = 0.0f;
    for (uint32_t it = 0; it < iters; ++it) {
        float v[kProbeLoads];
#pragma unroll
        for (int u = 0; u < kProbeLoads; ++u) {
            x = x * 1664525u + 1013904223u;  // LCG step (Numerical Recipes constants)
            const uint32_t line = (x >> 8) & mask;
            v[u] = region[line * 32u + (x >> 27)];
        }
#pragma unroll
        for (int u = 0; u < kProbeLoads; ++u) acc += v[u];
    }
    // the loads must not be dead: a store that never happens for real data
    if (acc == -1.0e30f) sink[blockIdx.x] = acc;
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status rose_gather_peak(const float* buf_dev, int64_t buf_elems, int32_t region_lines, int32_t blocks,
                             int32_t iters, uint32_t seed, float* sink_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(buf_dev && sink_dev, ROSE_E_ARG, "rose_gather_peak: NULL argument");
    ROSE_REQUIRE(region_lines >= 1 && region_lines <= (1 << 26) && (region_lines & (region_lines - 1)) == 0,
                 ROSE_E_ARG, "rose_gather_peak: region_lines = %d is not a power of two in [1, 2^26]", region_lines);
    ROSE_REQUIRE((int64_t)8 * region_lines * 32 <= buf_elems, ROSE_E_SHAPE,
                 "rose_gather_peak: 8 regions of %d lines need %lld floats, buffer has %lld", region_lines,
                 (long long)8 * region_lines * 32, (long long)buf_elems);
    ROSE_REQUIRE(blocks >= 8 && blocks % 8 == 0 && blocks <= (1 << 20), ROSE_E_ARG,
                 "rose_gather_peak: blocks = %d must be a positive multiple of 8", blocks);
    ROSE_REQUIRE(iters >= 1, ROSE_E_ARG, "rose_gather_peak: iters must be >= 1");
    hipLaunchKernelGGL(k_gather_peak, dim3(blocks), dim3(256), 0, s, buf_dev, (uint32_t)region_lines, (uint32_t)iters,
                       seed, sink_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

int32_t rose_gather_peak_loads_per_lane(void) { return kProbeLoads; }

}  // extern "C"
