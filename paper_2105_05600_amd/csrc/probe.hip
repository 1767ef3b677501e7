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

// L2 -> CU read bandwidth probe: coalesced 16-byte loads (kStreamLoads in
// flight per lane) sweeping a region per XCD that fits the XCD's L2 and is
// far larger than a CU's L1, so that after the first sweep every load is an
// L1 miss served by the L2.  The workgroups of an XCD start their sweeps at
// staggered offsets.  Its byte rate is the measured peak of L2 -> CU reads
// that bounds any kernel whose data is L2-resident.
constexpr int kStreamLoads = 4;

__global__ __launch_bounds__(256) void k_l2_stream(const float4* buf, uint32_t region_f4, uint32_t sweeps,
                                                  float* sink) {
    const uint32_t xcd = blockIdx.x & 7u;
    const float4* region = buf + (uint64_t)xcd * region_f4;
    const uint32_t mask = region_f4 - 1u;
    const uint32_t start = (blockIdx.x >> 3) * (256u * kStreamLoads * 7u);
    float acc = 0.0f;
    for (uint32_t sw = 0; sw < sweeps; ++sw) {
        for (uint32_t i = 0; i < region_f4; i += 256u * kStreamLoads) {
            float4 v[kStreamLoads];
#pragma unroll
            for (int u = 0; u < kStreamLoads; ++u) v[u] = region[(start + i + (uint32_t)u * 256u + threadIdx.x) & mask];
#pragma unroll
            for (int u = 0; u < kStreamLoads; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        }
    }
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

rose_status rose_l2_read_peak(const float* buf_dev, int64_t buf_elems, int32_t region_f4, int32_t blocks,
                              int32_t sweeps, float* sink_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(buf_dev && sink_dev, ROSE_E_ARG, "rose_l2_read_peak: NULL argument");
    ROSE_REQUIRE(region_f4 >= 1024 && region_f4 <= (1 << 24) && (region_f4 & (region_f4 - 1)) == 0, ROSE_E_ARG,
                 "rose_l2_read_peak: region_f4 = %d is not a power of two in [1024, 2^24]", region_f4);
    ROSE_REQUIRE((int64_t)8 * region_f4 * 4 <= buf_elems, ROSE_E_SHAPE,
                 "rose_l2_read_peak: 8 regions of %d float4 need %lld floats, buffer has %lld", region_f4,
                 (long long)8 * region_f4 * 4, (long long)buf_elems);
    ROSE_REQUIRE(((uintptr_t)buf_dev & 15u) == 0, ROSE_E_ARG, "rose_l2_read_peak: buffer not 16-byte aligned");
    ROSE_REQUIRE(blocks >= 8 && blocks % 8 == 0 && blocks <= (1 << 20), ROSE_E_ARG,
                 "rose_l2_read_peak: blocks = %d must be a positive multiple of 8", blocks);
    ROSE_REQUIRE(sweeps >= 1, ROSE_E_ARG, "rose_l2_read_peak: sweeps must be >= 1");
    hipLaunchKernelGGL(k_l2_stream, dim3(blocks), dim3(256), 0, s, (const float4*)buf_dev, (uint32_t)region_f4,
                       (uint32_t)sweeps, sink_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"
