// TSDF handle, volumetric fusion, layout conversion, PST sampling and the
// particle pose diagnostic of librose.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace rose {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ------------------------------------------------------------------ kernels
template <int FMT>
__global__ __launch_bounds__(256) void k_fill(Grid g, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    store_psi<FMT>(g.psi, (uint32_t)i, 1.0f);
    store_w<FMT>(g.wgt, (uint32_t)i, 0.0f);
}

// A: voxel index -> camera coordinates, binary32 3x4 (see tsdf_integrate).
struct IntegrateArgs {
    Grid g;
    float A[12];
    float fx, fy, cx, cy;
    int32_t W, H;
    const float* depth;
};

// The value store_psi<FMT> leaves in memory for v, decoded (computed here
// rather than read back, which would cost a round trip to memory).
template <int FMT>
__device__ inline float stored_psi(float v) {
    if constexpr (FMT == ROSE_TSDF_F32) {
        return v;
    } else if constexpr (FMT == ROSE_TSDF_F16) {
        return __half2float(__float2half_rn(v));
    } else {
        return (float)(int16_t)rintf(fminf(fmaxf(v, -1.0f), 1.0f) * 32767.0f) * (1.0f / 32767.0f);
    }
}

// One wavefront per 8x8x8 brick (4 per workgroup): lane l takes the voxels
// at in-brick offsets l + 64 m, m = 0..7 (z layer m of the brick), so each
// of its 8 loads and stores covers 64 contiguous voxels.
template <int FMT>
__global__ __launch_bounds__(256) void k_integrate(IntegrateArgs a, uint32_t n_bricks) {
    const Grid& g = a.g;
    const uint32_t b = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (b >= n_bricks) return;  // wave-uniform
    const uint32_t bx = b % (uint32_t)g.nbx;
    const uint32_t by = (b / (uint32_t)g.nbx) % (uint32_t)g.nby;
    const uint32_t bz = b / ((uint32_t)g.nbx * (uint32_t)g.nby);
    const uint32_t lane = threadIdx.x & 63u;
    // A brick that takes no measurement is left at once: its 8 corner voxels
    // all lie behind the camera, or all in front of it and beyond one edge of
    // the image.  Camera coordinates are affine in the voxel index and each
    // condition is a half-space, so every voxel of such a brick (inside the
    // corners' convex hull) fails the per-voxel test below.  The conditions
    // are evaluated in binary64 with margins (1 cm, 2 pixels) far above the
    // rounding of the per-voxel binary32 arithmetic (below 0.1 pixel in
    // front of the 1 cm plane).
    {
        bool behind = false, front = false, left = false, right = false, top = false, bottom = false;
        if (lane < 8) {
            const double ci = (double)(bx * 8 + 7 * (lane & 1u)), cj = (double)(by * 8 + 7 * ((lane >> 1) & 1u)),
                         ck = (double)(bz * 8 + 7 * (lane >> 2));
            const double x = (double)a.A[0] * ci + (double)a.A[1] * cj + (double)a.A[2] * ck + (double)a.A[3];
            const double y = (double)a.A[4] * ci + (double)a.A[5] * cj + (double)a.A[6] * ck + (double)a.A[7];
            const double z = (double)a.A[8] * ci + (double)a.A[9] * cj + (double)a.A[10] * ck + (double)a.A[11];
            behind = z < -0.01;
            front = z > 0.01;
            left = (double)a.fx * x + ((double)a.cx + 2.5) * z < 0.0;
            right = (double)a.fx * x + ((double)a.cx + 0.5 - (double)a.W - 2.0) * z > 0.0;
            top = (double)a.fy * y + ((double)a.cy + 2.5) * z < 0.0;
            bottom = (double)a.fy * y + ((double)a.cy + 0.5 - (double)a.H - 2.0) * z > 0.0;
        }
        auto all8 = [](bool c) { return (__builtin_amdgcn_ballot_w64(c) & 0xffull) == 0xffull; };
        if (all8(behind) || (all8(front) && (all8(left) || all8(right) || all8(top) || all8(bottom)))) return;
    }
    bool not_one = false;
#pragma unroll
    for (uint32_t m = 0; m < 8; ++m) {
        const uint32_t t = lane + 64u * m;
        const uint32_t i = bx * 8 + (t & 7u), j = by * 8 + ((t >> 3) & 7u), k = bz * 8 + m;
        const float fi = (float)i, fj = (float)j, fk = (float)k;
        const float xc = xf_row(a.A[0], a.A[1], a.A[2], a.A[3], fi, fj, fk);
        const float yc = xf_row(a.A[4], a.A[5], a.A[6], a.A[7], fi, fj, fk);
        const float zc = xf_row(a.A[8], a.A[9], a.A[10], a.A[11], fi, fj, fk);
        // `upd` marks the voxels that take this frame's measurement
        bool upd = zc > 0.0f;
        float pu = 0.0f, pv = 0.0f;
        if (upd) {
            pu = floorf(fmaf(a.fx, xc / zc, a.cx) + 0.5f);
            pv = floorf(fmaf(a.fy, yc / zc, a.cy) + 0.5f);
            upd = pu >= 0.0f && pu < (float)a.W && pv >= 0.0f && pv < (float)a.H;
        }
        float D = 0.0f;
        if (upd) {
            D = a.depth[(uint32_t)pv * (uint32_t)a.W + (uint32_t)pu];
            upd = D > 0.0f;
        }
        const float sdf = D - zc;
        upd = upd && !(sdf < -g.mu);
        if (upd) {
            const float d = fminf(1.0f, sdf / g.mu);
            const uint32_t off = (b << 9) | t;
            const float w0 = load_w<FMT>(g.wgt, off);
            const float p0 = load_psi<FMT>(g.psi, off);
            const float v = fmaf(w0, p0, d) / (w0 + 1.0f);
            store_psi<FMT>(g.psi, off, v);
            store_w<FMT>(g.wgt, off, fminf(w0 + 1.0f, g.w_max));
            not_one = not_one || stored_psi<FMT>(v) != 1.0f;
        }
    }
    // a brick with a value other than +1 leaves the all-ones set; bits only
    // ever clear during fusion, so a bit already seen clear needs no atomic
    // (most bricks of the truncation band were cleared by earlier frames)
    if (__builtin_amdgcn_ballot_w64(not_one) != 0ull && lane == 0 && ((g.ones[b >> 5] >> (b & 31u)) & 1u))
        atomicAnd(&g.ones[b >> 5], ~(1u << (b & 31u)));
}

// the all-ones bit of every brick from the stored values (one block per
// brick); words are cleared first by the caller
template <int FMT>
__global__ __launch_bounds__(512) void k_rescan(Grid g) {
    const uint32_t b = blockIdx.x;
    const bool one = load_psi<FMT>(g.psi, (b << 9) | threadIdx.x) == 1.0f;
    if (__syncthreads_and(one) && threadIdx.x == 0) atomicOr(&g.ones[b >> 5], 1u << (b & 31u));
}

__global__ __launch_bounds__(256) void k_clear_words(uint32_t* w, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 0u;
}

template <int FMT>
__global__ __launch_bounds__(256) void k_export(Grid g, float* psi_lin, float* w_lin) {
    const uint64_t n = (uint64_t)g.nx * g.ny * g.nz;
    const uint64_t lin = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lin >= n) return;
    const uint32_t i = (uint32_t)(lin % (uint64_t)g.nx);
    const uint32_t j = (uint32_t)((lin / (uint64_t)g.nx) % (uint64_t)g.ny);
    const uint32_t k = (uint32_t)(lin / ((uint64_t)g.nx * g.ny));
    const uint32_t off = brick_offset(g, i, j, k);
    if (psi_lin) psi_lin[lin] = load_psi<FMT>(g.psi, off);
    if (w_lin) w_lin[lin] = load_w<FMT>(g.wgt, off);
}

template <int FMT>
__global__ __launch_bounds__(256) void k_import(Grid g, const float* psi_lin, const float* w_lin) {
    const uint64_t n = (uint64_t)g.nx * g.ny * g.nz;
    const uint64_t lin = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lin >= n) return;
    const uint32_t i = (uint32_t)(lin % (uint64_t)g.nx);
    const uint32_t j = (uint32_t)((lin / (uint64_t)g.nx) % (uint64_t)g.ny);
    const uint32_t k = (uint32_t)(lin / ((uint64_t)g.nx * g.ny));
    const uint32_t off = brick_offset(g, i, j, k);
    const float p = psi_lin[lin];
    store_psi<FMT>(g.psi, off, p);
    store_w<FMT>(g.wgt, off, w_lin ? w_lin[lin] : (p < 1.0f ? 1.0f : 0.0f));
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds with the
// published multipliers and Weyl key increments.
__device__ inline void philox4x64(uint64_t x[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, x[0]), lo0 = M0 * x[0];
        const uint64_t hi1 = __umul64hi(M1, x[2]), lo1 = M1 * x[2];
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__global__ __launch_bounds__(256) void k_pst_sample(int32_t n, uint64_t seed, float* out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[6] = {0, 0, 0, 0, 0, 0};
    if (i > 0) {
        for (uint64_t a = 0; a < 1024; ++a) {
            uint64_t x[4] = {(uint64_t)i, a, 0, 0};
            philox4x64(x, seed, 0);
            const int64_t m[6] = {(int64_t)(x[0] >> 40), (int64_t)((x[0] >> 16) & 0xFFFFFFull),
                                  (int64_t)(x[1] >> 40), (int64_t)((x[1] >> 16) & 0xFFFFFFull),
                                  (int64_t)(x[2] >> 40), (int64_t)((x[2] >> 16) & 0xFFFFFFull)};
            int64_t s = 0, av[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                av[d] = 2 * m[d] + 1 - (int64_t(1) << 24);
                s += av[d] * av[d];
            }
            if (s <= (int64_t(1) << 48)) {
#pragma unroll
                for (int d = 0; d < 6; ++d) p[d] = (float)av[d] * 0x1p-24f;
                break;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) out[6 * (int64_t)i + d] = p[d];
}

__global__ __launch_bounds__(256) void k_particle_poses(double qc0, double qc1, double qc2, double qc3, double tc0,
                                                        double tc1, double tc2, double r0, double r1, double r2,
                                                        double r3, double r4, double r5, const float* pst,
                                                        int32_t n, double* T) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double qc[4] = {qc0, qc1, qc2, qc3}, tc[3] = {tc0, tc1, tc2}, r[6] = {r0, r1, r2, r3, r4, r5};
    float p[6];
    for (int d = 0; d < 6; ++d) p[d] = pst[6 * (int64_t)i + d];
    double t[12];
    particle_transform(qc, tc, r, p, t);
    for (int e = 0; e < 12; ++e) T[12 * (int64_t)i + e] = t[e];
}

// ------------------------------------------------------------ host helpers
static uint64_t n_voxels(const Grid& g) { return (uint64_t)g.nx * g.ny * g.nz; }
static uint32_t n_bricks(const Grid& g) { return (uint32_t)g.nbx * (uint32_t)g.nby * (uint32_t)g.nbz; }
static uint32_t n_one_words(const Grid& g) { return (n_bricks(g) + 31u) / 32u; }

// rebuild the all-ones bits of every brick from the stored values
static rose_status rescan_ones(const Grid& g, hipStream_t s) {
    const uint32_t w = n_one_words(g), nb = n_bricks(g);
    hipLaunchKernelGGL(k_clear_words, dim3((w + 255) / 256), dim3(256), 0, s, g.ones, w);
    if (g.fmt == ROSE_TSDF_F32) hipLaunchKernelGGL(k_rescan<ROSE_TSDF_F32>, dim3(nb), dim3(512), 0, s, g);
    else if (g.fmt == ROSE_TSDF_F16) hipLaunchKernelGGL(k_rescan<ROSE_TSDF_F16>, dim3(nb), dim3(512), 0, s, g);
    else hipLaunchKernelGGL(k_rescan<ROSE_TSDF_SN16>, dim3(nb), dim3(512), 0, s, g);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // namespace rose

using namespace rose;

extern "C" {

const char* rose_last_error(void) { return g_err; }
const char* rose_version(void) { return "rosehip 0.1 (gfx950)"; }

size_t tsdf_bytes(int32_t nx, int32_t ny, int32_t nz, rose_tsdf_fmt fmt, int32_t which) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 8 || ny % 8 || nz % 8 || nx > 2048 || ny > 2048 || nz > 2048)
        return 0;
    const uint64_t n = (uint64_t)nx * ny * nz;
    if (n > (uint64_t(1) << 31)) return 0;
    if (which != 0 && which != 1) return 0;
    if (fmt == ROSE_TSDF_F32) return (size_t)(n * 4);
    if (fmt == ROSE_TSDF_F16 || fmt == ROSE_TSDF_SN16) return (size_t)(n * 2);
    return 0;
}

rose_status tsdf_create(int32_t nx, int32_t ny, int32_t nz, float voxel_m, float trunc_m, const float origin_m[3],
                        rose_tsdf_fmt fmt, float w_max, void* psi_dev, void* weight_dev, hipStream_t s,
                        rose_tsdf** out) {
    clear_error();
    ROSE_REQUIRE(out != nullptr && origin_m != nullptr && psi_dev != nullptr && weight_dev != nullptr, ROSE_E_ARG,
                 "tsdf_create: NULL argument");
    *out = nullptr;
    ROSE_REQUIRE(fmt == ROSE_TSDF_F32 || fmt == ROSE_TSDF_F16 || fmt == ROSE_TSDF_SN16, ROSE_E_ARG,
                 "tsdf_create: unknown format %d", (int)fmt);
    ROSE_REQUIRE(tsdf_bytes(nx, ny, nz, fmt, 0) != 0, ROSE_E_SHAPE,
                 "tsdf_create: dimensions %dx%dx%d must be positive multiples of 8, each <= 2048, total <= 2^31",
                 nx, ny, nz);
    ROSE_REQUIRE(voxel_m > 0.0f && trunc_m > 0.0f && w_max >= 1.0f, ROSE_E_ARG,
                 "tsdf_create: voxel (%g), truncation (%g) must be > 0 and w_max (%g) >= 1", voxel_m, trunc_m,
                 w_max);
    ROSE_REQUIRE(fmt == ROSE_TSDF_F32 || w_max <= 65535.0f, ROSE_E_ARG, "tsdf_create: w_max > 65535 for u16 weights");
    rose_tsdf* h = (rose_tsdf*)calloc(1, sizeof(rose_tsdf));
    ROSE_REQUIRE(h != nullptr, ROSE_E_DEVICE, "tsdf_create: out of host memory");
    Grid& g = h->g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.nbx = nx / 8; g.nby = ny / 8; g.nbz = nz / 8;
    g.bstride_y = 64 * g.nbx - 8;
    g.bstride_z = 64 * g.nbx * g.nby - 64;
    g.vox = voxel_m; g.mu = trunc_m; g.w_max = w_max;
    g.origin[0] = origin_m[0]; g.origin[1] = origin_m[1]; g.origin[2] = origin_m[2];
    g.fmt = fmt;
    g.psi = psi_dev;
    g.wgt = weight_dev;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        free(h);
        set_error("tsdf_create: hipGetDevice: %s", hipGetErrorString(e));
        return ROSE_E_DEVICE;
    }
    e = hipMalloc((void**)&g.ones, sizeof(uint32_t) * (size_t)n_one_words(g));
    if (e != hipSuccess) {
        free(h);
        set_error("tsdf_create: brick bits (%u words): %s", n_one_words(g), hipGetErrorString(e));
        return ROSE_E_DEVICE;
    }
    const uint64_t n = n_voxels(g);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (fmt == ROSE_TSDF_F32) hipLaunchKernelGGL(k_fill<ROSE_TSDF_F32>, dim3(blocks), dim3(256), 0, s, g, n);
    else if (fmt == ROSE_TSDF_F16) hipLaunchKernelGGL(k_fill<ROSE_TSDF_F16>, dim3(blocks), dim3(256), 0, s, g, n);
    else hipLaunchKernelGGL(k_fill<ROSE_TSDF_SN16>, dim3(blocks), dim3(256), 0, s, g, n);
    e = hipGetLastError();
    if (e != hipSuccess || rescan_ones(g, s) != ROSE_OK) {
        (void)hipFree(g.ones);
        free(h);
        set_error("tsdf_create: fill launch: %s", hipGetErrorString(e));
        return ROSE_E_DEVICE;
    }
    *out = h;
    return ROSE_OK;
}

rose_status tsdf_destroy(rose_tsdf* h) {
    clear_error();
    if (h == nullptr) return ROSE_OK;
    (void)hipDeviceSynchronize();  // kernels in flight may still read the handle's buffers
    if (h->g.ones) (void)hipFree(h->g.ones);
    if (h->pts) (void)hipFree(h->pts);
    if (h->pts_o) (void)hipFree(h->pts_o);
    if (h->partial) (void)hipFree(h->partial);
    if (h->F) (void)hipFree(h->F);
    if (h->st) (void)hipFree(h->st);
    if (h->st_host) (void)hipHostFree(h->st_host);
    if (h->learn_in) (void)hipHostFree(h->learn_in);
    if (h->learn_ok) (void)hipHostFree(h->learn_ok);
    if (h->sw_x) (void)hipFree(h->sw_x);
    if (h->sw_v) (void)hipFree(h->sw_v);
    if (h->sw_p) (void)hipFree(h->sw_p);
    if (h->sw_pF) (void)hipFree(h->sw_pF);
    if (h->sw_C) (void)hipFree(h->sw_C);
    if (h->sw_st) (void)hipFree(h->sw_st);
    if (h->sw_host) (void)hipHostFree(h->sw_host);
    for (int i = 0; i < h->n_orders; ++i) (void)hipFree(h->orders[i].order);
    free(h);
    return ROSE_OK;
}

rose_status tsdf_integrate(rose_tsdf* h, const float* depth_dev, const rose_camera* cam, const rose_pose* T_wc,
                           hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && depth_dev && cam && T_wc, ROSE_E_ARG, "tsdf_integrate: NULL argument");
    ROSE_REQUIRE(cam->width > 0 && cam->height > 0 &&
                     (int64_t)cam->width * cam->height <= (int64_t)ROSE_MAX_IMAGE_PIXELS,
                 ROSE_E_SHAPE, "tsdf_integrate: image %dx%d out of range", cam->width, cam->height);
    ROSE_REQUIRE(cam->fx > 0 && cam->fy > 0, ROSE_E_ARG, "tsdf_integrate: focal lengths must be > 0");
    const Grid& g = h->g;
    // voxel (i,j,k) -> camera: x_c = R^T (origin + (idx + 1/2) vox - t),
    // folded in binary64 as [R^T vox | R^T (origin + vox/2 - t)], rounded once
    double R[9];
    quat_rot(T_wc->q, R);
    IntegrateArgs a;
    a.g = g;
    const double vx = (double)g.vox;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) a.A[4 * r + c] = (float)(R[3 * c + r] * vx);
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) acc += R[3 * c + r] * ((double)g.origin[c] + 0.5 * vx - T_wc->t[c]);
        a.A[4 * r + 3] = (float)acc;
    }
    a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
    a.W = cam->width; a.H = cam->height;
    a.depth = depth_dev;
    const uint32_t nb = n_bricks(g);
    const unsigned blocks = (nb + 3u) / 4u;
    const int tok = prof_begin(PROF_INTEGRATE, s);
    if (g.fmt == ROSE_TSDF_F32) hipLaunchKernelGGL(k_integrate<ROSE_TSDF_F32>, dim3(blocks), dim3(256), 0, s, a, nb);
    else if (g.fmt == ROSE_TSDF_F16) hipLaunchKernelGGL(k_integrate<ROSE_TSDF_F16>, dim3(blocks), dim3(256), 0, s, a, nb);
    else hipLaunchKernelGGL(k_integrate<ROSE_TSDF_SN16>, dim3(blocks), dim3(256), 0, s, a, nb);
    prof_end(tok, s, 0.0);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status tsdf_export(const rose_tsdf* h, float* psi_lin_dev, float* weight_lin_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && (psi_lin_dev || weight_lin_dev), ROSE_E_ARG, "tsdf_export: NULL argument");
    const uint64_t n = n_voxels(h->g);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (h->g.fmt == ROSE_TSDF_F32)
        hipLaunchKernelGGL(k_export<ROSE_TSDF_F32>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev, weight_lin_dev);
    else if (h->g.fmt == ROSE_TSDF_F16)
        hipLaunchKernelGGL(k_export<ROSE_TSDF_F16>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev, weight_lin_dev);
    else
        hipLaunchKernelGGL(k_export<ROSE_TSDF_SN16>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev,
                           weight_lin_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status tsdf_import(rose_tsdf* h, const float* psi_lin_dev, const float* weight_lin_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && psi_lin_dev, ROSE_E_ARG, "tsdf_import: NULL argument");
    const uint64_t n = n_voxels(h->g);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (h->g.fmt == ROSE_TSDF_F32)
        hipLaunchKernelGGL(k_import<ROSE_TSDF_F32>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev, weight_lin_dev);
    else if (h->g.fmt == ROSE_TSDF_F16)
        hipLaunchKernelGGL(k_import<ROSE_TSDF_F16>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev, weight_lin_dev);
    else
        hipLaunchKernelGGL(k_import<ROSE_TSDF_SN16>, dim3(blocks), dim3(256), 0, s, h->g, psi_lin_dev,
                           weight_lin_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return rescan_ones(h->g, s);
}

rose_status tsdf_rescan(rose_tsdf* h, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h, ROSE_E_ARG, "tsdf_rescan: NULL handle");
    return rescan_ones(h->g, s);
}

rose_status tsdf_forget_templates(rose_tsdf* h) {
    clear_error();
    ROSE_REQUIRE(h, ROSE_E_ARG, "tsdf_forget_templates: NULL handle");
    ROSE_CHECK_HIP(hipDeviceSynchronize());  // no launch may still read an order
    for (int i = 0; i < h->n_orders; ++i) {
        if (h->orders[i].order) ROSE_CHECK_HIP(hipFree(h->orders[i].order));
        h->orders[i].order = nullptr;
        h->orders[i].pst = nullptr;
        h->orders[i].n = 0;
    }
    h->n_orders = 0;
    return ROSE_OK;
}

int32_t tsdf_template_orders(const rose_tsdf* h) { return h ? h->n_orders : 0; }

}  // extern "C"

namespace rose {
// rows 0..n-1 of the template (any n >= 1; the Poisson-disk sampler draws
// its candidates from the same stream)
rose_status launch_pst_sample(int64_t n, uint64_t seed, float* out_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_pst_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int32_t)n, seed, out_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}
}  // namespace rose

extern "C" {

rose_status pst_sample(int32_t n, uint64_t seed, float* out_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(out_dev != nullptr, ROSE_E_ARG, "pst_sample: NULL output");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "pst_sample: n = %d out of [1, %d]", n,
                 ROSE_MAX_PARTICLES);
    hipLaunchKernelGGL(k_pst_sample, dim3((n + 255) / 256), dim3(256), 0, s, n, seed, out_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status pst_particle_poses(const rose_pose* c, const double r[6], const float* pst_dev, int32_t n, double* T_dev,
                               hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(c && r && pst_dev && T_dev, ROSE_E_ARG, "pst_particle_poses: NULL argument");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "pst_particle_poses: n = %d out of range", n);
    hipLaunchKernelGGL(k_particle_poses, dim3((n + 255) / 256), dim3(256), 0, s, c->q[0], c->q[1], c->q[2], c->q[3],
                       c->t[0], c->t[1], c->t[2], r[0], r[1], r[2], r[3], r[4], r[5], pst_dev, n, T_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"
