// Inputs of the learned PST proposal: a low-resolution raycast of the TSDF
// at the previous pose and the depth residual against the current frame.
#include "common.h"

namespace rose {

// trilinear psi at voxel-space point h = g - 1/2 (binary64; +1 when any of
// the 8 corners is outside the grid)
template <int FMT>
__device__ inline double trilinear64(const Grid& g, double hx, double hy, double hz) {
    const double h[3] = {hx, hy, hz};
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    int64_t i0[3];
    double f[3];
    for (int c = 0; c < 3; ++c) {
        if (!(h[c] >= 0.0 && h[c] < (double)(n[c] - 1))) return 1.0;
        i0[c] = (int64_t)floor(h[c]);
        if (i0[c] + 1 >= n[c]) return 1.0;
        f[c] = h[c] - (double)i0[c];
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                const uint32_t off =
                    brick_offset(g, (uint32_t)(i0[0] + dx), (uint32_t)(i0[1] + dy), (uint32_t)(i0[2] + dz));
                acc += w * (double)load_psi<FMT>(g.psi, off);
            }
    return acc;
}

struct RaycastArgs {
    Grid g;
    double R[9];
    double t[3];
    int32_t W, H;
    double fx, fy, cx, cy;
    double near_z, far_z, step;
    float* out;
};

// One wavefront per pixel: the fixed-step march of the ray is evaluated 64
// samples at a time, lane j taking sample k = base + j (z = near + k step,
// the same expression as a serial march, so the samples are identical).  A
// crossing at k is a + to - change between samples k-1 and k inside the
// truncation band; sample k-1 comes from the lane below (lane 0 keeps the
// previous chunk's last sample).  The first crossing in step order -- the
// lowest lane of the first chunk that has one -- gives the depth by linear
// interpolation, exactly as a serial march stopping there would.
template <int FMT>
__global__ __launch_bounds__(256) void k_raycast(RaycastArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= (int64_t)a.W * a.H) return;  // whole wavefronts leave together
    const int u = (int)(idx % a.W), v = (int)(idx / a.W);
    const double dc[3] = {((double)u - a.cx) / a.fx, ((double)v - a.cy) / a.fy, 1.0};
    double dw[3];
    for (int i = 0; i < 3; ++i) dw[i] = a.R[3 * i + 0] * dc[0] + a.R[3 * i + 1] * dc[1] + a.R[3 * i + 2] * dc[2];
    const double vox = (double)a.g.vox;
    double carry = 0.0;  // sample base - 1 (from the previous chunk)
    double out = 0.0;
    for (int64_t base = 0;; base += kWave) {
        const int64_t k = base + lane;
        const double z = a.near_z + (double)k * a.step;
        const bool valid = !(z > a.far_z);
        double s = 0.0;
        if (valid) {
            double h[3];
            for (int c = 0; c < 3; ++c) h[c] = (a.t[c] + z * dw[c] - (double)a.g.origin[c]) / vox - 0.5;
            s = trilinear64<FMT>(a.g, h[0], h[1], h[2]);
        }
        double prev = __shfl_up(s, 1, kWave);
        if (lane == 0) prev = carry;
        const bool cross = valid && k >= 1 && prev > 0.0 && s <= 0.0 && prev < 1.0 && s > -1.0;
        const uint64_t hits = __ballot(cross);
        if (hits) {
            const int first = __ffsll((unsigned long long)hits) - 1;
            const double zp = a.near_z + (double)(k - 1) * a.step;
            const double o = zp + a.step * prev / (prev - s);
            out = __shfl(o, first, kWave);
            break;
        }
        // any lane past `far` ends the march (later chunks are all past it)
        if (__ballot(!valid)) break;
        carry = __shfl(s, kWave - 1, kWave);
    }
    if (lane == 0) a.out[idx] = (float)out;
}

struct FeatureArgs {
    const float* depth;
    int32_t W, H;
    const float* render;
    int32_t w, hgt, scale;
    double vel[6];
    int32_t dim;
    float* out;
};

// residual = clamp(D(scale u + scale/2, scale v + scale/2) - render(u, v),
// -0.5, 0.5) where both are valid, else 0; then the 6D velocity; zero pad
__global__ __launch_bounds__(256) void k_features(FeatureArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.dim) return;
    const int npx = a.w * a.hgt;
    float v = 0.0f;
    if (i < npx) {
        const int u = i % a.w, r = i / a.w;
        const int U = a.scale * u + a.scale / 2, V = a.scale * r + a.scale / 2;
        const float d = (U < a.W && V < a.H) ? a.depth[(int64_t)V * a.W + U] : 0.0f;
        const float m = a.render[i];
        if (d > 0.0f && m > 0.0f) v = fminf(0.5f, fmaxf(-0.5f, d - m));
    } else if (i < npx + 6) {
        v = (float)a.vel[i - npx];
    }
    a.out[i] = v;
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status tsdf_raycast(const rose_tsdf* h, const rose_pose* T_wc, const rose_camera* cam, double near_m,
                         double far_m, double step_m, float* depth_out_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && T_wc && cam && depth_out_dev, ROSE_E_ARG, "tsdf_raycast: NULL argument");
    ROSE_REQUIRE(cam->width > 0 && cam->height > 0 && (int64_t)cam->width * cam->height <= 1 << 20, ROSE_E_SHAPE,
                 "tsdf_raycast: image %dx%d out of range (at most 2^20 pixels)", cam->width, cam->height);
    ROSE_REQUIRE(cam->fx > 0 && cam->fy > 0, ROSE_E_ARG, "tsdf_raycast: focal lengths must be > 0");
    ROSE_REQUIRE(near_m > 0 && far_m > near_m && step_m > 0 && (far_m - near_m) / step_m <= 1e6, ROSE_E_ARG,
                 "tsdf_raycast: need 0 < near < far and 0 < step, at most 1e6 steps");
    RaycastArgs a;
    a.g = h->g;
    quat_rot(T_wc->q, a.R);
    for (int i = 0; i < 3; ++i) a.t[i] = T_wc->t[i];
    a.W = cam->width;
    a.H = cam->height;
    a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
    a.near_z = near_m; a.far_z = far_m; a.step = step_m;
    a.out = depth_out_dev;
    const unsigned blocks = (unsigned)((a.W * a.H + 3) / 4);  // 4 pixels (wavefronts) per workgroup
    if (h->g.fmt == ROSE_TSDF_F32) hipLaunchKernelGGL(k_raycast<ROSE_TSDF_F32>, dim3(blocks), dim3(256), 0, s, a);
    else if (h->g.fmt == ROSE_TSDF_F16) hipLaunchKernelGGL(k_raycast<ROSE_TSDF_F16>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_raycast<ROSE_TSDF_SN16>, dim3(blocks), dim3(256), 0, s, a);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status proposal_features(const float* depth_dev, const rose_camera* cam, const float* render_dev,
                              const rose_camera* cam_low, int32_t scale, const double velocity[6], int32_t dim,
                              float* features_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(depth_dev && cam && render_dev && cam_low && velocity && features_dev, ROSE_E_ARG,
                 "proposal_features: NULL argument");
    ROSE_REQUIRE(scale >= 1 && cam->width > 0 && cam->height > 0 && cam_low->width > 0 && cam_low->height > 0,
                 ROSE_E_SHAPE, "proposal_features: bad sizes");
    const int npx = cam_low->width * cam_low->height;
    ROSE_REQUIRE(dim >= npx + 6 && dim <= (1 << 20), ROSE_E_SHAPE, "proposal_features: dim %d < pixels + 6", dim);
    FeatureArgs a;
    a.depth = depth_dev;
    a.W = cam->width;
    a.H = cam->height;
    a.render = render_dev;
    a.w = cam_low->width;
    a.hgt = cam_low->height;
    a.scale = scale;
    for (int i = 0; i < 6; ++i) a.vel[i] = velocity[i];
    a.dim = dim;
    a.out = features_dev;
    hipLaunchKernelGGL(k_features, dim3((dim + 255) / 256), dim3(256), 0, s, a);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"
