// The comparison optimisers of the Sec. 5 ablation of the optimisation
// strategy -- vanilla PFO (Sec. 3.1: Gaussian proposal, likelihood weights of
// Eq. pfolh, resampling) and PSO (inertia-weight, global best) -- on the same
// fitness kernel as PFO with PST.  Particles are free states x in the chart
// at the frame's initial pose c_0 (pose c_0 * Delta(x)), stored as binary32
// 6-vectors in the layout of a PST template, so the fitness kernel builds
// their transforms exactly as it builds template particles (with r = 1).
//
// Per iteration: the fitness kernel and the slice reduction (shared with
// the PST path), one single-workgroup kernel (best state, statistics, the
// resampling weights' prefix sums for PFO, and the overlap set of the next
// iteration from the best state), then one elementwise kernel moving the
// particles (resampling + Gaussian proposal, or the PSO velocity step).
// Random numbers are inputs; the host enqueues the loop and synchronises
// once.
#include <algorithm>
#include <cmath>

#include "track_dev.h"

namespace rose {

enum { SW_PFO = 0, SW_PSO = 1 };

struct SwarmDev {
    double qb[4], tb[3];  // best pose c_0 * Delta(x*)
    float xb[6];          // x*
    float Fb;             // F* (+inf before the first iteration)
    int32_t k;            // iterations done
    int32_t n_overlap[ROSE_MAX_ITERS];
    int32_t best_index[ROSE_MAX_ITERS];
    double rho_best[ROSE_MAX_ITERS];
    double rho_mean[ROSE_MAX_ITERS];
};

struct SwarmArgs {
    DevState* chart;  // chart centre c_0 (r = 1), point and overlap counts
    SwarmDev* sw;
    Cam cam;
    const float4* pts;  // valid points of the frame
    float4* pts_o;      // overlap set of the next iteration
    const float* F;     // fitness of the current iteration
    const float* pst;   // template rows (start only)
    float* x;           // current states
    float* xn;          // next states (PFO)
    float* v;           // velocities (PSO)
    float* p;           // personal bests (PSO)
    float* pF;          // personal best fitness (PSO)
    double* C;          // cumulative weights (PFO)
    double q0[4], t0[3];
    double r_init[6];
    float sigma[6], vmax[6];
    float c1, c2;
    double tau;
    int32_t n, iters, method, flags;
};

// initial particle set x_i = r_init (.) p_i, PSO velocities 0, empty bests
__global__ __launch_bounds__(256) void k_swarm_start(SwarmArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        SwarmDev* sw = a.sw;
        for (int e = 0; e < 4; ++e) sw->qb[e] = a.q0[e];
        for (int e = 0; e < 3; ++e) sw->tb[e] = a.t0[e];
        for (int d = 0; d < 6; ++d) sw->xb[d] = 0.0f;
        sw->Fb = INFINITY;
        sw->k = 0;
    }
    if (i >= a.n) return;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int64_t e = 6 * (int64_t)i + d;
        a.x[e] = (float)(a.r_init[d] * (double)a.pst[e]);
        if (a.method == SW_PSO) {
            a.v[e] = 0.0f;
            a.p[e] = 0.0f;
        }
    }
    if (a.method == SW_PSO) a.pF[i] = INFINITY;
}

// (value, index) minimum with the lower index winning ties
__device__ inline void argmin_merge(float* f, int* i, float of, int oi) {
    if (of < *f || (of == *f && oi < *i)) {
        *f = of;
        *i = oi;
    }
}

// One workgroup: best state and statistics of iteration k; for k + 1 < iters
// the PFO resampling weights' prefix sums and the next overlap set.
__global__ __launch_bounds__(1024) void k_swarm_best(SwarmArgs a, int k) {
    __shared__ float s_f[16];
    __shared__ int s_i[16];
    __shared__ double s_sum[16];
    __shared__ double s_pre[1024];
    __shared__ float A[12];
    __shared__ float s_Fb;
    __shared__ int go_on;
    __shared__ int lds[17];
    DevState* ch = a.chart;
    if (ch->stopped) return;  // the frame has no valid point
    const int n = a.n;
    float fmin = INFINITY;
    int imin = 0x7fffffff;
    double srho = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float f = a.F[i];
        argmin_merge(&fmin, &imin, f, i);
        srho += exp_rho(-(double)f / a.tau);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float of = __shfl_xor(fmin, off, kWave);
        const int oi = __shfl_xor(imin, off, kWave);
        argmin_merge(&fmin, &imin, of, oi);
    }
    srho = wave_sum(srho);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        s_f[wid] = fmin;
        s_i[wid] = imin;
        s_sum[wid] = srho;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float bf = s_f[0];
        int bi = s_i[0];
        double tot = s_sum[0];
        for (int w = 1; w < nw; ++w) {
            argmin_merge(&bf, &bi, s_f[w], s_i[w]);
            tot += s_sum[w];
        }
        SwarmDev* sw = a.sw;
        sw->best_index[k] = -1;
        if (bf < sw->Fb) {
            double u[6];
            sw->Fb = bf;
            for (int d = 0; d < 6; ++d) {
                sw->xb[d] = a.x[6 * (int64_t)bi + d];
                u[d] = (double)sw->xb[d];
            }
            double q[4] = {a.q0[0], a.q0[1], a.q0[2], a.q0[3]}, t[3] = {a.t0[0], a.t0[1], a.t0[2]};
            retract(q, t, u);
            for (int e = 0; e < 4; ++e) sw->qb[e] = q[e];
            for (int e = 0; e < 3; ++e) sw->tb[e] = t[e];
            sw->best_index[k] = bi;
        }
        sw->rho_best[k] = exp_rho(-(double)sw->Fb / a.tau);
        sw->rho_mean[k] = tot / (double)n;
        sw->n_overlap[k] = ch->n_overlap;
        sw->k = k + 1;
        s_Fb = sw->Fb;
        go_on = (k + 1 < a.iters);
        if (go_on) {
            double Tb[12], Ad[12];
            pose_matrix(sw->qb, sw->tb, Tb);
            relative_transform(ch->Tprev, Tb, Ad);
            for (int e = 0; e < 12; ++e) A[e] = (float)Ad[e];
        }
    }
    __syncthreads();
    if (!go_on) return;
    if (a.method == SW_PFO) {
        // C_i = w_0 + .. + w_i, w_i = exp(-(F_i - F*) / tau): contiguous chunks
        // per thread, chunk totals prefixed in thread order
        const double Fb = (double)s_Fb;
        const int chunk = (n + (int)blockDim.x - 1) / (int)blockDim.x;
        const int lo = min(n, (int)threadIdx.x * chunk), hi = min(n, lo + chunk);
        double part = 0.0;
        for (int i = lo; i < hi; ++i) part += exp_rho(-((double)a.F[i] - Fb) / a.tau);
        s_pre[threadIdx.x] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc = 0.0;
            for (int t = 0; t < (int)blockDim.x; ++t) {
                const double c = s_pre[t];
                s_pre[t] = acc;
                acc += c;
            }
        }
        __syncthreads();
        double acc = s_pre[threadIdx.x];
        for (int i = lo; i < hi; ++i) {
            acc += exp_rho(-((double)a.F[i] - Fb) / a.tau);
            a.C[i] = acc;
        }
    }
    const int nO = overlap_compact(a.cam, A, (a.flags & ROSE_FLAG_NO_OVERLAP) != 0, a.pts, ch->n_points, a.pts_o,
                                   lds);
    if (threadIdx.x == 0) ch->n_overlap = nO;
}

// PFO step: systematic resampling (ancestor of slot m = the first i with
// C_i > ((m + u) / n) C_{n-1}, n - 1 if none) and the Gaussian proposal
// x'_m = x_{a_m} + sigma (.) z_m.
__global__ __launch_bounds__(256) void k_pfo_move(SwarmArgs a, const float* z, const float* u_k) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n || a.chart->stopped) return;
    const int n = a.n;
    const double t = (((double)m + (double)*u_k) / (double)n) * a.C[n - 1];
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.C[mid] > t) hi = mid;
        else lo = mid + 1;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const float step = a.sigma[d] * z[6 * (int64_t)m + d];
        a.xn[6 * (int64_t)m + d] = a.x[6 * (int64_t)lo + d] + step;
    }
}

// PSO step: personal best, then v = ((w v + (c1 r1)(p - x)) + (c2 r2)(x* - x))
// clamped to [-vmax, vmax], x = x + v (binary32 in this order).
__global__ __launch_bounds__(256) void k_pso_move(SwarmArgs a, const float* R, float w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n || a.chart->stopped) return;
    const float f = a.F[i];
    const bool better = f < a.pF[i];
    if (better) a.pF[i] = f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int64_t e = 6 * (int64_t)i + d;
        const float x = a.x[e];
        const float p = better ? x : a.p[e];
        if (better) a.p[e] = x;
        const float g = a.sw->xb[d];
        const float t1 = a.c1 * R[12 * (int64_t)i + d], t2 = a.c2 * R[12 * (int64_t)i + 6 + d];
        const float d1 = p - x, d2 = g - x;
        const float aa = t1 * d1, bb = t2 * d2;
        float vv = w * a.v[e];
        vv = vv + aa;
        vv = vv + bb;
        vv = fminf(fmaxf(vv, -a.vmax[d]), a.vmax[d]);
        a.v[e] = vv;
        a.x[e] = x + vv;
    }
}

static bool finite_nonneg(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!(v[i] >= 0.0) || !std::isfinite(v[i])) return false;
    return true;
}

static rose_status swarm_track(rose_tsdf* h, const float* depth_dev, const rose_camera* cam, const float* pst_dev,
                               int32_t n, const rose_swarm_params* p, int method, const float* draws_dev,
                               const float* offsets_dev, rose_track_state* state, rose_swarm_stats* stats,
                               hipStream_t s, const char* who) {
    clear_error();
    ROSE_REQUIRE(h && depth_dev && pst_dev && p && state, ROSE_E_ARG, "%s: NULL argument", who);
    rose_status c = check_cam(cam, who);
    if (c != ROSE_OK) return c;
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "%s: n_particles = %d out of [1, %d]", who, n,
                 ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(p->iters >= 1 && p->iters <= ROSE_MAX_ITERS, ROSE_E_ARG, "%s: iters = %d out of [1, %d]", who,
                 p->iters, ROSE_MAX_ITERS);
    ROSE_REQUIRE(p->stride >= 1, ROSE_E_ARG, "%s: stride must be >= 1", who);
    ROSE_REQUIRE(p->lookup == ROSE_LOOKUP_NEAREST || p->lookup == ROSE_LOOKUP_TRILINEAR, ROSE_E_ARG,
                 "%s: bad lookup", who);
    ROSE_REQUIRE((p->flags & ~(ROSE_FLAG_NO_OVERLAP | ROSE_FLAG_NO_NORMALIZE)) == 0, ROSE_E_ARG,
                 "%s: only ROSE_FLAG_NO_OVERLAP and ROSE_FLAG_NO_NORMALIZE apply", who);
    ROSE_REQUIRE(p->tau > 0.0 && std::isfinite(p->tau), ROSE_E_ARG, "%s: tau must be > 0", who);
    ROSE_REQUIRE(finite_nonneg(p->r_init, 6) && finite_nonneg(p->sigma, 6) && finite_nonneg(p->vmax, 6),
                 ROSE_E_ARG, "%s: r_init, sigma and vmax must be finite and >= 0", who);
    ROSE_REQUIRE(std::isfinite(p->w_start) && std::isfinite(p->w_end) && std::isfinite(p->c1) &&
                     std::isfinite(p->c2),
                 ROSE_E_ARG, "%s: w_start, w_end, c1, c2 must be finite", who);
    ROSE_REQUIRE(p->iters == 1 || draws_dev != nullptr, ROSE_E_ARG, "%s: NULL random draws", who);
    ROSE_REQUIRE(p->iters == 1 || method != SW_PFO || offsets_dev != nullptr, ROSE_E_ARG,
                 "%s: NULL resampling offsets", who);
    if (stats) memset(stats, 0, sizeof(*stats));
    if (!state->tsdf_built) {  // no model to search against: the pose is kept
        state->frame += 1;
        return ROSE_OK;
    }

    const int su = (cam->width + p->stride - 1) / p->stride;
    const int sv = (cam->height + p->stride - 1) / p->stride;
    const int64_t mmax = (int64_t)su * sv;
    int shp_p, shp_u;
    float shp_thr, shp_zref;
    fit_launch_shape(h, p->lookup, &shp_p, &shp_u, &shp_thr, &shp_zref);
    const int splits = choose_splits(n, mmax, h->g.fmt, shp_p);
    rose_status g;
    if ((g = grow(&h->pts, &h->cap_points, mmax)) != ROSE_OK) return g;
    if ((g = grow(&h->pts_o, &h->cap_points_o, mmax)) != ROSE_OK) return g;
    if ((g = grow(&h->partial, &h->cap_partial, (int64_t)n * splits * kPartSub)) != ROSE_OK) return g;
    if ((g = grow(&h->F, &h->cap_particles, (int64_t)n)) != ROSE_OK) return g;
    if (!h->st) ROSE_CHECK_HIP(hipMalloc(&h->st, sizeof(DevState)));
    if (!h->st_host) ROSE_CHECK_HIP(hipHostMalloc(&h->st_host, sizeof(DevState), hipHostMallocDefault));
    if (h->cap_swarm < n || !h->sw_x) {
        int64_t cap = 0;
        if ((g = grow(&h->sw_x, &cap, 12 * (int64_t)n)) != ROSE_OK) return g;
        cap = 0;
        if ((g = grow(&h->sw_v, &cap, 6 * (int64_t)n)) != ROSE_OK) return g;
        cap = 0;
        if ((g = grow(&h->sw_p, &cap, 6 * (int64_t)n)) != ROSE_OK) return g;
        cap = 0;
        if ((g = grow(&h->sw_pF, &cap, (int64_t)n)) != ROSE_OK) return g;
        cap = 0;
        if ((g = grow(&h->sw_C, &cap, (int64_t)n)) != ROSE_OK) return g;
        h->cap_swarm = n;
    }
    if (!h->sw_st) ROSE_CHECK_HIP(hipMalloc(&h->sw_st, sizeof(SwarmDev)));
    if (!h->sw_host) ROSE_CHECK_HIP(hipHostMalloc(&h->sw_host, sizeof(SwarmDev), hipHostMallocDefault));

    // unprojection, chart state (c_0, r = 1) and the overlap set of c_0
    InitStatic ia;
    ia.st = h->st;
    ia.cam = to_cam(cam);
    ia.levels = 1;
    ia.flags = p->flags;
    for (int l = 0; l < ROSE_MAX_LEVELS; ++l) {
        ia.stride[l] = p->stride;
        ia.offset[l] = 0;
    }
    ia.pts = h->pts;
    ia.pts_o = h->pts_o;
    FrameIn fin;
    for (int i = 0; i < 4; ++i) fin.qc[i] = state->pose.q[i];
    for (int i = 0; i < 3; ++i) fin.tc[i] = state->pose.t[i];
    for (int d = 0; d < 6; ++d) fin.r[d] = 1.0;
    pose_matrix(state->pose.q, state->pose.t, fin.Tprev);
    fin.depth = depth_dev;
    fin.active = 1;
    fin.pad = 0;
    if ((g = launch_track_init(ia, fin, s)) != ROSE_OK) return g;

    SwarmArgs sa;
    sa.chart = h->st;
    sa.sw = (SwarmDev*)h->sw_st;
    sa.cam = ia.cam;
    sa.pts = h->pts;
    sa.pts_o = h->pts_o;
    sa.F = h->F;
    sa.pst = pst_dev;
    sa.x = h->sw_x;
    sa.xn = h->sw_x + 6 * (int64_t)n;
    sa.v = h->sw_v;
    sa.p = h->sw_p;
    sa.pF = h->sw_pF;
    sa.C = h->sw_C;
    for (int i = 0; i < 4; ++i) sa.q0[i] = state->pose.q[i];
    for (int i = 0; i < 3; ++i) sa.t0[i] = state->pose.t[i];
    for (int d = 0; d < 6; ++d) {
        sa.r_init[d] = p->r_init[d];
        sa.sigma[d] = (float)p->sigma[d];
        sa.vmax[d] = (float)p->vmax[d];
    }
    sa.c1 = (float)p->c1;
    sa.c2 = (float)p->c2;
    sa.tau = p->tau;
    sa.n = n;
    sa.iters = p->iters;
    sa.method = method;
    sa.flags = p->flags;
    const int eblocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_swarm_start, dim3(eblocks), dim3(256), 0, s, sa);
    ROSE_CHECK_HIP(hipGetLastError());

    FitLaunch fl{};
    fl.g = h->g;
    fl.pts = h->pts_o;
    fl.count_dev = &h->st->n_overlap;
    fl.T32 = nullptr;
    fl.st = h->st;
    fl.lookup = p->lookup;
    fl.partial = h->partial;
    fl.n = n;
    fl.splits = splits;
    fl.shape_p = shp_p;  // no switch: the comparison optimisers keep one shape
    fl.shape_u = shp_u;
    UpdateArgs ua{};
    ua.st = h->st;
    ua.partial = h->partial;
    ua.F = h->F;
    ua.n = n;
    ua.splits = splits;
    ua.flags = p->flags;
    for (int k = 0; k < p->iters; ++k) {
        fl.pst = sa.x;
        if ((g = launch_fitness(fl, s)) != ROSE_OK) return g;
        if ((g = launch_fitness_reduce(ua, s)) != ROSE_OK) return g;
        hipLaunchKernelGGL(k_swarm_best, dim3(1), dim3(1024), 0, s, sa, k);
        ROSE_CHECK_HIP(hipGetLastError());
        if (k + 1 >= p->iters) break;
        if (method == SW_PFO) {
            hipLaunchKernelGGL(k_pfo_move, dim3(eblocks), dim3(256), 0, s, sa, draws_dev + (int64_t)k * n * 6,
                               offsets_dev + k);
            std::swap(sa.x, sa.xn);
        } else {
            // inertia weight of iteration k + 1, linear from w_start to w_end
            const double w = p->w_start + (p->w_end - p->w_start) * (double)k / (double)(p->iters - 1);
            hipLaunchKernelGGL(k_pso_move, dim3(eblocks), dim3(256), 0, s, sa, draws_dev + (int64_t)k * n * 12,
                               (float)w);
        }
        ROSE_CHECK_HIP(hipGetLastError());
    }
    SwarmDev* out = (SwarmDev*)h->sw_host;
    ROSE_CHECK_HIP(hipMemcpyAsync(out, h->sw_st, sizeof(SwarmDev), hipMemcpyDeviceToHost, s));
    ROSE_CHECK_HIP(hipMemcpyAsync(h->st_host, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    ROSE_CHECK_HIP(hipStreamSynchronize(s));
    const DevState& ch = *h->st_host;
    if (ch.n_points == 0) {
        set_error("%s: the frame has no valid depth sample", who);
        return ROSE_E_STATE;
    }
    for (int i = 0; i < 4; ++i) state->pose.q[i] = out->qb[i];
    for (int i = 0; i < 3; ++i) state->pose.t[i] = out->tb[i];
    state->rho = exp_rho(-(double)out->Fb / p->tau);
    state->frame += 1;
    if (stats) {
        stats->iters = out->k;
        stats->n_points = ch.n_points;
        for (int k = 0; k < out->k && k < ROSE_MAX_ITERS; ++k) {
            stats->n_overlap[k] = out->n_overlap[k];
            stats->best_index[k] = out->best_index[k];
            stats->rho_best[k] = out->rho_best[k];
            stats->rho_mean[k] = out->rho_mean[k];
        }
    }
    return ROSE_OK;
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status vanilla_pfo_track_frame(rose_tsdf* h, const float* depth_dev, const rose_camera* cam,
                                    const float* pst_dev, int32_t n_particles, const rose_swarm_params* p,
                                    const float* normals_dev, const float* offsets_dev, rose_track_state* state,
                                    rose_swarm_stats* stats, hipStream_t s) {
    return swarm_track(h, depth_dev, cam, pst_dev, n_particles, p, SW_PFO, normals_dev, offsets_dev, state, stats, s,
                       "vanilla_pfo_track_frame");
}

rose_status plain_pso_track_frame(rose_tsdf* h, const float* depth_dev, const rose_camera* cam, const float* pst_dev,
                                  int32_t n_particles, const rose_swarm_params* p, const float* uniforms_dev,
                                  rose_track_state* state, rose_swarm_stats* stats, hipStream_t s) {
    return swarm_track(h, depth_dev, cam, pst_dev, n_particles, p, SW_PSO, uniforms_dev, nullptr, state, stats, s,
                       "plain_pso_track_frame");
}

}  // extern "C"
