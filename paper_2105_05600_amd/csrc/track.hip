// Per-frame PST pose search (Alg. 1 with the implementation choices of
// Sec. 4), run entirely on the device: one small setup kernel, then per
// iteration the fitness kernel (fitness.hip) and a single-workgroup update
// kernel that folds the fitness into the APS sums, applies CompBestState /
// CompAxisLength / MovePST and the corner cases, and compacts the overlap
// set for the next iteration.  The host enqueues the whole loop and
// synchronises once.
#include <algorithm>

#include "track_dev.h"

namespace rose {

// Stride-s unprojection of a frame into pts (8x8-sample tile order,
// order-preserving compaction); returns the number of valid samples.
__device__ int unproject_level(const Cam& cam, const float* depth, int stride, float4* pts, int* lds) {
    const int su = (cam.W + stride - 1) / stride;
    const int sv = (cam.H + stride - 1) / stride;
    const int total = sample_count(su, sv, true);
    int m = 0;
    for (int q0 = 0; q0 < total; q0 += blockDim.x) {
        const int q = q0 + threadIdx.x;
        int keep = 0;
        float4 x = make_float4(0, 0, 0, 0);
        int uu, vv;
        if (q < total && sample_at(q, su, sv, true, &uu, &vv)) {
            const int u = uu * stride, v = vv * stride;
            const float z = depth[(int64_t)v * cam.W + u];
            if (z > 0.0f) {
                keep = 1;
                x = unproject_px(cam, u, v, z);
            }
        }
        int tot;
        const int pos = block_scan_flag(keep, lds, &tot);
        if (keep) pts[m + pos] = x;
        m += tot;
    }
    return m;
}

// Unprojection of the frame at every resolution level, device-state
// initialisation and the first overlap set (level 0).
__device__ void track_init_body(const InitStatic& a, const FrameIn& in) {
    __shared__ int lds[17];
    __shared__ float A[12];
    if (!in.active) {
        if (threadIdx.x == 0) {
            a.st->stopped = 1;
            a.st->k = 0;
            a.st->n_points = -1;
        }
        return;
    }
    __shared__ int lvl_m[ROSE_MAX_LEVELS];
    if (threadIdx.x < ROSE_MAX_LEVELS) lvl_m[threadIdx.x] = 0;
    int m = 0, m_any = 0;
    for (int l = 0; l < a.levels; ++l) {
        const int ml = unproject_level(a.cam, in.depth, a.stride[l], a.pts + a.offset[l], lds);
        if (threadIdx.x == 0) lvl_m[l] = ml;  // read back by thread 0 only
        if (l == 0) m = ml;
        m_any += ml;
    }
    if (threadIdx.x == 0) {
        DevState* s = a.st;
        for (int i = 0; i < 4; ++i) s->qc[i] = in.qc[i];
        for (int i = 0; i < 3; ++i) s->tc[i] = in.tc[i];
        for (int i = 0; i < 6; ++i) s->r[i] = in.r[i];
        for (int i = 0; i < 6; ++i) s->r1[i] = in.r[i];
        for (int i = 0; i < 12; ++i) s->Tprev[i] = in.Tprev[i];
        s->rho_last = 0.5;
        s->thr = 0.0;
        s->k = 0;
        s->stopped = (m_any == 0) ? 1 : 0;
        s->empty_streak = 0;
        s->have_rho = 0;
        s->n_points = m;
        for (int l = 0; l < ROSE_MAX_LEVELS; ++l) s->lvl_points[l] = lvl_m[l];
        s->n_overlap = 0;
        s->status = 0;
        double Tc[12], Ad[12];
        pose_matrix(in.qc, in.tc, Tc);
        relative_transform(in.Tprev, Tc, Ad);
        for (int i = 0; i < 12; ++i) A[i] = (float)Ad[i];
    }
    __syncthreads();
    const int nO = overlap_compact(a.cam, A, (a.flags & ROSE_FLAG_NO_OVERLAP) != 0, a.pts, m, a.pts_o, lds);
    if (threadIdx.x == 0) a.st->n_overlap = nO;
}

__global__ __launch_bounds__(1024) void k_track_init(InitStatic a, FrameIn in) { track_init_body(a, in); }

rose_status launch_track_init(const InitStatic& a, const FrameIn& in, hipStream_t s) {
    hipLaunchKernelGGL(k_track_init, dim3(1), dim3(1024), 0, s, a, in);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

// the batched fitness launches' per-XCD work counters (n_ctr <= 1024) are
// cleared by the kernel that precedes each launch on the stream
__device__ inline void clear_counters(int* ctr, int n_ctr) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n_ctr) ctr[threadIdx.x] = 0;
}

// one workgroup per sequence; the per-frame inputs are read from pinned host
// memory (so that a captured graph replays with new inputs)
__global__ __launch_bounds__(1024) void k_track_init_batch(const InitStatic* a, const FrameIn* in_host, int* ctr,
                                                           int n_ctr) {
    clear_counters(ctr, n_ctr);
    __shared__ FrameIn fin;
    constexpr int kWords = sizeof(FrameIn) / sizeof(uint64_t);
    if (threadIdx.x < kWords)
        ((uint64_t*)&fin)[threadIdx.x] = ((const volatile uint64_t*)&in_host[blockIdx.x])[threadIdx.x];
    __syncthreads();
    track_init_body(a[blockIdx.x], fin);
}

// F_i of every particle from its slice partials (fixed slice order), before
// the update: many workgroups, so the update kernel's single workgroup reads
// n floats instead of n x splits doubles.
// one wavefront per particle i (wave-uniform exits)
__device__ inline void reduce_fitness_body(const UpdateArgs& a, int i) {
    if (i >= a.n || a.st->stopped) return;
    const float f = final_fitness(a, i, a.st->n_overlap);
    if ((threadIdx.x & 63) == 0) a.F[i] = f;
}

// 4 particles per workgroup of 256 threads
constexpr int kReducePerBlock = 256 / kWave;

__global__ __launch_bounds__(256) void k_fitness_reduce(UpdateArgs a) {
    reduce_fitness_body(a, blockIdx.x * kReducePerBlock + (int)(threadIdx.x >> 6));
}

rose_status launch_fitness_reduce(const UpdateArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_fitness_reduce, dim3((a.n + kReducePerBlock - 1) / kReducePerBlock), dim3(256), 0, s, a);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

// one column of workgroups per sequence
__global__ __launch_bounds__(256) void k_fitness_reduce_batch(const UpdateArgs* a) {
    reduce_fitness_body(a[blockIdx.y], blockIdx.x * kReducePerBlock + (int)(threadIdx.x >> 6));
}

__device__ void track_update_body(const UpdateArgs& a) {
    __shared__ int lds[17];
    __shared__ double red[16][9];
    __shared__ float A[12];
    __shared__ int go_on;
    DevState* st = a.st;
    if (st->stopped) return;
    const int nO = st->n_overlap;
    const float F0 = a.F[0];
    // APS threshold rho(s*_{k-1}): the carried Eq. wafit value from k = 2 on;
    // the centre's exact fitness (particle 0) at k = 1 or with
    // ROSE_FLAG_CENTRE_THRESHOLD
    const double centre = exp_rho(-(double)F0 / a.tau);
    const double rho0 = (st->k == 0 || (a.flags & ROSE_FLAG_CENTRE_THRESHOLD)) ? centre : st->thr;
    double r[6];
    for (int d = 0; d < 6; ++d) r[d] = st->r[d];
    // per-thread APS sums: count, sum w, sum w rho, sum w u_d, over the
    // thread's particles i = threadIdx.x + j blockDim.x in increasing j; the
    // loads of 8 of them are issued before their arithmetic (latency)
    double cnt = 0.0, sw = 0.0, swr = 0.0, su[6] = {0, 0, 0, 0, 0, 0};
    constexpr int kAhead = 8;
    const int bd = (int)blockDim.x;
    for (int i0 = threadIdx.x; i0 < a.n; i0 += kAhead * bd) {
        float f[kAhead], pr[kAhead][6];
#pragma unroll
        for (int q = 0; q < kAhead; ++q) {
            const int i = min(i0 + q * bd, a.n - 1);
            f[q] = a.F[i];
#pragma unroll
            for (int d = 0; d < 6; ++d) pr[q][d] = a.pst[6 * (int64_t)i + d];
        }
#pragma unroll
        for (int q = 0; q < kAhead; ++q) {
            if (i0 + q * bd >= a.n) break;
            const double rho = exp_rho(-(double)f[q] / a.tau);
            if (rho > rho0) {
                const double w = rho - rho0;
                cnt += 1.0;
                sw += w;
                swr += w * rho;
#pragma unroll
                for (int d = 0; d < 6; ++d) su[d] += w * (r[d] * (double)pr[q][d]);
            }
        }
    }
    double v9[9] = {cnt, sw, swr, su[0], su[1], su[2], su[3], su[4], su[5]};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int e = 0; e < 9; ++e) v9[e] = wave_sum(v9[e]);
    if (lane == 0)
        for (int e = 0; e < 9; ++e) red[wid][e] = v9[e];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < nw; ++w)
            for (int e = 0; e < 9; ++e) tot[e] += red[w][e];
        const int aps = (int)tot[0];
        const double inv_sqrt6 = 1.0 / sqrt(6.0);
        double rhat[6], rt;
        if (aps > 0) {
            const double W = tot[1];
            double us[6], nv = 0.0;
            for (int d = 0; d < 6; ++d) {
                us[d] = tot[3 + d] / W;
                nv += us[d] * us[d];
            }
            nv = sqrt(nv);
            rt = tot[2] / W;
            // Eq. rsinter; the rescaling ablation keeps one of its two parts
            const double iso = (a.flags & ROSE_FLAG_ANISO_ONLY) ? 1.0 : (1.0 - rt);
            const bool aniso = nv > 0.0 && !(a.flags & ROSE_FLAG_ISO_ONLY);
            for (int d = 0; d < 6; ++d) rhat[d] = iso * (aniso ? fabs(us[d]) / nv : inv_sqrt6) + a.eps;
            retract(st->qc, st->tc, us);
            st->rho_last = rt;
            st->have_rho = 1;
            st->empty_streak = 0;
            if (a.early_stop) {
                bool small = true;
                for (int d = 0; d < 6; ++d) small = small && (fabs(us[d]) < a.stop_tol);
                if (small) st->stopped = 1;
            }
        } else {
            rt = rho0;
            for (int d = 0; d < 6; ++d) rhat[d] = 2.0 * (1.0 - rho0) * inv_sqrt6;
            if (!st->have_rho) st->rho_last = rho0;
            st->empty_streak += 1;
            if (a.early_stop && st->empty_streak >= 2) st->stopped = 1;
        }
        for (int d = 0; d < 6; ++d) st->r[d] = a.beta * r[d] + (1.0 - a.beta) * rhat[d];
        st->thr = (aps > 0) ? rt : rho0;
        const int k = st->k;
        st->aps[k] = aps;
        st->n_overlap_iter[k] = nO;
        st->rho_iter[k] = rt;
        st->rho_centre[k] = centre;
        for (int d = 0; d < 6; ++d) st->r_iter[k][d] = r[d];
        st->k = k + 1;
        if (k == 0)
            for (int d = 0; d < 6; ++d) st->r1[d] = st->r[d];
        if (k + 1 >= a.max_iters) st->stopped = 1;
        go_on = !st->stopped;
        if (go_on) {
            double Tc[12], Ad[12];
            pose_matrix(st->qc, st->tc, Tc);
            relative_transform(st->Tprev, Tc, Ad);
            for (int i = 0; i < 12; ++i) A[i] = (float)Ad[i];
        }
    }
    __syncthreads();
    if (!go_on) return;
    const int nO2 = overlap_compact(a.cam, A, (a.flags & ROSE_FLAG_NO_OVERLAP) != 0, a.pts,
                                    st->lvl_points[a.next_level], a.pts_o, lds);
    if (threadIdx.x == 0) st->n_overlap = nO2;
}

__global__ __launch_bounds__(1024) void k_track_update(UpdateArgs a) { track_update_body(a); }

__global__ __launch_bounds__(1024) void k_track_update_batch(const UpdateArgs* a, int* ctr, int n_ctr) {
    clear_counters(ctr, n_ctr);
    track_update_body(a[blockIdx.x]);
}

// copy every sequence's device state to pinned host memory
__global__ __launch_bounds__(64) void k_track_finish_batch(DevState* const* st, DevState* out_host) {
    const uint32_t* src = (const uint32_t*)st[blockIdx.x];
    uint32_t* dst = (uint32_t*)&out_host[blockIdx.x];
    for (int i = threadIdx.x; i < (int)(sizeof(DevState) / 4); i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------- diagnostic entry kernels
__global__ __launch_bounds__(1024) void k_unproject_only(Cam cam, const float* depth, int32_t stride, int32_t tiled,
                                                         float* pts3, int32_t* count) {
    __shared__ int lds[17];
    const int su = (cam.W + stride - 1) / stride;
    const int sv = (cam.H + stride - 1) / stride;
    const int total = sample_count(su, sv, tiled != 0);
    int m = 0;
    for (int q0 = 0; q0 < total; q0 += blockDim.x) {
        const int q = q0 + threadIdx.x;
        int keep = 0;
        float4 x = make_float4(0, 0, 0, 0);
        int uu, vv;
        if (q < total && sample_at(q, su, sv, tiled != 0, &uu, &vv)) {
            const int u = uu * stride, v = vv * stride;
            const float z = depth[(int64_t)v * cam.W + u];
            if (z > 0.0f) {
                keep = 1;
                x = unproject_px(cam, u, v, z);
            }
        }
        int tot;
        const int pos = block_scan_flag(keep, lds, &tot);
        if (keep) {
            pts3[3 * (int64_t)(m + pos)] = x.x;
            pts3[3 * (int64_t)(m + pos) + 1] = x.y;
            pts3[3 * (int64_t)(m + pos) + 2] = x.z;
        }
        m += tot;
    }
    if (threadIdx.x == 0) *count = m;
}

struct OverlapArgs {
    Cam cam;
    float A[12];
    const float* pts3;
    int32_t m;
    uint8_t* mask;
};

__global__ __launch_bounds__(256) void k_overlap_only(OverlapArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.m) return;
    const float4 x = make_float4(a.pts3[3 * (int64_t)j], a.pts3[3 * (int64_t)j + 1], a.pts3[3 * (int64_t)j + 2], 0.f);
    a.mask[j] = overlap_keep(a.cam, a.A, x) ? 1 : 0;
}

}  // namespace rose

using namespace rose;

// Which kernel of a fitness launch did the work for axis lengths r: 0 when
// the launch has one fixed shape; in the switching mode the footprint test
// that both kernels evaluate on the device (largest translation axis length
// plus the reference depth times the largest rotation axis length, against
// the threshold in voxels): 1 points across the lanes, 2 one particle per
// lane.  The same expression in the same precision as the kernels'.
static int32_t switch_mode(const FitLaunch& L, const double r[6]) {
    const uint64_t bytes = (uint64_t)L.g.nx * L.g.ny * L.g.nz * (L.g.fmt == ROSE_TSDF_F32 ? 4u : 2u);
    if (!(L.pl_thr > 0.0f && L.st && !L.T32 && bytes < (uint64_t(1) << 32))) return 0;
    const double rr = std::max(std::max(r[0], r[1]), r[2]);
    const double rt = std::max(std::max(r[3], r[4]), r[5]);
    return (rt + (double)L.pl_zref * rr) <= (double)L.pl_thr * (double)L.g.vox ? 2 : 1;
}

extern "C" {

rose_status depth_unproject(const float* depth_dev, const rose_camera* cam, int32_t stride, int32_t order,
                            float* pts_dev, int32_t* count_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(depth_dev && pts_dev && count_dev, ROSE_E_ARG, "depth_unproject: NULL argument");
    rose_status c = check_cam(cam, "depth_unproject");
    if (c != ROSE_OK) return c;
    ROSE_REQUIRE(stride >= 1, ROSE_E_ARG, "depth_unproject: stride must be >= 1");
    ROSE_REQUIRE(order == 0 || order == 1, ROSE_E_ARG, "depth_unproject: order must be 0 or 1");
    hipLaunchKernelGGL(k_unproject_only, dim3(1), dim3(1024), 0, s, to_cam(cam), depth_dev, stride, order, pts_dev,
                       count_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status overlap_mask(const float* pts_dev, int32_t m, const rose_pose* centre, const rose_pose* prev,
                         const rose_camera* cam, const float* prev_depth_dev, uint8_t* mask_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(pts_dev && centre && prev && mask_dev, ROSE_E_ARG, "overlap_mask: NULL argument");
    rose_status c = check_cam(cam, "overlap_mask");
    if (c != ROSE_OK) return c;
    ROSE_REQUIRE(m >= 0 && m <= ROSE_MAX_IMAGE_PIXELS, ROSE_E_ARG, "overlap_mask: m out of range");
    if (m == 0) return ROSE_OK;
    OverlapArgs a;
    a.cam = to_cam(cam, prev_depth_dev);
    double Tc[12], Tp[12], Ad[12];
    pose_matrix(centre->q, centre->t, Tc);
    pose_matrix(prev->q, prev->t, Tp);
    relative_transform(Tp, Tc, Ad);
    for (int i = 0; i < 12; ++i) a.A[i] = (float)Ad[i];
    a.pts3 = pts_dev;
    a.m = m;
    a.mask = mask_dev;
    hipLaunchKernelGGL(k_overlap_only, dim3((m + 255) / 256), dim3(256), 0, s, a);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status pso_track_frame(rose_tsdf* h, const float* depth_dev, const float* prev_depth_dev,
                            const rose_camera* cam, const float* pst_dev, int32_t n_particles,
                            const rose_track_params* p, const rose_pose* init_centre, const double* init_r,
                            rose_track_state* state, rose_track_stats* stats, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && depth_dev && pst_dev && p && state, ROSE_E_ARG, "pso_track_frame: NULL argument");
    rose_status c = check_cam(cam, "pso_track_frame");
    if (c != ROSE_OK) return c;
    ROSE_REQUIRE(n_particles >= 1 && n_particles <= ROSE_MAX_PARTICLES, ROSE_E_ARG,
                 "pso_track_frame: n_particles = %d out of [1, %d]", n_particles, ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(p->max_iters >= 1 && p->max_iters <= ROSE_MAX_ITERS, ROSE_E_ARG,
                 "pso_track_frame: max_iters = %d out of [1, %d]", p->max_iters, ROSE_MAX_ITERS);
    ROSE_REQUIRE((p->flags & (ROSE_FLAG_ISO_ONLY | ROSE_FLAG_ANISO_ONLY)) !=
                     (ROSE_FLAG_ISO_ONLY | ROSE_FLAG_ANISO_ONLY),
                 ROSE_E_ARG, "pso_track_frame: ISO_ONLY and ANISO_ONLY exclude each other");
    ROSE_REQUIRE(p->levels >= 0 && p->levels <= ROSE_MAX_LEVELS, ROSE_E_ARG,
                 "pso_track_frame: levels = %d out of [0, %d]", p->levels, ROSE_MAX_LEVELS);
    if (p->levels > 1) {
        for (int l = 0; l < p->levels; ++l) {
            ROSE_REQUIRE(p->level_n[l] >= 1 && p->level_n[l] <= n_particles, ROSE_E_ARG,
                         "pso_track_frame: level %d has %d particles (template has %d)", l, p->level_n[l],
                         n_particles);
            ROSE_REQUIRE(p->level_stride[l] >= 1, ROSE_E_ARG, "pso_track_frame: level %d stride must be >= 1", l);
        }
    } else {
        ROSE_REQUIRE(p->stride >= 1, ROSE_E_ARG, "pso_track_frame: stride must be >= 1");
    }
    ROSE_REQUIRE(p->lookup == ROSE_LOOKUP_NEAREST || p->lookup == ROSE_LOOKUP_TRILINEAR, ROSE_E_ARG,
                 "pso_track_frame: bad lookup");
    ROSE_REQUIRE(!(p->flags & ROSE_FLAG_NO_KAHAN) ||
                     (h->g.fmt == ROSE_TSDF_F32 &&
                      (uint64_t)h->g.nx * h->g.ny * h->g.nz * 4u < (uint64_t(1) << 32)),
                 ROSE_E_UNSUPPORTED, "pso_track_frame: ROSE_FLAG_NO_KAHAN needs a binary32 volume below 4 GB");
    ROSE_REQUIRE(p->tau > 0.0 && p->beta >= 0.0 && p->beta <= 1.0, ROSE_E_ARG,
                 "pso_track_frame: tau must be > 0 and beta in [0, 1]");
    const double* r0 = init_r ? init_r : state->r;
    const rose_pose* c0 = init_centre ? init_centre : &state->pose;

    if (!state->tsdf_built) {
        // Sec. 4, first corner case: no fitness; rhat = 0.5 * 1, pose kept
        for (int d = 0; d < 6; ++d) state->r[d] = p->beta * r0[d] + (1.0 - p->beta) * 0.5;
        state->pose = *c0;
        state->rho = 0.5;
        state->frame += 1;
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->iters = 1;
            stats->rho_iter[0] = 0.5;
        }
        return ROSE_OK;
    }

    // resolution levels: one (n_particles, stride), or the schedule
    const int L = p->levels > 1 ? p->levels : 1;
    int lv_n[ROSE_MAX_LEVELS], lv_splits[ROSE_MAX_LEVELS];
    int64_t lv_off[ROSE_MAX_LEVELS + 1];
    InitStatic ia;
    ia.levels = L;
    lv_off[0] = 0;
    int64_t mmax_all = 0, partial_need = 0;
    for (int l = 0; l < ROSE_MAX_LEVELS; ++l) {
        ia.stride[l] = 1;
        ia.offset[l] = 0;
    }
    int shp_p, shp_u;
    float shp_thr, shp_zref;
    fit_launch_shape(h, p->lookup, &shp_p, &shp_u, &shp_thr, &shp_zref);
    for (int l = 0; l < L; ++l) {
        const int st_l = L > 1 ? p->level_stride[l] : p->stride;
        lv_n[l] = L > 1 ? p->level_n[l] : n_particles;
        const int su = (cam->width + st_l - 1) / st_l;
        const int sv = (cam->height + st_l - 1) / st_l;
        const int64_t mmax = (int64_t)su * sv;
        lv_splits[l] = choose_splits(lv_n[l], mmax, h->g.fmt, shp_p);
        lv_off[l + 1] = lv_off[l] + mmax;
        mmax_all = std::max(mmax_all, mmax);
        partial_need = std::max(partial_need, (int64_t)lv_n[l] * lv_splits[l] * kPartSub);
        ia.stride[l] = st_l;
        ia.offset[l] = (int32_t)lv_off[l];
    }
    rose_status g;
    if ((g = grow(&h->pts, &h->cap_points, lv_off[L])) != ROSE_OK) return g;
    if ((g = grow(&h->pts_o, &h->cap_points_o, mmax_all)) != ROSE_OK) return g;
    if ((g = grow(&h->partial, &h->cap_partial, partial_need)) != ROSE_OK) return g;
    if ((g = grow(&h->F, &h->cap_particles, (int64_t)n_particles)) != ROSE_OK) return g;
    if (!h->st) ROSE_CHECK_HIP(hipMalloc(&h->st, sizeof(DevState)));
    if (!h->st_host) ROSE_CHECK_HIP(hipHostMalloc(&h->st_host, sizeof(DevState), hipHostMallocDefault));

    ia.st = h->st;
    ia.cam = to_cam(cam, prev_depth_dev);
    ia.flags = p->flags;
    ia.pts = h->pts;
    ia.pts_o = h->pts_o;
    FrameIn fin;
    for (int i = 0; i < 4; ++i) fin.qc[i] = c0->q[i];
    for (int i = 0; i < 3; ++i) fin.tc[i] = c0->t[i];
    for (int i = 0; i < 6; ++i) fin.r[i] = r0[i];
    pose_matrix(state->pose.q, state->pose.t, fin.Tprev);
    fin.depth = depth_dev;
    fin.active = 1;
    fin.pad = 0;
    // schedule order of each level's particles (first use: reads the template)
    const int32_t* lv_order[ROSE_MAX_LEVELS] = {nullptr, nullptr, nullptr, nullptr};
    for (int l = 0; l < L; ++l)
        if ((g = particle_order(h, pst_dev, lv_n[l], s, &lv_order[l])) != ROSE_OK) return g;
    hipLaunchKernelGGL(k_track_init, dim3(1), dim3(1024), 0, s, ia, fin);
    ROSE_CHECK_HIP(hipGetLastError());

    FitLaunch fl{};
    fl.g = h->g;
    fl.pts = h->pts_o;
    fl.count_dev = &h->st->n_overlap;
    fl.T32 = nullptr;
    fl.st = h->st;
    fl.pst = pst_dev;
    fl.lookup = p->lookup;
    fl.partial = h->partial;
    fl.acc32 = (p->flags & ROSE_FLAG_NO_KAHAN) ? 1 : 0;
    fl.shape_p = shp_p;
    fl.shape_u = shp_u;
    fl.pl_thr = shp_thr;
    fl.pl_zref = shp_zref;

    UpdateArgs ua{};
    ua.st = h->st;
    ua.cam = ia.cam;
    ua.pst = pst_dev;
    ua.partial = h->partial;
    ua.F = h->F;
    ua.pts_o = h->pts_o;
    ua.max_iters = p->max_iters;
    ua.early_stop = p->early_stop;
    ua.flags = p->flags;
    ua.beta = p->beta;
    ua.eps = p->eps;
    ua.tau = p->tau;
    ua.stop_tol = p->stop_tol;
    int tok_fit[ROSE_MAX_ITERS];
    for (int k = 0; k < p->max_iters; ++k) {
        // iteration k + 1 runs level k mod L and prepares level (k + 1) mod L
        const int l = k % L, ln = (k + 1) % L;
        fl.n = lv_n[l];
        fl.order = lv_order[l];
        fl.splits = lv_splits[l];
        ua.n = lv_n[l];
        ua.splits = lv_splits[l];
        ua.pts = h->pts + lv_off[ln];
        ua.next_level = ln;
        tok_fit[k] = prof_begin(PROF_FITNESS, s);
        if ((g = launch_fitness(fl, s)) != ROSE_OK) return g;
        prof_end(tok_fit[k], s, 0.0);
        const int tu = prof_begin(PROF_UPDATE, s);
        hipLaunchKernelGGL(k_fitness_reduce, dim3((ua.n + kReducePerBlock - 1) / kReducePerBlock), dim3(256), 0, s,
                           ua);
        hipLaunchKernelGGL(k_track_update, dim3(1), dim3(1024), 0, s, ua);
        prof_end(tu, s, 0.0);
        ROSE_CHECK_HIP(hipGetLastError());
    }
    ROSE_CHECK_HIP(hipMemcpyAsync(h->st_host, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    ROSE_CHECK_HIP(hipStreamSynchronize(s));
    const DevState& r = *h->st_host;
    for (int k = 0; k < p->max_iters; ++k)
        prof_set_evals(tok_fit[k], k < r.k ? (double)lv_n[k % L] * (double)r.n_overlap_iter[k] : 0.0);
    int64_t any = 0;
    for (int l = 0; l < L; ++l) any += r.lvl_points[l];
    if (any == 0) {
        set_error("pso_track_frame: the frame has no valid depth sample");
        return ROSE_E_STATE;
    }
    for (int i = 0; i < 4; ++i) state->pose.q[i] = r.qc[i];
    for (int i = 0; i < 3; ++i) state->pose.t[i] = r.tc[i];
    for (int d = 0; d < 6; ++d) state->r[d] = r.r1[d];
    state->rho = r.rho_last;
    state->frame += 1;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->iters = r.k;
        stats->n_points = r.n_points;
        stats->n_overlap_last = r.n_overlap;
        for (int k = 0; k < r.k && k < ROSE_MAX_ITERS; ++k) {
            stats->aps_size[k] = r.aps[k];
            stats->n_overlap[k] = r.n_overlap_iter[k];
            stats->rho_iter[k] = r.rho_iter[k];
            stats->rho_centre[k] = r.rho_centre[k];
            for (int d = 0; d < 6; ++d) stats->r_iter[k][d] = r.r_iter[k][d];
            stats->n_particles[k] = lv_n[k % L];
            stats->fit_mode[k] = switch_mode(fl, r.r_iter[k]);
        }
    }
    return ROSE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batching
// Many sequences tracked in lockstep: per frame step one init launch (one
// workgroup per sequence), then per iteration one persistent fitness launch
// per group over the small sequences' work, the fitness launches of each
// large switching-mode sequence (the single path's), one slice-reduction
// launch and one update launch (one workgroup per sequence), then one
// launch copying the states to pinned host memory.  The
// sequence of launches is captured once into a HIP graph and replayed every
// frame step; per-frame inputs are read by the init kernel from pinned host
// memory, so the graph itself never changes.
#include <vector>

// sequences of one storage format and lookup: one fitness launch each
// The learned PST proposal from the network outputs o (12 per sequence: the
// chart offset mu, then the log axis lengths l): c_0 = s * Delta(mu) (the
// chart retraction of the pose s held in in[i].qc, in[i].tc on entry) and
// r_0 = clamp(kappa exp(l), r_min, r_max), written over in[i] (pinned host
// memory read by the tracker's init kernel or by the host).  A sequence
// whose outputs are not all finite keeps its pose and axis lengths and is
// flagged ok[i] = 0.  One thread per sequence.
__global__ __launch_bounds__(64) void k_learned_proposal(const float* o, int32_t n, FrameIn* in, int32_t* ok,
                                                         double kappa, double r_min, double r_max) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* oi = o + 12 * (int64_t)i;
    bool fin = true;
    for (int e = 0; e < 12; ++e) fin = fin && isfinite(oi[e]);
    ok[i] = fin ? 1 : 0;
    if (!fin || !in[i].active) return;
    double mu[6], q[4], t[3];
    for (int d = 0; d < 6; ++d) mu[d] = (double)oi[d];
    for (int e = 0; e < 4; ++e) q[e] = in[i].qc[e];
    for (int e = 0; e < 3; ++e) t[e] = in[i].tc[e];
    retract(q, t, mu);
    for (int e = 0; e < 4; ++e) in[i].qc[e] = q[e];
    for (int e = 0; e < 3; ++e) in[i].tc[e] = t[e];
    for (int d = 0; d < 6; ++d) in[i].r[d] = fmin(r_max, fmax(r_min, kappa * exp_rho((double)oi[6 + d])));
}

struct BatchGroup {
    int fmt, lk;
    int first, count;  // positions in the group-ordered work arrays
    int base, end;     // work items [base, end)
    int grid;
};

// Sequences in the switching mode whose iteration holds at least this many
// particle x point evaluations (n_particles x the points at the stride) take
// launches of their own in a batch; read when a batch is created.
static int64_t g_batch_own_min = int64_t(1) << 23;

struct rose_batch {
    int32_t count = 0, K = 0, P = 4, U = 2, total = 0, max_n = 1;
    std::vector<BatchGroup> groups;
    // sequences with launches of their own (the single path's fitness
    // launches, switching included), and those launch records
    std::vector<int> own;
    std::vector<FitLaunch> own_fl;
    std::vector<int> own_of;  // per sequence: its index in own, or -1
    bool use_graph = true;
    std::vector<rose_tsdf*> h;
    std::vector<rose_camera> cams;
    std::vector<rose_track_params> params;
    std::vector<int32_t> n;
    FitLaunch* fit_dev = nullptr;
    int* begin_dev = nullptr;
    int* ctr_dev = nullptr;  // 8 work counters per group
    InitStatic* init_dev = nullptr;
    UpdateArgs* upd_dev = nullptr;
    DevState** stp_dev = nullptr;
    FrameIn* in_host = nullptr;
    DevState* out_host = nullptr;
    int32_t* prop_ok = nullptr;  // pinned: the learned proposal's finite flag per sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    // host copies of the per-sequence launch records (fit in group order: pos)
    std::vector<FitLaunch> fit_host;
    std::vector<InitStatic> init_host;
    std::vector<UpdateArgs> upd_host;
    std::vector<int> pos;
};

// The launch records hold each handle's scratch pointers.  A handle tracked
// through another path (the learned step's plain fallback) may have grown,
// i.e. reallocated, its scratch since; rewrite the records from the handles
// and upload them (the captured graph reads them at execution).  Call outside
// stream capture.
static rose_status batch_refresh(rose_batch* b, bool force) {
    bool stale = force;
    for (int i = 0; i < b->count && !stale; ++i) {
        const rose_tsdf* h = b->h[i];
        const UpdateArgs& u = b->upd_host[i];
        stale = u.partial != h->partial || u.F != h->F || u.pts != h->pts || u.pts_o != h->pts_o || u.st != h->st;
    }
    if (!stale) return ROSE_OK;
    for (size_t j = 0; j < b->own.size(); ++j) {
        const rose_tsdf* h = b->h[b->own[j]];
        FitLaunch& L = b->own_fl[j];
        L.pts = h->pts_o;
        L.count_dev = &h->st->n_overlap;
        L.st = h->st;
        L.partial = h->partial;
    }
    // a captured graph holds the own launches' records by value: capture again
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (int i = 0; i < b->count; ++i) {
        rose_tsdf* h = b->h[i];
        FitLaunch& L = b->fit_host[b->pos[i]];
        L.pts = h->pts_o;
        L.count_dev = &h->st->n_overlap;
        L.st = h->st;
        L.partial = h->partial;
        InitStatic& ia = b->init_host[i];
        ia.st = h->st;
        ia.pts = h->pts;
        ia.pts_o = h->pts_o;
        UpdateArgs& ua = b->upd_host[i];
        ua.st = h->st;
        ua.partial = h->partial;
        ua.F = h->F;
        ua.pts = h->pts;
        ua.pts_o = h->pts_o;
    }
    const size_t n = (size_t)b->count;
    ROSE_CHECK_HIP(hipMemcpy(b->fit_dev, b->fit_host.data(), sizeof(FitLaunch) * n, hipMemcpyHostToDevice));
    ROSE_CHECK_HIP(hipMemcpy(b->init_dev, b->init_host.data(), sizeof(InitStatic) * n, hipMemcpyHostToDevice));
    ROSE_CHECK_HIP(hipMemcpy(b->upd_dev, b->upd_host.data(), sizeof(UpdateArgs) * n, hipMemcpyHostToDevice));
    std::vector<DevState*> stp(n);
    for (size_t i = 0; i < n; ++i) stp[i] = b->h[i]->st;
    ROSE_CHECK_HIP(hipMemcpy(b->stp_dev, stp.data(), sizeof(DevState*) * n, hipMemcpyHostToDevice));
    return ROSE_OK;
}

static void batch_free(rose_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->fit_dev) (void)hipFree(b->fit_dev);
    if (b->begin_dev) (void)hipFree(b->begin_dev);
    if (b->ctr_dev) (void)hipFree(b->ctr_dev);
    if (b->init_dev) (void)hipFree(b->init_dev);
    if (b->upd_dev) (void)hipFree(b->upd_dev);
    if (b->stp_dev) (void)hipFree(b->stp_dev);
    if (b->in_host) (void)hipHostFree(b->in_host);
    if (b->out_host) (void)hipHostFree(b->out_host);
    if (b->prop_ok) (void)hipHostFree(b->prop_ok);
    delete b;
}

static rose_status batch_enqueue(rose_batch* b, hipStream_t s) {
    // every group's counters are cleared before each round of fitness launches
    // (by the init kernel, then by each update kernel); each group has its own
    // 8 counters, so the launches of one round do not disturb each other
    const int n_ctr = 8 * (int)b->groups.size();
    hipLaunchKernelGGL(k_track_init_batch, dim3(b->count), dim3(1024), 0, s, b->init_dev, b->in_host, b->ctr_dev,
                       n_ctr);
    ROSE_CHECK_HIP(hipGetLastError());
    for (int k = 0; k < b->K; ++k) {
        for (size_t q = 0; q < b->groups.size(); ++q) {
            const BatchGroup& gr = b->groups[q];
            rose_status st = launch_fitness_batch(b->fit_dev + gr.first, b->begin_dev + gr.first, gr.count, gr.base,
                                                  gr.end, gr.grid, b->P, b->U, gr.fmt, gr.lk, b->ctr_dev + 8 * q, s);
            if (st != ROSE_OK) return st;
        }
        for (const FitLaunch& L : b->own_fl) {
            rose_status st = launch_fitness(L, s);
            if (st != ROSE_OK) return st;
        }
        hipLaunchKernelGGL(k_fitness_reduce_batch, dim3((b->max_n + kReducePerBlock - 1) / kReducePerBlock, b->count),
                           dim3(256), 0, s,
                           b->upd_dev);
        hipLaunchKernelGGL(k_track_update_batch, dim3(b->count), dim3(1024), 0, s, b->upd_dev, b->ctr_dev, n_ctr);
        ROSE_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_track_finish_batch, dim3(b->count), dim3(64), 0, s, b->stp_dev, b->out_host);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

static rose_status batch_track_impl(rose_batch* b, const float* const* depth_devs, const rose_pose* init_centres,
                                    const double* init_rs, const float* prop_dev, const rose_learned_params* lp,
                                    rose_track_state* states, rose_track_stats* stats, hipStream_t s);

extern "C" {

rose_status pso_batch_create(int32_t count, rose_tsdf* const* tsdfs, const rose_camera* cams,
                             const float* const* pst_devs, const int32_t* n_particles,
                             const rose_track_params* params, int32_t use_graph, rose_batch** out) {
    clear_error();
    ROSE_REQUIRE(out && tsdfs && cams && pst_devs && n_particles && params, ROSE_E_ARG,
                 "pso_batch_create: NULL argument");
    *out = nullptr;
    ROSE_REQUIRE(count >= 1 && count <= 4096, ROSE_E_ARG, "pso_batch_create: count = %d out of [1, 4096]", count);
    for (int i = 0; i < count; ++i) {
        ROSE_REQUIRE(tsdfs[i] && pst_devs[i], ROSE_E_ARG, "pso_batch_create: NULL handle or template %d", i);
        rose_status c = check_cam(&cams[i], "pso_batch_create");
        if (c != ROSE_OK) return c;
        ROSE_REQUIRE(n_particles[i] >= 1 && n_particles[i] <= ROSE_MAX_PARTICLES, ROSE_E_ARG,
                     "pso_batch_create: n_particles[%d] = %d out of range", i, n_particles[i]);
        const rose_track_params& p = params[i];
        ROSE_REQUIRE(p.max_iters >= 1 && p.max_iters <= ROSE_MAX_ITERS && p.stride >= 1 &&
                         (p.lookup == ROSE_LOOKUP_NEAREST || p.lookup == ROSE_LOOKUP_TRILINEAR) && p.tau > 0.0 &&
                         p.beta >= 0.0 && p.beta <= 1.0,
                     ROSE_E_ARG, "pso_batch_create: bad parameters for sequence %d", i);
        ROSE_REQUIRE((p.flags & (ROSE_FLAG_ISO_ONLY | ROSE_FLAG_ANISO_ONLY)) !=
                         (ROSE_FLAG_ISO_ONLY | ROSE_FLAG_ANISO_ONLY),
                     ROSE_E_ARG, "pso_batch_create: ISO_ONLY and ANISO_ONLY exclude each other (sequence %d)", i);
        ROSE_REQUIRE(p.levels <= 1, ROSE_E_UNSUPPORTED,
                     "pso_batch_create: multi-resolution schedules are not batched (sequence %d)", i);
        const uint64_t bytes =
            (uint64_t)tsdfs[i]->g.nx * tsdfs[i]->g.ny * tsdfs[i]->g.nz * (tsdfs[i]->g.fmt == ROSE_TSDF_F32 ? 4u : 2u);
        ROSE_REQUIRE(bytes < (uint64_t(1) << 32), ROSE_E_UNSUPPORTED,
                     "pso_batch_create: volume %d is 4 GB or larger (use pso_track_frame)", i);
        ROSE_REQUIRE(!(params[i].flags & ROSE_FLAG_NO_KAHAN), ROSE_E_UNSUPPORTED,
                     "pso_batch_create: ROSE_FLAG_NO_KAHAN is not batched (sequence %d)", i);
        for (int j = 0; j < i; ++j)
            ROSE_REQUIRE(tsdfs[j] != tsdfs[i], ROSE_E_ARG, "pso_batch_create: handle %d repeated", i);
    }
    rose_batch* b = new rose_batch();
    b->count = count;
    b->use_graph = use_graph != 0;
    // the first handle's launch configuration: its fixed shape, or in the
    // switching mode its points-across shape (the batch does not switch)
    const FitConfig cfg = fit_config(tsdfs[0]);
    int P = cfg.sw ? cfg.wide_p : cfg.p, U = cfg.sw ? cfg.wide_u : cfg.u;
    if (!batch_shape_valid(P, U)) {
        P = 4;
        U = 2;
    }
    b->P = P;
    b->U = U;
    // sequences in the switching mode with enough work per iteration to fill
    // the GPU alone take the single path's fitness launches (both kernels,
    // chosen on the device); the rest share the persistent launches
    const int64_t own_min = g_batch_own_min;
    std::vector<char> own(count, 0);
    for (int i = 0; i < count; ++i) {
        int sp, su;
        float thr, zref;
        fit_launch_shape(tsdfs[i], params[i].lookup, &sp, &su, &thr, &zref);
        const int64_t mm = (int64_t)((cams[i].width + params[i].stride - 1) / params[i].stride) *
                           ((cams[i].height + params[i].stride - 1) / params[i].stride);
        own[i] = thr > 0.0f && (int64_t)n_particles[i] * mm >= own_min;
    }
    // the fitness work arrays list the sequences grouped by (format, lookup),
    // the sequences with launches of their own last (in no group)
    auto group_key = [&](int x) { return own[x] ? 1 << 20 : tsdfs[x]->g.fmt * 2 + params[x].lookup; };
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return group_key(x) < group_key(y); });
    b->own_of.assign(count, -1);
    std::vector<int> pos(count);
    for (int k = 0; k < count; ++k) pos[order[k]] = k;
    std::vector<FitLaunch> fit(count);
    std::vector<int> nblk(count, 0);
    std::vector<InitStatic> init(count);
    std::vector<UpdateArgs> upd(count);
    std::vector<DevState*> stp(count);
    rose_status g = ROSE_OK;
    for (int i = 0; i < count && g == ROSE_OK; ++i) {
        rose_tsdf* h = tsdfs[i];
        const rose_track_params& p = params[i];
        const int su = (cams[i].width + p.stride - 1) / p.stride;
        const int sv = (cams[i].height + p.stride - 1) / p.stride;
        const int64_t mmax = (int64_t)su * sv;
        int shp_p = P, shp_u = U;
        float shp_thr = 0.0f, shp_zref = 0.0f;
        if (own[i]) fit_launch_shape(h, p.lookup, &shp_p, &shp_u, &shp_thr, &shp_zref);
        const int splits = choose_splits(n_particles[i], mmax, h->g.fmt, shp_p);
        if ((g = grow(&h->pts, &h->cap_points, mmax)) != ROSE_OK) break;
        if ((g = grow(&h->pts_o, &h->cap_points_o, mmax)) != ROSE_OK) break;
        if ((g = grow(&h->partial, &h->cap_partial, (int64_t)n_particles[i] * splits * kPartSub)) != ROSE_OK) break;
        if ((g = grow(&h->F, &h->cap_particles, (int64_t)n_particles[i])) != ROSE_OK) break;
        if (!h->st && hipMalloc(&h->st, sizeof(DevState)) != hipSuccess) {
            set_error("pso_batch_create: hipMalloc failed");
            g = ROSE_E_DEVICE;
            break;
        }
        FitLaunch& L = fit[pos[i]];
        L = FitLaunch{};
        L.g = h->g;
        L.pts = h->pts_o;
        L.count_dev = &h->st->n_overlap;
        L.T32 = nullptr;
        L.st = h->st;
        L.pst = pst_devs[i];
        L.n = n_particles[i];
        if ((g = particle_order(h, pst_devs[i], n_particles[i], nullptr, &L.order)) != ROSE_OK) break;
        L.splits = splits;
        L.lookup = p.lookup;
        L.shape_p = shp_p;
        L.shape_u = shp_u;
        L.pl_thr = shp_thr;
        L.pl_zref = shp_zref;
        L.partial = h->partial;
        nblk[pos[i]] = own[i] ? 0 : fitness_blocks(L, P);
        if (own[i]) {
            b->own_of[i] = (int)b->own.size();
            b->own.push_back(i);
            b->own_fl.push_back(L);
        }
        InitStatic& ia = init[i];
        ia = InitStatic{};
        ia.st = h->st;
        ia.cam = to_cam(&cams[i]);
        ia.levels = 1;
        ia.flags = p.flags;
        for (int l = 0; l < ROSE_MAX_LEVELS; ++l) ia.stride[l] = p.stride;
        ia.pts = h->pts;
        ia.pts_o = h->pts_o;
        UpdateArgs& ua = upd[i];
        ua.st = h->st;
        ua.cam = to_cam(&cams[i]);
        ua.pst = pst_devs[i];
        ua.partial = h->partial;
        ua.F = h->F;
        ua.pts = h->pts;
        ua.pts_o = h->pts_o;
        ua.next_level = 0;
        ua.n = n_particles[i];
        ua.splits = splits;
        ua.max_iters = p.max_iters;
        ua.early_stop = p.early_stop;
        ua.flags = p.flags;
        ua.beta = p.beta;
        ua.eps = p.eps;
        ua.tau = p.tau;
        ua.stop_tol = p.stop_tol;
        stp[i] = h->st;
        b->h.push_back(h);
        b->cams.push_back(cams[i]);
        b->params.push_back(p);
        b->n.push_back(n_particles[i]);
        b->max_n = std::max(b->max_n, n_particles[i]);
        b->K = std::max(b->K, (int32_t)p.max_iters);
    }
    if (g != ROSE_OK) {
        batch_free(b);
        return g;
    }
    std::vector<int> begin(count + 1, 0);
    for (int k = 0; k < count; ++k) begin[k + 1] = begin[k] + (nblk[k] + 7) / 8 * 8;
    b->total = begin[count];
    for (int k = 0; k < count && !own[order[k]];) {
        const int key = group_key(order[k]);
        int e = k;
        while (e < count && group_key(order[e]) == key) ++e;
        BatchGroup gr;
        gr.fmt = tsdfs[order[k]]->g.fmt;
        gr.lk = params[order[k]].lookup;
        gr.first = k;
        gr.count = e - k;
        gr.base = begin[k];
        gr.end = begin[e];
        gr.grid = batch_grid(P, U, gr.fmt, gr.lk, gr.end - gr.base);
        b->groups.push_back(gr);
        k = e;
    }
    const size_t n_ctr = std::max<size_t>(8, 8 * b->groups.size());
    bool ok = hipMalloc(&b->fit_dev, sizeof(FitLaunch) * count) == hipSuccess &&
              hipMalloc(&b->begin_dev, sizeof(int) * (count + 1)) == hipSuccess &&
              hipMalloc(&b->ctr_dev, sizeof(int) * n_ctr) == hipSuccess &&
              hipMemset(b->ctr_dev, 0, sizeof(int) * n_ctr) == hipSuccess &&
              hipMalloc(&b->init_dev, sizeof(InitStatic) * count) == hipSuccess &&
              hipMalloc(&b->upd_dev, sizeof(UpdateArgs) * count) == hipSuccess &&
              hipMalloc(&b->stp_dev, sizeof(DevState*) * count) == hipSuccess &&
              hipHostMalloc(&b->in_host, sizeof(FrameIn) * count, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&b->out_host, sizeof(DevState) * count, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&b->prop_ok, sizeof(int32_t) * count, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMemcpy(b->fit_dev, fit.data(), sizeof(FitLaunch) * count, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->begin_dev, begin.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->init_dev, init.data(), sizeof(InitStatic) * count, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->upd_dev, upd.data(), sizeof(UpdateArgs) * count, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->stp_dev, stp.data(), sizeof(DevState*) * count, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        batch_free(b);
        set_error("pso_batch_create: device allocation or copy failed");
        return ROSE_E_DEVICE;
    }
    memset(b->in_host, 0, sizeof(FrameIn) * count);
    b->fit_host = fit;
    b->init_host = init;
    b->upd_host = upd;
    b->pos = pos;
    *out = b;
    return ROSE_OK;
}

rose_status rose_batch_set_own_launch(int64_t min_evals) {
    clear_error();
    ROSE_REQUIRE(min_evals >= 0, ROSE_E_ARG, "rose_batch_set_own_launch: min_evals = %lld is negative",
                 (long long)min_evals);
    g_batch_own_min = min_evals;
    return ROSE_OK;
}

rose_status pso_batch_destroy(rose_batch* b) {
    clear_error();
    if (!b) return ROSE_OK;
    (void)hipDeviceSynchronize();
    batch_free(b);
    return ROSE_OK;
}

rose_status pso_batch_track(rose_batch* b, const float* const* depth_devs, const rose_pose* init_centres,
                            const double* init_rs, rose_track_state* states, rose_track_stats* stats,
                            hipStream_t s) {
    return batch_track_impl(b, depth_devs, init_centres, init_rs, nullptr, nullptr, states, stats, s);
}

}  // extern "C"

// One batched frame step.  prop_dev (nullable): network outputs (12 per
// sequence, device) from which k_learned_proposal sets every active
// sequence's c_0 and r_0 on the device, after the host has written the
// carried pose and axis lengths and before the step's launches, so the
// outputs never travel to the host; its finite flags land in b->prop_ok.
static rose_status batch_track_impl(rose_batch* b, const float* const* depth_devs, const rose_pose* init_centres,
                                    const double* init_rs, const float* prop_dev, const rose_learned_params* lp,
                                    rose_track_state* states, rose_track_stats* stats, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(b && depth_devs && states, ROSE_E_ARG, "pso_batch_track: NULL argument");
    for (int i = 0; i < b->count; ++i) ROSE_REQUIRE(depth_devs[i], ROSE_E_ARG, "pso_batch_track: NULL depth %d", i);
    {
        rose_status rs = batch_refresh(b, false);
        if (rs != ROSE_OK) return rs;
    }
    // per-frame inputs (pinned host memory, read by the init kernel)
    for (int i = 0; i < b->count; ++i) {
        FrameIn& in = b->in_host[i];
        rose_track_state& st = states[i];
        const rose_track_params& p = b->params[i];
        const rose_pose* c0 = init_centres ? &init_centres[i] : &st.pose;
        const double* r0 = init_rs ? &init_rs[6 * i] : st.r;
        for (int k = 0; k < 4; ++k) in.qc[k] = c0->q[k];
        for (int k = 0; k < 3; ++k) in.tc[k] = c0->t[k];
        for (int k = 0; k < 6; ++k) in.r[k] = r0[k];
        pose_matrix(st.pose.q, st.pose.t, in.Tprev);
        in.depth = depth_devs[i];
        in.active = st.tsdf_built ? 1 : 0;
        in.pad = 0;
        if (!st.tsdf_built) {
            // Sec. 4, first corner case (no fitness): rhat = 0.5 * 1, pose kept
            for (int d = 0; d < 6; ++d) st.r[d] = p.beta * r0[d] + (1.0 - p.beta) * 0.5;
            st.pose = *c0;
            st.rho = 0.5;
            st.frame += 1;
            if (stats) {
                memset(&stats[i], 0, sizeof(rose_track_stats));
                stats[i].iters = 1;
                stats[i].rho_iter[0] = 0.5;
            }
        }
    }
    if (prop_dev) {
        hipLaunchKernelGGL(k_learned_proposal, dim3((b->count + 63) / 64), dim3(64), 0, s, prop_dev, b->count,
                           b->in_host, b->prop_ok, lp->kappa, lp->r_min, lp->r_max);
        ROSE_CHECK_HIP(hipGetLastError());
    }
    const bool graph = b->use_graph && s != nullptr;
    if (graph) {
        if (!b->exec || b->graph_stream != s) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            ROSE_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            rose_status st = batch_enqueue(b, s);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(s, &gr);
            if (st != ROSE_OK) return st;
            if (e != hipSuccess) {
                set_error("pso_batch_track: graph capture failed: %s", hipGetErrorString(e));
                return ROSE_E_DEVICE;
            }
            b->graph = gr;
            ROSE_CHECK_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->graph_stream = s;
        }
        ROSE_CHECK_HIP(hipGraphLaunch(b->exec, s));
    } else {
        rose_status st = batch_enqueue(b, s);
        if (st != ROSE_OK) return st;
    }
    ROSE_CHECK_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < b->count; ++i) {
        if (!b->in_host[i].active) continue;
        const DevState& r = b->out_host[i];
        rose_track_state& st = states[i];
        if (stats) {
            memset(&stats[i], 0, sizeof(rose_track_stats));
            stats[i].status = (r.n_points == 0) ? ROSE_E_STATE : ROSE_OK;
        }
        if (r.n_points == 0) continue;  // no valid depth: state unchanged
        for (int k = 0; k < 4; ++k) st.pose.q[k] = r.qc[k];
        for (int k = 0; k < 3; ++k) st.pose.t[k] = r.tc[k];
        for (int d = 0; d < 6; ++d) st.r[d] = r.r1[d];
        st.rho = r.rho_last;
        st.frame += 1;
        if (stats) {
            stats[i].iters = r.k;
            stats[i].n_points = r.n_points;
            stats[i].n_overlap_last = r.n_overlap;
            for (int k = 0; k < r.k && k < ROSE_MAX_ITERS; ++k) {
                stats[i].aps_size[k] = r.aps[k];
                stats[i].n_overlap[k] = r.n_overlap_iter[k];
                stats[i].rho_iter[k] = r.rho_iter[k];
                stats[i].rho_centre[k] = r.rho_centre[k];
                for (int d = 0; d < 6; ++d) stats[i].r_iter[k][d] = r.r_iter[k][d];
                stats[i].n_particles[k] = b->n[i];
                if (b->own_of[i] >= 0) stats[i].fit_mode[k] = switch_mode(b->own_fl[b->own_of[i]], r.r_iter[k]);
            }
        }
    }
    return ROSE_OK;
}

// ------------------------------------------------------- learned proposal
extern "C" {

rose_status rose_chart_log(const rose_pose* a, const rose_pose* b, double u[6]) {
    clear_error();
    ROSE_REQUIRE(a && b && u, ROSE_E_ARG, "rose_chart_log: NULL argument");
    // a^-1 b: q = conj(q_a) q_b, t = R_a^T (t_b - t_a); chart = (imag(q) with w >= 0, t)
    const double qa_c[4] = {a->q[0], -a->q[1], -a->q[2], -a->q[3]};
    double q[4], Ra[9];
    quat_prod(qa_c, b->q, q);
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = (q[0] < 0.0) ? -1.0 : 1.0;
    quat_rot(a->q, Ra);
    const double d[3] = {b->t[0] - a->t[0], b->t[1] - a->t[1], b->t[2] - a->t[2]};
    for (int i = 0; i < 3; ++i) u[i] = sg * q[i + 1] / n;
    for (int i = 0; i < 3; ++i) u[3 + i] = Ra[0 * 3 + i] * d[0] + Ra[1 * 3 + i] * d[1] + Ra[2 * 3 + i] * d[2];
    return ROSE_OK;
}

rose_status rose_chart_exp(const rose_pose* a, const double u[6], rose_pose* out) {
    clear_error();
    ROSE_REQUIRE(a && u && out, ROSE_E_ARG, "rose_chart_exp: NULL argument");
    double q[4] = {a->q[0], a->q[1], a->q[2], a->q[3]}, t[3] = {a->t[0], a->t[1], a->t[2]};
    retract(q, t, u);
    for (int i = 0; i < 4; ++i) out->q[i] = q[i];
    for (int i = 0; i < 3; ++i) out->t[i] = t[i];
    return ROSE_OK;
}

}  // extern "C"

extern "C" {

rose_status pso_track_frame_learned(rose_tsdf* h, const float* depth_dev, const rose_camera* cam,
                                    const float* pst_small_dev, int32_t n_small, const float* pst_plain_dev,
                                    int32_t n_plain, rose_mlp* mlp, const float* mlp_params_dev, float* work_dev,
                                    const double velocity[6], const rose_track_params* p,
                                    const rose_learned_params* lp, rose_track_state* state, rose_track_stats* stats,
                                    int32_t* fallback_out, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && depth_dev && cam && pst_small_dev && pst_plain_dev && mlp && mlp_params_dev && work_dev &&
                     velocity && p && lp && state,
                 ROSE_E_ARG, "pso_track_frame_learned: NULL argument");
    ROSE_REQUIRE(lp->scale >= 1 && lp->low_w >= 1 && lp->low_h >= 1 && lp->feature_dim >= lp->low_w * lp->low_h + 6 &&
                     lp->kappa > 0 && lp->r_min > 0 && lp->r_max >= lp->r_min,
                 ROSE_E_ARG, "pso_track_frame_learned: bad learned parameters");
    ROSE_REQUIRE(lp->iters >= 0 && lp->iters <= ROSE_MAX_ITERS, ROSE_E_ARG,
                 "pso_track_frame_learned: iters = %d out of [0, %d]", lp->iters, ROSE_MAX_ITERS);
    ROSE_REQUIRE(p->levels <= 1, ROSE_E_UNSUPPORTED,
                 "pso_track_frame_learned: multi-resolution schedules are not supported here");
    if (fallback_out) *fallback_out = 0;
    if (!state->tsdf_built)
        return pso_track_frame(h, depth_dev, nullptr, cam, pst_plain_dev, n_plain, p, nullptr, nullptr, state, stats,
                               s);
    rose_camera low;
    low.fx = cam->fx / (float)lp->scale;
    low.fy = cam->fy / (float)lp->scale;
    low.cx = (cam->cx + 0.5f) / (float)lp->scale - 0.5f;
    low.cy = (cam->cy + 0.5f) / (float)lp->scale - 0.5f;
    low.width = lp->low_w;
    low.height = lp->low_h;
    float* render = work_dev;
    float* X = render + lp->low_w * lp->low_h;
    float* out = X + lp->feature_dim;
    rose_status st;
    if ((st = tsdf_raycast(h, &state->pose, &low, lp->near_m, lp->far_m, lp->step_m, render, s)) != ROSE_OK) return st;
    if ((st = proposal_features(depth_dev, cam, render, &low, lp->scale, velocity, lp->feature_dim, X, s)) != ROSE_OK)
        return st;
    if ((st = rose_mlp_forward(mlp, mlp_params_dev, X, 1, out, s)) != ROSE_OK) return st;
    // the proposal on the device, by the same kernel as the batched step's
    if (!h->learn_in) ROSE_CHECK_HIP(hipHostMalloc(&h->learn_in, sizeof(FrameIn), hipHostMallocDefault));
    if (!h->learn_ok) ROSE_CHECK_HIP(hipHostMalloc(&h->learn_ok, sizeof(int32_t), hipHostMallocDefault));
    FrameIn& lin = *h->learn_in;
    for (int i = 0; i < 4; ++i) lin.qc[i] = state->pose.q[i];
    for (int i = 0; i < 3; ++i) lin.tc[i] = state->pose.t[i];
    for (int d = 0; d < 6; ++d) lin.r[d] = state->r[d];
    lin.active = 1;
    hipLaunchKernelGGL(k_learned_proposal, dim3(1), dim3(64), 0, s, out, 1, h->learn_in, h->learn_ok, lp->kappa,
                       lp->r_min, lp->r_max);
    ROSE_CHECK_HIP(hipGetLastError());
    ROSE_CHECK_HIP(hipStreamSynchronize(s));
    const bool finite = *h->learn_ok != 0;
    bool fallback = !finite;
    if (finite) {
        double r0[6];
        rose_pose c0;
        for (int i = 0; i < 4; ++i) c0.q[i] = lin.qc[i];
        for (int i = 0; i < 3; ++i) c0.t[i] = lin.tc[i];
        for (int d = 0; d < 6; ++d) r0[d] = lin.r[d];
        rose_track_state trial = *state;
        rose_track_params pl = *p;
        if (lp->iters > 0) pl.max_iters = lp->iters;
        st = pso_track_frame(h, depth_dev, nullptr, cam, pst_small_dev, n_small, &pl, &c0, r0, &trial, stats, s);
        if (st == ROSE_OK && trial.rho >= state->rho - lp->delta) {
            *state = trial;
        } else if (st == ROSE_OK || st == ROSE_E_STATE) {
            fallback = true;
        } else {
            return st;
        }
    }
    if (fallback) {
        if (fallback_out) *fallback_out = 1;
        return pso_track_frame(h, depth_dev, nullptr, cam, pst_plain_dev, n_plain, p, nullptr, nullptr, state, stats,
                               s);
    }
    return ROSE_OK;
}

}  // extern "C"

// ------------------------------------------------ batched learned frame step
extern "C" {

rose_status pso_batch_track_learned(rose_batch* b, const float* const* depth_devs, rose_mlp* mlp,
                                    const float* mlp_params_dev, float* work_dev, const double* velocities,
                                    const rose_learned_params* lp, const float* const* pst_plain_devs,
                                    const int32_t* n_plain, const rose_track_params* plain_params,
                                    rose_track_state* states, rose_track_stats* stats, int32_t* fallback_out,
                                    hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(b && depth_devs && mlp && mlp_params_dev && work_dev && velocities && lp && pst_plain_devs &&
                     n_plain && plain_params && states,
                 ROSE_E_ARG, "pso_batch_track_learned: NULL argument");
    ROSE_REQUIRE(lp->scale >= 1 && lp->low_w >= 1 && lp->low_h >= 1 && lp->feature_dim >= lp->low_w * lp->low_h + 6 &&
                     lp->kappa > 0 && lp->r_min > 0 && lp->r_max >= lp->r_min,
                 ROSE_E_ARG, "pso_batch_track_learned: bad learned parameters");
    const int n = b->count;
    for (int i = 0; i < n; ++i)
        ROSE_REQUIRE(depth_devs[i] && pst_plain_devs[i] && n_plain[i] >= 1 && n_plain[i] <= ROSE_MAX_PARTICLES,
                     ROSE_E_ARG, "pso_batch_track_learned: bad depth or plain template for sequence %d", i);
    // size every handle's scratch for a plain fallback now, so that no
    // fallback reallocates it under the batch's launch records
    for (int i = 0; i < n; ++i) {
        rose_tsdf* h = b->h[i];
        const rose_track_params& pp = plain_params[i];
        ROSE_REQUIRE(pp.stride >= 1 && pp.levels <= 1, ROSE_E_ARG,
                     "pso_batch_track_learned: plain parameters of sequence %d need stride >= 1 and one level", i);
        const int64_t mmax = (int64_t)((b->cams[i].width + pp.stride - 1) / pp.stride) *
                             ((b->cams[i].height + pp.stride - 1) / pp.stride);
        int sp, su;
        float thr, zref;
        fit_launch_shape(h, pp.lookup, &sp, &su, &thr, &zref);
        const int splits = choose_splits(n_plain[i], mmax, h->g.fmt, sp);
        rose_status g;
        if ((g = grow(&h->pts, &h->cap_points, mmax)) != ROSE_OK) return g;
        if ((g = grow(&h->pts_o, &h->cap_points_o, mmax)) != ROSE_OK) return g;
        if ((g = grow(&h->partial, &h->cap_partial, (int64_t)n_plain[i] * splits * kPartSub)) != ROSE_OK) return g;
        if ((g = grow(&h->F, &h->cap_particles, (int64_t)n_plain[i])) != ROSE_OK) return g;
    }
    const int64_t npx = (int64_t)lp->low_w * lp->low_h, fd = lp->feature_dim;
    float* renders = work_dev;
    float* X = renders + n * npx;
    float* out = X + n * fd;
    if (fallback_out)
        for (int i = 0; i < n; ++i) fallback_out[i] = 0;
    // inputs of the network for every sequence whose model exists, one batched forward
    rose_status st;
    for (int i = 0; i < n; ++i) {
        float* Xi = X + i * fd;
        if (!states[i].tsdf_built) {
            ROSE_CHECK_HIP(hipMemsetAsync(Xi, 0, sizeof(float) * (size_t)fd, s));
            continue;
        }
        const rose_camera& cam = b->cams[i];
        rose_camera low;
        low.fx = cam.fx / (float)lp->scale;
        low.fy = cam.fy / (float)lp->scale;
        low.cx = (cam.cx + 0.5f) / (float)lp->scale - 0.5f;
        low.cy = (cam.cy + 0.5f) / (float)lp->scale - 0.5f;
        low.width = lp->low_w;
        low.height = lp->low_h;
        float* Ri = renders + i * npx;
        if ((st = tsdf_raycast(b->h[i], &states[i].pose, &low, lp->near_m, lp->far_m, lp->step_m, Ri, s)) != ROSE_OK)
            return st;
        if ((st = proposal_features(depth_devs[i], &cam, Ri, &low, lp->scale, velocities + 6 * i, (int32_t)fd, Xi,
                                    s)) != ROSE_OK)
            return st;
    }
    if ((st = rose_mlp_forward(mlp, mlp_params_dev, X, n, out, s)) != ROSE_OK) return st;
    // proposals c_0 = s^{t-1} * Delta(mu), r_0 = kappa exp(l) clamped, set on
    // the device inside the step (the network outputs stay on the device);
    // sequences without a finite proposal run from their own state and fall
    // back below
    std::vector<rose_track_state> trial(states, states + n);
    std::vector<rose_track_stats> tstats(n);
    if ((st = batch_track_impl(b, depth_devs, nullptr, nullptr, out, lp, trial.data(), tstats.data(), s)) != ROSE_OK)
        return st;
    std::vector<char> finite(n, 1);
    for (int i = 0; i < n; ++i) finite[i] = !states[i].tsdf_built || b->prop_ok[i] != 0;
    for (int i = 0; i < n; ++i) {
        const bool keep = !states[i].tsdf_built ||
                          (finite[i] && tstats[i].status == ROSE_OK && trial[i].rho >= states[i].rho - lp->delta);
        if (keep) {
            states[i] = trial[i];
            if (stats) stats[i] = tstats[i];
            continue;
        }
        // fallback: plain PST from the unchanged state
        if (fallback_out) fallback_out[i] = 1;
        rose_track_stats fs;
        st = pso_track_frame(b->h[i], depth_devs[i], nullptr, &b->cams[i], pst_plain_devs[i], n_plain[i],
                             &plain_params[i], nullptr, nullptr, &states[i], &fs, s);
        if (st != ROSE_OK && st != ROSE_E_STATE) return st;
        fs.status = st;
        if (stats) stats[i] = fs;
    }
    clear_error();
    return ROSE_OK;
}

}  // extern "C"
