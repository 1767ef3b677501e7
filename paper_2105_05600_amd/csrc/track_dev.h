// Device helpers and launch records of the per-frame pose searches
// (track.hip: PFO with PST; swarm.hip: the comparison optimisers), shared by
// their translation units.
#pragma once

#include "common.h"

namespace rose {

struct Cam {
    float fx, fy, cx, cy;
    int32_t W, H;
    const float* prev;  // depth of frame t-1 (H x W) for the stricter overlap test, or nullptr
};

// Eq. unproj in binary32: x = (((float)u - cx) z) / fx, y likewise.
__device__ inline float4 unproject_px(const Cam& c, int u, int v, float z) {
    return make_float4((((float)u - c.cx) * z) / c.fx, (((float)v - c.cy) * z) / c.fy, z, 0.0f);
}

// Eq. validness with A = T_prev^-1 T_c rounded to binary32:
// x' = A x (fmaf chain); kept iff z' > 0 and the projection
// (fmaf(fx, x'/z', cx), fmaf(fy, y'/z', cy)) lies in [0, W-1] x [0, H-1];
// with a previous depth image, also iff its pixel nearest to the projection,
// (floor(px + 1/2), floor(py + 1/2)) in binary32, holds a depth > 0.  The
// bounds test keeps that pixel inside the image.
__device__ inline bool overlap_keep(const Cam& c, const float* A, float4 x) {
    const float xp = xf_row(A[0], A[1], A[2], A[3], x.x, x.y, x.z);
    const float yp = xf_row(A[4], A[5], A[6], A[7], x.x, x.y, x.z);
    const float zp = xf_row(A[8], A[9], A[10], A[11], x.x, x.y, x.z);
    if (!(zp > 0.0f)) return false;
    const float px = fmaf(c.fx, xp / zp, c.cx);
    const float py = fmaf(c.fy, yp / zp, c.cy);
    if (!(px >= 0.0f && px <= (float)(c.W - 1) && py >= 0.0f && py <= (float)(c.H - 1))) return false;
    if (!c.prev) return true;
    const int u = min((int)floorf(px + 0.5f), c.W - 1), v = min((int)floorf(py + 0.5f), c.H - 1);
    return c.prev[(size_t)v * (size_t)c.W + (size_t)u] > 0.0f;
}

// Enumeration of the stride-s sample grid (su x sv samples).  Row-major
// (tiled = false), or 8x8-sample tiles in row-major tile order with
// row-major samples inside a tile (tiled = true), so that the 64 lanes of a
// wavefront see a compact image patch and their TSDF gathers share cache
// lines.  Returns false for the padding positions of partial tiles.
__device__ inline int sample_count(int su, int sv, bool tiled) {
    return tiled ? ((su + 7) / 8) * ((sv + 7) / 8) * 64 : su * sv;
}

__device__ inline bool sample_at(int q, int su, int sv, bool tiled, int* uu, int* vv) {
    if (!tiled) {
        *uu = q % su;
        *vv = q / su;
        return true;
    }
    const int ntx = (su + 7) / 8;
    const int t = q >> 6, e = q & 63;
    *uu = (t % ntx) * 8 + (e & 7);
    *vv = (t / ntx) * 8 + (e >> 3);
    return *uu < su && *vv < sv;
}

// Whole-block order-preserving overlap compaction of m points, kRounds
// coalesced rounds of blockDim points at a time: every thread loads and
// tests its point of each round (all loads in flight together), the waves'
// ballots give per-round, per-wave counts, one table in LDS turns them into
// output offsets, and each thread writes its kept points.  The output is the
// kept points in index order.  (lds is unused; kept for the callers' shape.)
__device__ inline int overlap_compact(const Cam& c, const float* A, bool all, const float4* pts, int m, float4* out,
                                      int* lds) {
    (void)lds;
    constexpr int kRounds = 8, kMaxWaves = 16;
    __shared__ int cnt[kMaxWaves * kRounds];   // wave w, round q: kept count, then exclusive wave offset
    __shared__ int start[kRounds + 1];         // round offsets; start[kRounds] = batch total
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int bd = (int)blockDim.x;
    int base = 0;
    for (int j0 = 0; j0 < m; j0 += kRounds * bd) {
        float4 x[kRounds];
        uint64_t ball[kRounds];
#pragma unroll
        for (int q = 0; q < kRounds; ++q) x[q] = pts[min(j0 + q * bd + (int)threadIdx.x, m - 1)];
#pragma unroll
        for (int q = 0; q < kRounds; ++q) {
            const int j = j0 + q * bd + (int)threadIdx.x;
            const bool keep = (j < m) && (all || overlap_keep(c, A, x[q]));
            ball[q] = __ballot(keep);
            if (lane == 0) cnt[wid * kRounds + q] = __popcll(ball[q]);
        }
        __syncthreads();
        if ((int)threadIdx.x < kRounds) {  // one thread per round: offsets of the waves
            const int q = threadIdx.x;
            int acc = 0;
            for (int w = 0; w < nw; ++w) {
                const int cw = cnt[w * kRounds + q];
                cnt[w * kRounds + q] = acc;
                acc += cw;
            }
            start[q] = acc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int q = 0; q < kRounds; ++q) {
                const int t = start[q];
                start[q] = acc;
                acc += t;
            }
            start[kRounds] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRounds; ++q)
            if ((ball[q] >> lane) & 1ull)
                out[base + start[q] + cnt[wid * kRounds + q] + __popcll(ball[q] & lt)] = x[q];
        base += start[kRounds];
        __syncthreads();  // the tables are rewritten by the next batch
    }
    return base;
}

struct InitStatic {
    DevState* st;
    Cam cam;
    int32_t levels;                        // 1, or the multi-resolution level count
    int32_t flags;
    int32_t stride[ROSE_MAX_LEVELS];       // subsampling stride per level
    int32_t offset[ROSE_MAX_LEVELS];       // first point of each level in pts
    float4* pts;
    float4* pts_o;
};

struct UpdateArgs {
    DevState* st;
    Cam cam;
    const float* pst;
    const uint64_t* partial;
    float* F;
    const float4* pts;  // points of the next iteration's level
    float4* pts_o;
    int32_t next_level; // level of the next iteration (its count is st->lvl_points[next_level])
    int32_t n;
    int32_t splits;
    int32_t max_iters;
    int32_t early_stop;
    int32_t flags;
    double beta, eps, tau, stop_tol;
};

// F_i = S_i / |O| (Eq. normallh) from the slice sums on the 2^-39 grid
// (exact integer sum, then one rounding to binary64, an exact scaling, one
// correctly rounded division and one rounding to binary32).  One wavefront
// per particle: lane l adds the particle's slots l, l + 64, ... (coalesced
// 8-byte reads of its splits x kPartSub consecutive slots), then the wave
// adds the lanes' integers; every lane returns F_i.
__device__ inline float final_fitness(const UpdateArgs& a, int i, int nO) {
    const int lane = threadIdx.x & 63;
    const int S = a.splits * kPartSub;
    const uint64_t* row = a.partial + (int64_t)i * S;
    uint64_t q = 0;
    for (int k = lane; k < S; k += kWave) q += row[k];
    q = wave_sum_u64(q);
    const double s = (double)q * kGridScale;
    double f;
    if (a.flags & ROSE_FLAG_NO_NORMALIZE) f = s;
    else f = (nO > 0) ? s / (double)nO : 1.0;
    return (float)f;
}

rose_status launch_track_init(const InitStatic& a, const FrameIn& in, hipStream_t s);
rose_status launch_fitness_reduce(const UpdateArgs& a, hipStream_t s);

inline Cam to_cam(const rose_camera* c, const float* prev_depth = nullptr) {
    return Cam{c->fx, c->fy, c->cx, c->cy, c->width, c->height, prev_depth};
}

inline rose_status check_cam(const rose_camera* c, const char* who) {
    ROSE_REQUIRE(c != nullptr, ROSE_E_ARG, "%s: NULL camera", who);
    ROSE_REQUIRE(c->width > 0 && c->height > 0 && (int64_t)c->width * c->height <= (int64_t)ROSE_MAX_IMAGE_PIXELS,
                 ROSE_E_SHAPE, "%s: image %dx%d out of range", who, c->width, c->height);
    ROSE_REQUIRE(c->fx > 0 && c->fy > 0, ROSE_E_ARG, "%s: focal lengths must be > 0", who);
    return ROSE_OK;
}

template <typename T>
inline rose_status grow(T** p, int64_t* cap, int64_t need) {
    if (*cap >= need && *p) return ROSE_OK;
    if (*p) ROSE_CHECK_HIP(hipFree(*p));
    *p = nullptr;
    ROSE_CHECK_HIP(hipMalloc((void**)p, sizeof(T) * (size_t)(need > 0 ? need : 1)));
    *cap = need;
    return ROSE_OK;
}

}  // namespace rose
