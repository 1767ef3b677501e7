// Particle fitness evaluation (Eq. ourlh with the normalisation of
// Eq. normallh) -- the hot loop of the pose search.
//
// Mapping on gfx950: one wavefront evaluates P particles over one slice of
// the point list.  The P transforms are built once per wave in binary64
// (c * Delta(r (.) p), folded with the voxel scale, rounded once to binary32)
// and held wave-uniform; the slice's points are striped across the 64 lanes,
// so each point is loaded once (one 16-byte load) and reused for P
// particles, and the P TSDF gathers per point are independent loads in
// flight together.  Squares are accumulated in binary64 (the product of two
// binary32 values is exact in binary64, so one fma per term), reduced over
// the wave with butterfly shuffles, and written as one partial sum per
// (particle, slice); a second pass adds the slices in a fixed order.
#include <algorithm>
#include <vector>

#include "common.h"

namespace rose {

// Byte offset of an element; volumes below 4 GB use 32-bit offsets so the
// gather is a global load with a scalar base and a 32-bit vector offset.
template <int FMT>
__device__ inline uint32_t elem_bytes() {
    return FMT == ROSE_TSDF_F32 ? 4u : 2u;
}

template <int FMT, bool WIDE>
__device__ inline float gather(const void* base, uint32_t off) {
    if constexpr (WIDE) {
        return load_psi<FMT>(base, off);
    } else {
        const char* p = (const char*)base + (off * elem_bytes<FMT>());
        if constexpr (FMT == ROSE_TSDF_F32) return *(const float*)p;
        else if constexpr (FMT == ROSE_TSDF_F16) return __half2float(*(const __half*)p);
        else return (float)(*(const int16_t*)p) * (1.0f / 32767.0f);
    }
}

struct VoxelTest {
    float fx, fy, fz;  // grid extent as float
};

// NEAREST voxel of voxel-space coordinate g: inside iff 0 <= g < n on every
// axis (NaN is outside); then floor(g) == (uint32)g.
__device__ inline bool nearest_offset(const Grid& g, const VoxelTest& e, float gx, float gy, float gz, uint32_t* off) {
    const bool in = (gx >= 0.0f) & (gx < e.fx) & (gy >= 0.0f) & (gy < e.fy) & (gz >= 0.0f) & (gz < e.fz);
    // out-of-range conversions saturate; their offset is replaced below
    const uint32_t o = brick_offset(g, (uint32_t)gx, (uint32_t)gy, (uint32_t)gz);
    *off = in ? o : 0u;
    return in;
}

template <int FMT, bool WIDE>
__device__ inline float lookup_trilinear(const Grid& g, float gx, float gy, float gz) {
    const float hx = gx - 0.5f, hy = gy - 0.5f, hz = gz - 0.5f;
    const bool in = (hx >= 0.0f) & (hx < (float)(g.nx - 1)) & (hy >= 0.0f) & (hy < (float)(g.ny - 1)) &
                    (hz >= 0.0f) & (hz < (float)(g.nz - 1));
    const uint32_t ix = in ? (uint32_t)hx : 0u, iy = in ? (uint32_t)hy : 0u, iz = in ? (uint32_t)hz : 0u;
    const float fx = hx - (float)ix, fy = hy - (float)iy, fz = hz - (float)iz;
    const float v000 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix, iy, iz));
    const float v100 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix + 1, iy, iz));
    const float v010 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix, iy + 1, iz));
    const float v110 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix + 1, iy + 1, iz));
    const float v001 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix, iy, iz + 1));
    const float v101 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix + 1, iy, iz + 1));
    const float v011 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix, iy + 1, iz + 1));
    const float v111 = gather<FMT, WIDE>(g.psi, brick_offset(g, ix + 1, iy + 1, iz + 1));
    const float c00 = fmaf(fx, v100 - v000, v000);
    const float c10 = fmaf(fx, v110 - v010, v010);
    const float c01 = fmaf(fx, v101 - v001, v001);
    const float c11 = fmaf(fx, v111 - v011, v011);
    const float c0 = fmaf(fy, c10 - c00, c00);
    const float c1 = fmaf(fy, c11 - c01, c01);
    const float v = fmaf(fz, c1 - c0, c0);
    return in ? v : 1.0f;
}

__device__ inline float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// P particles per wave, U points per lane per loop step; all P*U gathers of
// a step are issued before any is consumed.
__device__ inline float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Mapping switch: the footprint of the search -- how far one point moves
// across the particles -- is taken as the largest translation axis length
// plus the largest rotation axis length times a reference depth, in voxels.
// Both kernels of a switched launch evaluate this same expression on the
// same device state, so exactly one of them does the work.
__device__ inline bool switch_skips(const FitLaunch& a) {
    if (a.pl_side == 0) return false;
    const double* r = a.st->r;
    const double rr = fmax(fmax(r[0], r[1]), r[2]);
    const double rt = fmax(fmax(r[3], r[4]), r[5]);
    const bool small = (rt + (double)a.pl_zref * rr) <= (double)a.pl_thr * (double)a.g.vox;
    return small != (a.pl_side == 1);
}

template <int P, int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false>
__device__ void fitness_body(const FitLaunch& a, const int blk) {
    constexpr int kU = U;
    const int lane = threadIdx.x & 63;
    // XCD-aware mapping: consecutive workgroups go to the 8 XCDs in turn
    // (XCD = workgroup index mod 8).  With splits a multiple of 8, XCD x owns
    // the contiguous slices x*splits/8 .. (x+1)*splits/8 - 1, i.e. a fixed 1/8
    // of the point list, so its L2 only holds the voxels around those
    // points; its workgroups cycle through those slices before moving to the
    // next particles, so the particles in flight on an XCD are few (and, in
    // the schedule order, similar).  The 4 waves of a workgroup take 4
    // consecutive particle groups of the same slice (shared point loads and
    // nearby gathers in the CU's L1).
    const int s8 = a.splits >> 3;
    const int r = blk % a.splits;
    const int split = (r & 7) * s8 + (r >> 3);
    const int group = (blk / a.splits) * 4 + (threadIdx.x >> 6);
    const int p0 = group * P;
    if (p0 >= a.n) return;
    if (FROM_STATE && (a.st->stopped || switch_skips(a))) return;
    const int m = a.count_dev ? *a.count_dev : a.count;

    // particle transforms: lane l < P builds particle p0 + l
    float V[12];
    {
        int pi = p0 + (lane < P ? lane : 0);
        if (pi >= a.n) pi = a.n - 1;
        if (FROM_STATE && a.order) pi = a.order[pi];
        double T[12];
        if (FROM_STATE) {
            float p[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) p[d] = a.pst[6 * (int64_t)pi + d];
            particle_transform(a.st->qc, a.st->tc, a.st->r, p, T);
        } else {
#pragma unroll
            for (int e = 0; e < 12; ++e) T[e] = (double)a.T32[12 * (int64_t)pi + e];
        }
        fold_to_voxel(T, (double)a.g.vox, a.g.origin, V);
    }
    // rotation entries wave-uniform (scalar registers); the translation column
    // is broadcast with a cross-lane shuffle so that each fma reads at most
    // one scalar operand
    float S[P][12];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < 12; ++e) S[p][e] = (e % 4 == 3) ? __shfl(V[e], p, kWave) : bcast(V[e], p);

    const Grid g = a.g;
    const VoxelTest ext{(float)g.nx, (float)g.ny, (float)g.nz};
    const int chunk = (m + a.splits - 1) / a.splits;
    const int j0 = split * chunk;
    const int j1 = min(m, j0 + chunk);
    double acc[P];
    float accf[P];  // ACC32: plain binary32 running sums
#pragma unroll
    for (int p = 0; p < P; ++p) {
        acc[p] = 0.0;
        accf[p] = 0.0f;
    }
    // the next step's points are loaded one step ahead, so their latency
    // overlaps the current step's gathers
    float4 xn[kU];
    bool okn[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * kWave + lane;
        okn[u] = j < j1;
        xn[u] = a.pts[okn[u] ? j : (j1 > j0 ? j0 : 0)];
    }
    for (int jb = j0; jb < j1; jb += kWave * kU) {
        float4 x[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            x[u] = xn[u];
            ok[u] = okn[u];
            const int j = jb + kWave * kU + u * kWave + lane;
            okn[u] = j < j1;
            xn[u] = a.pts[okn[u] ? j : j0];
        }
        float v[kU][P];
        if constexpr (LK == ROSE_LOOKUP_NEAREST) {
            uint32_t off[kU][P];
            bool in[kU][P];
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float gx = xf_row(S[p][0], S[p][1], S[p][2], S[p][3], x[u].x, x[u].y, x[u].z);
                    const float gy = xf_row(S[p][4], S[p][5], S[p][6], S[p][7], x[u].x, x[u].y, x[u].z);
                    const float gz = xf_row(S[p][8], S[p][9], S[p][10], S[p][11], x[u].x, x[u].y, x[u].z);
                    in[u][p] = nearest_offset(g, ext, gx, gy, gz, &off[u][p]);
                }
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p) v[u][p] = gather<FMT, WIDE>(g.psi, off[u][p]);
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p) v[u][p] = in[u][p] ? v[u][p] : 1.0f;
        } else {
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float gx = xf_row(S[p][0], S[p][1], S[p][2], S[p][3], x[u].x, x[u].y, x[u].z);
                    const float gy = xf_row(S[p][4], S[p][5], S[p][6], S[p][7], x[u].x, x[u].y, x[u].z);
                    const float gz = xf_row(S[p][8], S[p][9], S[p][10], S[p][11], x[u].x, x[u].y, x[u].z);
                    v[u][p] = lookup_trilinear<FMT, WIDE>(g, gx, gy, gz);
                }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if constexpr (ACC32) {
                    const float d = ok[u] ? v[u][p] : 0.0f;
                    accf[p] = fmaf(d, d, accf[p]);
                } else {
                    const double d = (double)(ok[u] ? v[u][p] : 0.0f);
                    acc[p] = fma(d, d, acc[p]);
                }
            }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if constexpr (ACC32) acc[p] = (double)wave_sum_f(accf[p]);
        else acc[p] = wave_sum(acc[p]);
    }
    if (lane == 0) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (p0 + p < a.n) {
                const int pi = (FROM_STATE && a.order) ? a.order[p0 + p] : p0 + p;
                a.partial[(int64_t)pi * a.splits + split] = acc[p];
            }
    }
}

// Transposed mapping (shape (64, U)): one particle per lane.  A wave takes 64
// consecutive particles of the schedule order over one slice of the point
// list; each lane builds and keeps its own transform, the wave loads 64
// points at a time (one 16-byte load per lane) and hands them out one by one
// from lane registers (readlane: the point is wave-uniform).  Every gather
// instruction then looks up one point under 64 neighbouring poses of the
// schedule order: once the search radius has shrunk to a few centimetres
// these land in a handful of voxels, and the lanes share cache lines (a CPU
// count on the room frames: ~4 lanes per 128-byte line at r = 0.03, ~13 at
// 0.01, against ~1.1 when the lanes hold 64 neighbouring points).  U points
// are looked up per step, their gathers in flight together.  Slices, XCD
// mapping and the partial-sum layout are those of fitness_body, but a
// workgroup takes one group of 64 particles and its 4 waves take the 4
// quarters of the slice (4x the waves of one wave per group and slice, which
// the points-across slice counts would leave too few); each lane sums its
// particle's squares in point order, and the quarters are added in order
// through LDS.  Every exit before the barrier is uniform over the workgroup.
template <int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false>
__device__ void fitness_body_pl(const FitLaunch& a, const int blk) {
    __shared__ double s_part[4][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int s8 = a.splits >> 3;
    const int r = blk % a.splits;
    const int split = (r & 7) * s8 + (r >> 3);
    const int group = blk / a.splits;
    const int p0 = group * kWave;
    if (p0 >= a.n) return;
    if (FROM_STATE && (a.st->stopped || switch_skips(a))) return;
    const int m = a.count_dev ? *a.count_dev : a.count;

    const bool live = p0 + lane < a.n;
    int pi = live ? p0 + lane : a.n - 1;
    if (FROM_STATE && a.order) pi = a.order[pi];
    float V[12];
    {
        double T[12];
        if (FROM_STATE) {
            float p[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) p[d] = a.pst[6 * (int64_t)pi + d];
            particle_transform(a.st->qc, a.st->tc, a.st->r, p, T);
        } else {
#pragma unroll
            for (int e = 0; e < 12; ++e) T[e] = (double)a.T32[12 * (int64_t)pi + e];
        }
        fold_to_voxel(T, (double)a.g.vox, a.g.origin, V);
    }

    const Grid g = a.g;
    const VoxelTest ext{(float)g.nx, (float)g.ny, (float)g.nz};
    const int chunk = (m + a.splits - 1) / a.splits;
    const int s0 = split * chunk;
    const int s1 = min(m, s0 + chunk);
    const int quarter = (max(s1 - s0, 0) + 3) / 4;
    const int j0 = s0 + wave * quarter;
    const int j1 = min(s1, j0 + quarter);
    double acc = 0.0;
    float accf = 0.0f;
    for (int jb = j0; jb < j1; jb += kWave) {
        // wave-uniform, >= 1; held in a scalar register so that the lane
        // index of each broadcast below is scalar arithmetic
        const int cnt = __builtin_amdgcn_readfirstlane(min(kWave, j1 - jb));
        const float4 xl = a.pts[jb + (lane < cnt ? lane : 0)];
        for (int u0 = 0; u0 < cnt; u0 += U) {
            float v[U];
            if constexpr (LK == ROSE_LOOKUP_NEAREST) {
                uint32_t off[U];
                bool in[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int src = min(u0 + u, cnt - 1);
                    const float x = bcast(xl.x, src), y = bcast(xl.y, src), z = bcast(xl.z, src);
                    const float gx = xf_row(V[0], V[1], V[2], V[3], x, y, z);
                    const float gy = xf_row(V[4], V[5], V[6], V[7], x, y, z);
                    const float gz = xf_row(V[8], V[9], V[10], V[11], x, y, z);
                    in[u] = nearest_offset(g, ext, gx, gy, gz, &off[u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = gather<FMT, WIDE>(g.psi, off[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = in[u] ? v[u] : 1.0f;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int src = min(u0 + u, cnt - 1);
                    const float x = bcast(xl.x, src), y = bcast(xl.y, src), z = bcast(xl.z, src);
                    const float gx = xf_row(V[0], V[1], V[2], V[3], x, y, z);
                    const float gy = xf_row(V[4], V[5], V[6], V[7], x, y, z);
                    const float gz = xf_row(V[8], V[9], V[10], V[11], x, y, z);
                    v[u] = lookup_trilinear<FMT, WIDE>(g, gx, gy, gz);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = u0 + u < cnt;  // wave-uniform
                if constexpr (ACC32) {
                    const float d = ok ? v[u] : 0.0f;
                    accf = fmaf(d, d, accf);
                } else {
                    const double d = (double)(ok ? v[u] : 0.0f);
                    acc = fma(d, d, acc);
                }
            }
        }
    }
    s_part[wave][lane] = ACC32 ? (double)accf : acc;
    __syncthreads();
    if (wave == 0 && live) {
        double sum;
        if constexpr (ACC32) {
            float f = (float)s_part[0][lane];
#pragma unroll
            for (int w = 1; w < 4; ++w) f += (float)s_part[w][lane];
            sum = (double)f;
        } else {
            sum = s_part[0][lane];
#pragma unroll
            for (int w = 1; w < 4; ++w) sum += s_part[w][lane];
        }
        a.partial[(int64_t)pi * a.splits + split] = sum;
    }
}

template <int P, int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false>
__global__ __launch_bounds__(256) void k_fitness(FitLaunch a) {
    if constexpr (P == kWave) fitness_body_pl<U, FMT, LK, FROM_STATE, WIDE, ACC32>(a, blockIdx.x);
    else fitness_body<P, U, FMT, LK, FROM_STATE, WIDE, ACC32>(a, blockIdx.x);
}

// workgroups of a launch: 4 particle groups per workgroup (points across the
// lanes) or one (one particle per lane, its 4 waves splitting the slice)
int fitness_blocks(const FitLaunch& L, int P) {
    const int groups = (L.n + P - 1) / P;
    return (P == kWave ? groups : (groups + 3) / 4) * L.splits;
}

__device__ inline int fitness_blocks_dev(const FitLaunch& L, int P) {
    const int groups = (L.n + P - 1) / P;
    return (P == kWave ? groups : (groups + 3) / 4) * L.splits;
}

// Persistent fitness over many tracked sequences of one storage format and
// lookup (a batch launches one kernel per such group, so each kernel holds a
// single fitness body and keeps its registers): a grid of a few workgroups
// per CU walks the group's concatenated work lists [base, end) (sequence i
// owns items [begin[i], begin[i+1]), every begin a multiple of 8).  Items
// are handed out by one counter per XCD: workgroup b (on XCD b mod 8 -- the
// grid is a multiple of 8 and workgroups are dealt to the XCDs in turn)
// takes the next item w = base + (b mod 8) + 8 k of its XCD's queue, so the
// slice <-> XCD pairing of k_fitness holds for every sequence and the items
// in flight stay a contiguous window of the list (static striding lets slow
// and fast workgroups drift apart across sequences and volumes).  The
// counters (ctr[0..7]) are zero at launch: the kernel that runs before each
// launch on the stream clears them, and every workgroup leaves once its
// queue passes `end`.
template <int P, int U, int FMT, int LK>
__global__ __launch_bounds__(256) void k_fitness_batch(const FitLaunch* __restrict__ seqs,
                                                       const int* __restrict__ begin, int count, int base, int end,
                                                       int* __restrict__ ctr) {
    __shared__ int s_k;
    const int xcd = (int)(blockIdx.x & 7u);
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(&ctr[xcd], 1);
        __syncthreads();
        const int w = base + xcd + 8 * s_k;
        __syncthreads();
        if (w >= end) break;
        int lo = 0, hi = count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (begin[mid] <= w) lo = mid;
            else hi = mid;
        }
        const FitLaunch L = seqs[lo];  // wave-uniform: scalar loads of read-only memory
        const int blk = w - begin[lo];
        if (blk >= fitness_blocks_dev(L, P)) continue;
        // the particle-per-lane body synchronises its workgroup once; every
        // branch above is uniform over the workgroup (one item per workgroup)
        if constexpr (P == kWave) fitness_body_pl<U, FMT, LK, true, false>(L, blk);
        else fitness_body<P, U, FMT, LK, true, false>(L, blk);
    }
}

// A persistent grid must fit on the device at once: workgroups that only
// start when others finish would take their full static share of items late.
// grid = min(requested, resident workgroups of this kernel), a multiple of 8.
template <typename K>
static int resident_grid(K kernel, int requested) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), 256, 0) !=
            hipSuccess ||
        per_cu < 1)
        return std::max(8, requested / 8 * 8);
    return std::max(8, std::min(requested, cus * per_cu) / 8 * 8);
}

template <int P, int U, int FMT, int LK>
static void launch_batch_kernel(const FitLaunch* seqs, const int* begin, int count, int base, int end, int grid,
                                int* ctr, hipStream_t s) {
    hipLaunchKernelGGL((k_fitness_batch<P, U, FMT, LK>), dim3(grid), dim3(256), 0, s, seqs, begin, count, base, end,
                       ctr);
}

template <int P, int U>
static int batch_grid_shape(int fmt, int lk, int requested) {
    if (fmt == ROSE_TSDF_F32)
        return lk == ROSE_LOOKUP_TRILINEAR
                   ? resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_F32, ROSE_LOOKUP_TRILINEAR>, requested)
                   : resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_F32, ROSE_LOOKUP_NEAREST>, requested);
    if (fmt == ROSE_TSDF_F16)
        return lk == ROSE_LOOKUP_TRILINEAR
                   ? resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_F16, ROSE_LOOKUP_TRILINEAR>, requested)
                   : resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_F16, ROSE_LOOKUP_NEAREST>, requested);
    return lk == ROSE_LOOKUP_TRILINEAR
               ? resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_SN16, ROSE_LOOKUP_TRILINEAR>, requested)
               : resident_grid(&k_fitness_batch<P, U, ROSE_TSDF_SN16, ROSE_LOOKUP_NEAREST>, requested);
}

// grid of the persistent batch launch for a group (host query; call outside
// stream capture)
int batch_grid(int P, int U, int fmt, int lk, int requested) {
    if (P == kWave && U == 8) return batch_grid_shape<kWave, 8>(fmt, lk, requested);
    if (P == 8 && U == 4) return batch_grid_shape<8, 4>(fmt, lk, requested);
    if (P == 8 && U == 2) return batch_grid_shape<8, 2>(fmt, lk, requested);
    if (P == 4 && U == 4) return batch_grid_shape<4, 4>(fmt, lk, requested);
    return batch_grid_shape<4, 2>(fmt, lk, requested);
}

template <int P, int U>
static void launch_batch_shape(const FitLaunch* seqs, const int* begin, int count, int base, int end, int grid,
                               int fmt, int lk, int* ctr, hipStream_t s) {
    if (fmt == ROSE_TSDF_F32) {
        if (lk == ROSE_LOOKUP_TRILINEAR)
            launch_batch_kernel<P, U, ROSE_TSDF_F32, ROSE_LOOKUP_TRILINEAR>(seqs, begin, count, base, end, grid, ctr, s);
        else
            launch_batch_kernel<P, U, ROSE_TSDF_F32, ROSE_LOOKUP_NEAREST>(seqs, begin, count, base, end, grid, ctr, s);
    } else if (fmt == ROSE_TSDF_F16) {
        if (lk == ROSE_LOOKUP_TRILINEAR)
            launch_batch_kernel<P, U, ROSE_TSDF_F16, ROSE_LOOKUP_TRILINEAR>(seqs, begin, count, base, end, grid, ctr, s);
        else
            launch_batch_kernel<P, U, ROSE_TSDF_F16, ROSE_LOOKUP_NEAREST>(seqs, begin, count, base, end, grid, ctr, s);
    } else {
        if (lk == ROSE_LOOKUP_TRILINEAR)
            launch_batch_kernel<P, U, ROSE_TSDF_SN16, ROSE_LOOKUP_TRILINEAR>(seqs, begin, count, base, end, grid, ctr, s);
        else
            launch_batch_kernel<P, U, ROSE_TSDF_SN16, ROSE_LOOKUP_NEAREST>(seqs, begin, count, base, end, grid, ctr, s);
    }
}

bool batch_shape_valid(int P, int U) {
    return (P == 4 && U == 2) || (P == 8 && U == 2) || (P == 4 && U == 4) || (P == 8 && U == 4) ||
           (P == kWave && U == 8);
}

rose_status launch_fitness_batch(const FitLaunch* seqs_dev, const int* begin_dev, int count, int base, int end,
                                 int grid, int P, int U, int fmt, int lk, int* ctr_dev, hipStream_t s) {
    if (P == kWave && U == 8)
        launch_batch_shape<kWave, 8>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 8 && U == 4) launch_batch_shape<8, 4>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 8 && U == 2) launch_batch_shape<8, 2>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 4 && U == 4) launch_batch_shape<4, 4>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else launch_batch_shape<4, 2>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

// fitness_eval second pass: F_i = sum of slices / m (m = 0: F = 1)
__global__ __launch_bounds__(256) void k_fitness_finish(const double* partial, int32_t n, int32_t splits, int32_t m,
                                                        float* F, float* rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += partial[(int64_t)i * splits + k];
    const float f = (m > 0) ? (float)(s / (double)m) : 1.0f;
    F[i] = f;
    if (rho) rho[i] = (float)exp(-(double)f);
}

__global__ __launch_bounds__(256) void k_voxel_indices(Grid g, const float* pts, int32_t m, const float* T32,
                                                       int32_t n, int64_t* idx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * m) return;
    const int32_t i = (int32_t)(t / m), j = (int32_t)(t % m);
    double T[12];
    for (int e = 0; e < 12; ++e) T[e] = (double)T32[12 * (int64_t)i + e];
    float V[12];
    fold_to_voxel(T, (double)g.vox, g.origin, V);
    const float x = pts[3 * (int64_t)j], y = pts[3 * (int64_t)j + 1], z = pts[3 * (int64_t)j + 2];
    const float gx = xf_row(V[0], V[1], V[2], V[3], x, y, z);
    const float gy = xf_row(V[4], V[5], V[6], V[7], x, y, z);
    const float gz = xf_row(V[8], V[9], V[10], V[11], x, y, z);
    const bool in = gx >= 0.0f && gx < (float)g.nx && gy >= 0.0f && gy < (float)g.ny && gz >= 0.0f &&
                    gz < (float)g.nz;
    idx[t] = in ? (((int64_t)(uint32_t)gz * g.ny + (uint32_t)gy) * g.nx + (uint32_t)gx) : -1;
}

__global__ __launch_bounds__(256) void k_pack_points(const float* pts3, int32_t m, float4* pts4) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    pts4[j] = make_float4(pts3[3 * (int64_t)j], pts3[3 * (int64_t)j + 1], pts3[3 * (int64_t)j + 2], 0.0f);
}

// launch shape (particles per wave, points per lane per step); the tuner
// may change it process-wide
static int g_shape_p = 4, g_shape_u = 2;

template <int P, int U, int FMT, int LK, bool WIDE>
static void launch_pu(const FitLaunch& L, hipStream_t s) {
    const unsigned blocks = (unsigned)fitness_blocks(L, P);
    if (L.T32)
        hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, false, WIDE>), dim3(blocks), dim3(256), 0, s, L);
    else if constexpr (FMT == ROSE_TSDF_F32 && !WIDE) {
        if (L.acc32)
            hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE, true>), dim3(blocks), dim3(256), 0, s, L);
        else
            hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE>), dim3(blocks), dim3(256), 0, s, L);
    } else
        hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE>), dim3(blocks), dim3(256), 0, s, L);
}

template <int FMT, int LK>
static void launch_w(const FitLaunch& L, hipStream_t s) {
    const uint64_t bytes = (uint64_t)L.g.nx * L.g.ny * L.g.nz * (FMT == ROSE_TSDF_F32 ? 4u : 2u);
    if (bytes >= (uint64_t(1) << 32)) {
        launch_pu<4, 2, FMT, LK, true>(L, s);
        return;
    }
    const int p = L.shape_p, u = L.shape_u;
    if (p == 2 && u == 4) launch_pu<2, 4, FMT, LK, false>(L, s);
    else if (p == 4 && u == 4) launch_pu<4, 4, FMT, LK, false>(L, s);
    else if (p == 8 && u == 2) launch_pu<8, 2, FMT, LK, false>(L, s);
    else if (p == 8 && u == 4) launch_pu<8, 4, FMT, LK, false>(L, s);
    else if (p == kWave && u == 4) launch_pu<kWave, 4, FMT, LK, false>(L, s);
    else if (p == kWave && u == 8) launch_pu<kWave, 8, FMT, LK, false>(L, s);
    else if (p == kWave && u == 16) launch_pu<kWave, 16, FMT, LK, false>(L, s);
    else launch_pu<4, 2, FMT, LK, false>(L, s);
}

template <int FMT>
static void launch_f(const FitLaunch& L, hipStream_t s) {
    if (L.lookup == ROSE_LOOKUP_TRILINEAR) launch_w<FMT, ROSE_LOOKUP_TRILINEAR>(L, s);
    else launch_w<FMT, ROSE_LOOKUP_NEAREST>(L, s);
}

static void launch_fmt(const FitLaunch& L, hipStream_t s) {
    if (L.g.fmt == ROSE_TSDF_F32) launch_f<ROSE_TSDF_F32>(L, s);
    else if (L.g.fmt == ROSE_TSDF_F16) launch_f<ROSE_TSDF_F16>(L, s);
    else launch_f<ROSE_TSDF_SN16>(L, s);
}

rose_status launch_fitness(const FitLaunch& L, hipStream_t s) {
    const uint64_t bytes = (uint64_t)L.g.nx * L.g.ny * L.g.nz * (L.g.fmt == ROSE_TSDF_F32 ? 4u : 2u);
    if (L.pl_thr > 0.0f && L.st && !L.T32 && bytes < (uint64_t(1) << 32)) {
        // switched: the points-across kernel above the threshold (the given
        // shape; 4x2 for trilinear lookups, whose 8 gathers per evaluation
        // make deeper shapes register-bound: 1.80 ms for 4x2 against 2.80
        // for 8x4 on a room frame), the particle-per-lane kernel at or below
        // it; both write the same partial-sum slices
        FitLaunch a = L, b = L;
        a.pl_side = 2;
        if (L.lookup == ROSE_LOOKUP_TRILINEAR) {
            a.shape_p = 4;
            a.shape_u = 2;
        }
        b.pl_side = 1;
        b.shape_p = kWave;
        b.shape_u = 8;
        launch_fmt(a, s);
        launch_fmt(b, s);
    } else {
        FitLaunch a = L;
        a.pl_side = 0;
        launch_fmt(a, s);
    }
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

bool fitness_shape_valid(int p, int u) {
    return (p == 2 && u == 4) || (p == 4 && u == 2) || (p == 4 && u == 4) || (p == 8 && u == 2) ||
           (p == 8 && u == 4) || (p == kWave && (u == 4 || u == 8 || u == 16));
}

void fitness_shape(int* p, int* u) {
    *p = g_shape_p;
    *u = g_shape_u;
}

// switching mode: the points-across shape (8, 4) while the search footprint
// exceeds the threshold, one particle per lane (64, 8) at or below it.
// Default threshold 48 voxels at a 3 m reference depth, measured on the
// 640x480 room workload (1 cm voxels, 10240 particles): 8, 16, 32, 48, 64,
// 96 voxels -> 0.709, 0.703, 0.618, 0.595, 0.632, 0.638 ms per fitness step
// (fixed (8, 4): 0.707 ms, fixed (64, 8): 0.651 ms).  With one shared
// footprint for all six axes the crossover sits above the one measured with
// equal axis lengths (about 25 voxels): the largest axis overstates the
// spread of the others.
// Trilinear lookups (8 gathers per evaluation) cross over earlier: on the
// same workload 8, 16, 32, 48 voxels -> 2.099, 2.075, 2.055, 2.217 ms per
// step (4x2 alone: 2.100), so their default is 32.
static bool g_switch = false;
static float g_switch_vox[2] = {48.0f, 32.0f};  // by lookup: nearest, trilinear
static float g_switch_zref = 3.0f;

bool fitness_switching(int lookup, float* thr_vox, float* zref_m) {
    *thr_vox = g_switch ? g_switch_vox[lookup == ROSE_LOOKUP_TRILINEAR ? 1 : 0] : 0.0f;
    *zref_m = g_switch_zref;
    return g_switch;
}

// Point slices: a multiple of the 8 XCDs (see k_fitness).  For binary32
// volumes 16 (two slices per XCD, halving the particles in flight per XCD)
// once a slice keeps at least 512 points -- measured on the 640x480 room
// workload: 8 slices 0.737 ms per launch, 16: 0.692, 32: 0.701, 64: 0.710;
// the 16-bit volumes, half the bytes and resident in the Infinity Cache,
// lose with 16 (0.508 -> 0.577 ms) -- and raised further while the grid
// holds fewer waves than the chip runs at once and each slice still has at
// least ~4 lane-steps (256 points).
int choose_splits(int32_t n_particles, int64_t max_points, int32_t fmt, int P) {
    const int64_t groups = (n_particles + P - 1) / P;
    const int64_t target_waves = 256 * 4 * 8;  // CUs x SIMDs x waves per SIMD
    int64_t s = (fmt == ROSE_TSDF_F32 && max_points / 16 >= 512) ? 16 : 8;
    while (s < 64 && groups * s < target_waves && max_points / (2 * s) >= 256) s *= 2;
    return (int)s;
}

// Schedule order of template rows.  Waves take particles in this order, so
// that the particles evaluated together -- a wave's P, and the waves in
// flight on an XCD -- have similar poses and their gathers share cache lines
// in L1 and L2.  A particle's footprint moves with its rotation about
// (depth x angle) and with its translation, and at a few metres depth the
// rotation weighs most: the key interleaves, from the top bit down, 9 bits
// of each rotation coordinate with 7 bits of each translation coordinate (a
// Morton order in which rotation leads by two levels).  Any permutation
// gives the same fitness values (each particle's sums are written at its own
// index), so the order affects speed only.
static uint64_t order_key(const float* p) {
    uint32_t q[6];
    for (int d = 0; d < 6; ++d) {
        float v = p[d];
        if (!(v >= -1.0f)) v = -1.0f;  // also NaN
        if (v > 1.0f) v = 1.0f;
        const int bits = d < 3 ? 9 : 7;
        const uint32_t top = (1u << bits) - 1u;
        q[d] = std::min(top, (uint32_t)((v + 1.0f) * 0.5f * (float)(1u << bits)));
    }
    uint64_t key = 0;
    for (int lvl = 8; lvl >= 0; --lvl) {
        for (int d = 0; d < 3; ++d) key = (key << 1) | ((q[d] >> lvl) & 1u);
        if (lvl < 7)
            for (int d = 3; d < 6; ++d) key = (key << 1) | ((q[d] >> lvl) & 1u);
    }
    return key;
}

rose_status particle_order(rose_tsdf* h, const float* pst_dev, int32_t n, hipStream_t s, const int32_t** out) {
    *out = nullptr;
    for (int i = 0; i < h->n_orders; ++i)
        if (h->orders[i].pst == pst_dev && h->orders[i].n == n) {
            *out = h->orders[i].order;
            return ROSE_OK;
        }
    constexpr int kSlots = (int)(sizeof(h->orders) / sizeof(h->orders[0]));
    if (h->n_orders >= kSlots || n < 1) return ROSE_OK;  // index order
    std::vector<float> rows((size_t)n * 6);
    ROSE_CHECK_HIP(hipMemcpyAsync(rows.data(), pst_dev, sizeof(float) * rows.size(), hipMemcpyDeviceToHost, s));
    ROSE_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<uint64_t> key((size_t)n);
    std::vector<int32_t> idx((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        key[i] = order_key(&rows[6 * (size_t)i]);
        idx[i] = i;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    int32_t* dev = nullptr;
    ROSE_CHECK_HIP(hipMalloc(&dev, sizeof(int32_t) * (size_t)n));
    ROSE_CHECK_HIP(hipMemcpy(dev, idx.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
    h->orders[h->n_orders].pst = pst_dev;
    h->orders[h->n_orders].n = n;
    h->orders[h->n_orders].order = dev;
    h->n_orders += 1;
    *out = dev;
    return ROSE_OK;
}

}  // namespace rose

using namespace rose;

extern "C" {

rose_status fitness_eval(const rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                         rose_lookup lk, float* F_dev, float* rho_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && T_dev && F_dev && (pts_dev || m == 0), ROSE_E_ARG, "fitness_eval: NULL argument");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "fitness_eval: n = %d out of [1, %d]", n,
                 ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(m >= 0 && m <= ROSE_MAX_IMAGE_PIXELS, ROSE_E_ARG, "fitness_eval: m = %d out of range", m);
    ROSE_REQUIRE(lk == ROSE_LOOKUP_NEAREST || lk == ROSE_LOOKUP_TRILINEAR, ROSE_E_ARG, "fitness_eval: bad lookup");
    rose_tsdf* hm = const_cast<rose_tsdf*>(h);
    const int splits = choose_splits(n, m, h->g.fmt, g_shape_p);
    // scratch: packed points and partial sums, owned by the handle
    if (hm->cap_points < m) {
        if (hm->pts) ROSE_CHECK_HIP(hipFree(hm->pts));
        hm->pts = nullptr;
        ROSE_CHECK_HIP(hipMalloc(&hm->pts, sizeof(float4) * (size_t)(m > 0 ? m : 1)));
        hm->cap_points = m;
    }
    const int64_t need = (int64_t)n * splits;
    if (hm->cap_partial < need) {
        if (hm->partial) ROSE_CHECK_HIP(hipFree(hm->partial));
        hm->partial = nullptr;
        ROSE_CHECK_HIP(hipMalloc(&hm->partial, sizeof(double) * (size_t)need));
        hm->cap_partial = need;
    }
    if (m > 0) {
        hipLaunchKernelGGL(k_pack_points, dim3((m + 255) / 256), dim3(256), 0, s, pts_dev, m, hm->pts);
        ROSE_CHECK_HIP(hipGetLastError());
    }
    FitLaunch L{};
    L.g = h->g;
    L.pts = hm->pts;
    L.count_dev = nullptr;
    L.count = m;
    L.T32 = T_dev;
    L.n = n;
    L.splits = splits;
    L.lookup = lk;
    L.partial = hm->partial;
    fitness_shape(&L.shape_p, &L.shape_u);
    rose_status st = launch_fitness(L, s);
    if (st != ROSE_OK) return st;
    hipLaunchKernelGGL(k_fitness_finish, dim3((n + 255) / 256), dim3(256), 0, s, hm->partial, n, splits, m, F_dev,
                       rho_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status fitness_voxel_indices(const rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                                  int64_t* idx_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && pts_dev && T_dev && idx_dev, ROSE_E_ARG, "fitness_voxel_indices: NULL argument");
    ROSE_REQUIRE(n >= 1 && m >= 1 && (int64_t)n * m <= (int64_t(1) << 31), ROSE_E_ARG,
                 "fitness_voxel_indices: n*m out of range");
    const int64_t total = (int64_t)n * m;
    hipLaunchKernelGGL(k_voxel_indices, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, h->g, pts_dev, m,
                       T_dev, n, idx_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"

extern "C" rose_status rose_fitness_set_switch(float footprint_voxels, float reference_depth_m) {
    clear_error();
    if (footprint_voxels == 0.0f) {  // the defaults
        g_switch_vox[0] = 48.0f;
        g_switch_vox[1] = 32.0f;
        g_switch_zref = 3.0f;
        return ROSE_OK;
    }
    ROSE_REQUIRE(footprint_voxels > 0.0f && footprint_voxels <= 1.0e6f && reference_depth_m >= 0.0f &&
                     reference_depth_m <= 1.0e3f,
                 ROSE_E_ARG, "rose_fitness_set_switch: threshold %g voxels / depth %g m out of range",
                 (double)footprint_voxels, (double)reference_depth_m);
    g_switch_vox[0] = g_switch_vox[1] = footprint_voxels;
    g_switch_zref = reference_depth_m;
    return ROSE_OK;
}

extern "C" rose_status rose_fitness_set_shape(int32_t particles_per_wave, int32_t points_per_lane) {
    clear_error();
    if (particles_per_wave == 0 && points_per_lane == 0) {
        g_switch = true;
        g_shape_p = 8;
        g_shape_u = 4;
        return ROSE_OK;
    }
    ROSE_REQUIRE(fitness_shape_valid(particles_per_wave, points_per_lane), ROSE_E_UNSUPPORTED,
                 "rose_fitness_set_shape: (%d, %d) is not a compiled shape", particles_per_wave, points_per_lane);
    g_switch = false;
    g_shape_p = particles_per_wave;
    g_shape_u = points_per_lane;
    return ROSE_OK;
}
