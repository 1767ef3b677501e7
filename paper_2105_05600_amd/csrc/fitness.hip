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
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"

namespace rose {

template <int FMT>
__device__ inline uint32_t elem_bytes() {
    return FMT == ROSE_TSDF_F32 ? 4u : 2u;
}

// The psi buffer as a raw buffer resource (volumes below 4 GB): a gather is
// one buffer load with a 32-bit byte offset in a vector register and the
// base in scalar registers, and a load past the buffer's end returns 0
// instead of touching memory, so no offset needs clamping for safety (the
// value of an evaluation outside the grid is replaced by +1 anyway).
// The brick bits (Grid::ones) are read the same way.
struct PsiBuf {
    __amdgpu_buffer_rsrc_t r;
    __amdgpu_buffer_rsrc_t ones;
};

template <int FMT>
__device__ inline PsiBuf psi_buffer(const Grid& g) {
    const uint32_t bytes = (uint32_t)g.nx * (uint32_t)g.ny * (uint32_t)g.nz * elem_bytes<FMT>();
    const uint32_t words = ((uint32_t)g.nbx * (uint32_t)g.nby * (uint32_t)g.nbz + 31u) / 32u;
    // dword 3 of a raw (stride 0) buffer resource on gfx9-family targets
    return PsiBuf{__builtin_amdgcn_make_buffer_rsrc(g.psi, (short)0, (int)bytes, 0x00020000),
                  __builtin_amdgcn_make_buffer_rsrc(g.ones, (short)0, (int)(4u * words), 0x00020000)};
}

// whether the brick holding the voxel at element offset `off` is all +1
// (offset / 512 = brick; bit brick mod 32 of word brick / 32, at byte
// 4 (off >> 14))
__device__ inline bool brick_all_ones(const PsiBuf& b, uint32_t off) {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(b.ones, (int)((off >> 12) & ~3u), 0, 0);
    return __builtin_amdgcn_ubfe(w, off >> 9, 1) != 0u;
}

template <int FMT, bool WIDE>
__device__ inline float gather(const Grid& g, const PsiBuf& b, uint32_t off) {
    if constexpr (WIDE) {
        return load_psi<FMT>(g.psi, off);
    } else {
        const int bo = (int)(off * elem_bytes<FMT>());
        if constexpr (FMT == ROSE_TSDF_F32) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(b.r, bo, 0, 0));
        } else if constexpr (FMT == ROSE_TSDF_F16) {
            return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(b.r, bo, 0, 0)));
        } else {
            return (float)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(b.r, bo, 0, 0) * (1.0f / 32767.0f);
        }
    }
}

struct VoxelTest {
    uint32_t bx, by, bz;  // bit patterns of the grid extent as binary32
};

__device__ inline VoxelTest voxel_test(const Grid& g) {
    return VoxelTest{__float_as_uint((float)g.nx), __float_as_uint((float)g.ny), __float_as_uint((float)g.nz)};
}

// The voxel-space particle transform as the bounds test below needs it.  A
// transform with a non-finite entry makes every coordinate it produces NaN
// or infinite (an infinity never cancels to a finite value), i.e. every
// evaluation outside the grid: it is replaced by one that puts every point
// at -1 on each axis, also outside.  The translation entries get + 0, which
// turns -0 into +0 and leaves every other value as it is; then no
// coordinate of the fmaf chain is ever -0 (its innermost addend is not, and
// an exact zero sum rounds to +0).  No evaluation changes.
__device__ inline void sanitize_voxel_transform(float V[12]) {
    bool fin = true;
#pragma unroll
    for (int e = 0; e < 12; ++e) fin = fin && isfinite(V[e]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) V[4 * r + c] = fin ? V[4 * r + c] : 0.0f;
        V[4 * r + 3] = fin ? V[4 * r + 3] + 0.0f : -1.0f;
    }
}

// NEAREST voxel of voxel-space coordinate g: inside iff 0 <= g < n on every
// axis (NaN is outside); then floor(g) == (uint32)g.  The test compares the
// binary32 bit patterns as unsigned integers, one comparison per axis: for
// values >= +0 their order is the order of the values, and a negative
// value, -0 or NaN of either sign lies above every extent's pattern.  It
// equals the float test except at g = -0, which the sanitized transforms
// never produce.  Outside the grid the conversions saturate and the offset
// would be meaningless: it is replaced by one past the end of any buffer
// below 4 GB, where a buffer load fetches no cache line and returns 0 (WIDE
// volumes, read through plain pointers, get offset 0); the caller supplies
// the +1.
// The offset is computed for every lane (the volatile empty asm keeps the
// compiler from turning the select below into a branch around it).
template <bool WIDE>
__device__ inline bool nearest_offset(const Grid& g, const VoxelTest& e, float gx, float gy, float gz, uint32_t* off) {
    uint32_t o = brick_offset(g, (uint32_t)gx, (uint32_t)gy, (uint32_t)gz);
    asm volatile("" : "+v"(o));
    const bool in = (__float_as_uint(gx) < e.bx) & (__float_as_uint(gy) < e.by) & (__float_as_uint(gz) < e.bz);
    *off = in ? o : (WIDE ? 0u : 0xffffffffu);
    return in;
}

template <int FMT, bool WIDE>
__device__ inline float lookup_trilinear(const Grid& g, const PsiBuf& b, float gx, float gy, float gz) {
    const float hx = gx - 0.5f, hy = gy - 0.5f, hz = gz - 0.5f;
    const bool in = (hx >= 0.0f) & (hx < (float)(g.nx - 1)) & (hy >= 0.0f) & (hy < (float)(g.ny - 1)) &
                    (hz >= 0.0f) & (hz < (float)(g.nz - 1));
    const uint32_t ix = in ? (uint32_t)hx : 0u, iy = in ? (uint32_t)hy : 0u, iz = in ? (uint32_t)hz : 0u;
    const float fx = hx - (float)ix, fy = hy - (float)iy, fz = hz - (float)iz;
    const float v000 = gather<FMT, WIDE>(g, b, brick_offset(g, ix, iy, iz));
    const float v100 = gather<FMT, WIDE>(g, b, brick_offset(g, ix + 1, iy, iz));
    const float v010 = gather<FMT, WIDE>(g, b, brick_offset(g, ix, iy + 1, iz));
    const float v110 = gather<FMT, WIDE>(g, b, brick_offset(g, ix + 1, iy + 1, iz));
    const float v001 = gather<FMT, WIDE>(g, b, brick_offset(g, ix, iy, iz + 1));
    const float v101 = gather<FMT, WIDE>(g, b, brick_offset(g, ix + 1, iy, iz + 1));
    const float v011 = gather<FMT, WIDE>(g, b, brick_offset(g, ix, iy + 1, iz + 1));
    const float v111 = gather<FMT, WIDE>(g, b, brick_offset(g, ix + 1, iy + 1, iz + 1));
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

// psi of one evaluation from its voxel-space coordinate: NEAREST takes the
// voxel containing it (+1 outside the grid), TRILINEAR interpolates.
// Evaluations are done in batches of K: all K addresses first, then all K
// gathers (in flight together), then the selects.
template <int K, int FMT, int LK, bool WIDE>
__device__ inline void psi_batch(const Grid& g, const PsiBuf& b, const VoxelTest& ext, const float (&gx)[K],
                                 const float (&gy)[K], const float (&gz)[K], float (&v)[K]) {
    if constexpr (LK == ROSE_LOOKUP_NEAREST) {
        uint32_t off[K];
        bool in[K];
#pragma unroll
        for (int k = 0; k < K; ++k) in[k] = nearest_offset<WIDE>(g, ext, gx[k], gy[k], gz[k], &off[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = gather<FMT, WIDE>(g, b, off[k]);
        // select in binary32 (one v_cndmask); the empty asm keeps the
        // compiler from moving the select past the widening to binary64,
        // where it costs two
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = in[k] ? v[k] : 1.0f;
            asm("" : "+v"(v[k]));
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = lookup_trilinear<FMT, WIDE>(g, b, gx[k], gy[k], gz[k]);
    }
}

// add psi^2: on the 2^-39 grid (kGridBase + k per term; the caller removes
// kGridBase once per added term), or plain binary32 for the no-Kahan
// ablation
template <bool ACC32>
__device__ inline void add_sq(uint64_t& acc, float& accf, float v) {
    if constexpr (ACC32) accf = fmaf(v, v, accf);
    else acc += grid_term_bits(v);
}

// a binary32 sum (no-Kahan ablation) as a grid integer
__device__ inline uint64_t grid_of_f32_sum(float f) { return (uint64_t)__double2ull_rn((double)f * 0x1p39); }

template <int P, int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false>
__device__ void fitness_body(const FitLaunch& a, const int blk) {
    constexpr int kU = U;
    constexpr int kStep = kWave * kU;
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
        sanitize_voxel_transform(V);
    }
    // Up to 4 particles per wave: rotation entries wave-uniform in scalar
    // registers and the translation column broadcast with a cross-lane
    // shuffle, so that each fma reads at most one scalar operand.  With 8
    // particles the 72 rotation entries would crowd out the scalar registers
    // the loop needs (and spill), so all entries are broadcast to vector
    // registers.
    constexpr bool kRotScalar = true;
    float S[P][12];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < 12; ++e)
            S[p][e] = (!kRotScalar || e % 4 == 3) ? __shfl(V[e], p, kWave) : bcast(V[e], p);

    const Grid g = a.g;
    const PsiBuf pb = psi_buffer<FMT>(g);
    const VoxelTest ext = voxel_test(g);
    const int chunk = (m + a.splits - 1) / a.splits;
    const int j0 = split * chunk;
    const int j1 = min(m, j0 + chunk);
    uint64_t acc[P];  // grid sums (kGridBase + k per added term)
    float accf[P];    // ACC32: plain binary32 running sums
    // Evaluations outside the grid or in a brick that holds only +1 (psi =
    // +1, i.e. +1 to the sum each): with grid sums and NEAREST lookups they
    // are counted per particle on the scalar unit (a population count of the
    // wave's lanes) and their gathers aimed past the buffer's end, where the
    // load fetches no cache line and returns 0; the count is added after the
    // wave sum.  This keeps no per-evaluation lane mask alive across the
    // gathers (P x U of them would not fit the scalar registers), and when
    // the search spreads the particles far from the surfaces it spares the
    // gathers that land in free space (a fifth of all evaluations when the
    // axis lengths are 0.2).
    constexpr bool kCount = (LK == ROSE_LOOKUP_NEAREST) && !ACC32 && !WIDE;
    int nout[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        acc[p] = 0;
        accf[p] = 0.0f;
        nout[p] = 0;
    }
    auto eval = [&](const float4 (&x)[kU], const bool (&okl)[kU], float (&v)[kU][P]) {
        float gx[kU * P], gy[kU * P], gz[kU * P], w[kU * P];
        if constexpr (kCount) {
            // one particle's kU addresses at a time (the scheduling barriers
            // keep the compiler from computing every evaluation's bounds
            // test first, whose lane masks would not fit the scalar
            // registers), then all P x kU gathers in flight together
            uint32_t off[kU * P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int k = u * P + p;
                    gx[k] = xf_row(S[p][0], S[p][1], S[p][2], S[p][3], x[u].x, x[u].y, x[u].z);
                    gy[k] = xf_row(S[p][4], S[p][5], S[p][6], S[p][7], x[u].x, x[u].y, x[u].z);
                    gz[k] = xf_row(S[p][8], S[p][9], S[p][10], S[p][11], x[u].x, x[u].y, x[u].z);
                    bool in = nearest_offset<false>(g, ext, gx[k], gy[k], gz[k], &off[k]);
                    if (in && brick_all_ones(pb, off[k])) {
                        in = false;
                        off[k] = 0xffffffffu;
                    }
                    nout[p] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(!in && okl[u]));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
#pragma unroll
            for (int k = 0; k < kU * P; ++k) w[k] = gather<FMT, false>(g, pb, off[k]);
        } else {
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    gx[u * P + p] = xf_row(S[p][0], S[p][1], S[p][2], S[p][3], x[u].x, x[u].y, x[u].z);
                    gy[u * P + p] = xf_row(S[p][4], S[p][5], S[p][6], S[p][7], x[u].x, x[u].y, x[u].z);
                    gz[u * P + p] = xf_row(S[p][8], S[p][9], S[p][10], S[p][11], x[u].x, x[u].y, x[u].z);
                }
            psi_batch<kU * P, FMT, LK, WIDE>(g, pb, ext, gx, gy, gz, w);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int p = 0; p < P; ++p) v[u][p] = w[u * P + p];
    };
    bool all[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) all[u] = true;
    // full steps (every lane's kU points valid), the next step's points
    // loaded one step ahead so that their latency overlaps the gathers.  An
    // empty slice loads nothing (with no points at all the point buffer may
    // not exist) and writes a zero partial sum.
    const int nfull = (j1 > j0) ? (j1 - j0) / kStep : 0;
    float4 xn[kU];
    if (j1 > j0) {
#pragma unroll
        for (int u = 0; u < kU; ++u) xn[u] = a.pts[min(j0 + u * kWave + lane, j1 - 1)];
    }
    for (int st = 0; st < nfull; ++st) {
        float4 x[kU];
        const int jn = j0 + (st + 1) * kStep;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            x[u] = xn[u];
            xn[u] = a.pts[min(jn + u * kWave + lane, j1 - 1)];
        }
        float v[kU][P];
        eval(x, all, v);
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int p = 0; p < P; ++p) add_sq<ACC32>(acc[p], accf[p], v[u][p]);
    }
    // the last, partial step: lanes past the slice end add nothing
    const int jt = j0 + nfull * kStep;
    if (jt < j1) {
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) ok[u] = jt + u * kWave + lane < j1;
        float v[kU][P];
        eval(xn, ok, v);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
#pragma unroll
            for (int p = 0; p < P; ++p) add_sq<ACC32>(acc[p], accf[p], ok[u] ? v[u][p] : 0.0f);
        }
    }
    // every lane added kU terms per particle in each step it ran (lanes past
    // the slice end added 0); remove their kGridBase parts, modulo 2^64
    const uint64_t terms = (uint64_t)kWave * kU * (uint64_t)(nfull + (jt < j1 ? 1 : 0));
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if constexpr (ACC32) acc[p] = grid_of_f32_sum(wave_sum_f(accf[p]));
        else acc[p] = wave_sum_u64(acc[p]) - terms * kGridBase + (uint64_t)nout[p] * kGridOne;
    }
    if (lane == 0) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (p0 + p < a.n) {
                const int pi = (FROM_STATE && a.order) ? a.order[p0 + p] : p0 + p;
                uint64_t* dst = a.partial + partial_index(pi, a.splits, split, 0);
                dst[0] = acc[p];
#pragma unroll
                for (int q = 1; q < kPartSub; ++q) dst[q] = 0;
            }
    }
}


// Transposed mapping (shape (64, U)): one particle per lane.  A wave takes 64
// consecutive particles of the schedule order; each lane builds and keeps
// its own transform and the points are read U at a time from LDS
// (wave-uniform broadcasts).  Every gather instruction then looks up one
// point under 64 neighbouring poses of the schedule order: once the search
// radius has shrunk to a few centimetres these land in a handful of voxels,
// and the lanes share cache lines (a CPU count on the room frames: ~4 lanes
// per 128-byte line at r = 0.03, ~13 at 0.01, against ~1.1 when the lanes
// hold 64 neighbouring points).  The U gathers of a step are in flight
// together.  A workgroup takes 256 particles (its 4 waves, 64 consecutive
// particles each) and one quarter of a slice: the 4 waves evaluate the same
// points in step -- the workgroup stages them in LDS 64 at a time (one
// coalesced load by wave 0, the next batch loaded one batch ahead) -- so
// the neighbouring poses of its 256 particles gather from the same lines at
// about the same time and share them in the CU's L1.  Each lane sums its
// particle's squares over the quarter into the quarter's own partial slot.
// Slices and their XCD mapping are those of fitness_body counted in
// quarters (XCD x owns the contiguous quarter-slices x 4S/8 ...).  Every
// exit before a barrier is uniform over the workgroup.
template <int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false, int WG = 4>
__device__ void fitness_body_pl(const FitLaunch& a, const int blk) {
    __shared__ float4 s_pts[kWave];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int R = a.splits * kPartSub;  // quarter-slices, a multiple of 8
    const int r = blk % R;
    const int qs = (r & 7) * (R >> 3) + (r >> 3);
    const int split = qs / kPartSub, sub = qs % kPartSub;
    const int g4 = blk / R;
    if (g4 * WG * kWave >= a.n) return;
    if (FROM_STATE && (a.st->stopped || switch_skips(a))) return;
    const int m = a.count_dev ? *a.count_dev : a.count;

    const int p0 = (g4 * WG + wave) * kWave;
    const bool live = p0 + lane < a.n;  // a wave past the last particle still keeps the barriers
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
        sanitize_voxel_transform(V);
    }

    const Grid g = a.g;
    const PsiBuf pb = psi_buffer<FMT>(g);
    const VoxelTest ext = voxel_test(g);
    const int chunk = (m + a.splits - 1) / a.splits;
    const int s0 = split * chunk;
    const int s1 = min(m, s0 + chunk);
    const int quarter = (max(s1 - s0, 0) + kPartSub - 1) / kPartSub;
    const int j0 = __builtin_amdgcn_readfirstlane(s0 + sub * quarter);
    const int j1 = __builtin_amdgcn_readfirstlane(min(s1, j0 + quarter));
    uint64_t acc = 0;  // grid sum (kGridBase + k per added term)
    float accf = 0.0f;
    auto eval = [&](auto kk, int u0) {
        constexpr int K = decltype(kk)::value;
        float gx[K], gy[K], gz[K], v[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const float4 x = s_pts[u0 + u];
            gx[u] = xf_row(V[0], V[1], V[2], V[3], x.x, x.y, x.z);
            gy[u] = xf_row(V[4], V[5], V[6], V[7], x.x, x.y, x.z);
            gz[u] = xf_row(V[8], V[9], V[10], V[11], x.x, x.y, x.z);
        }
        psi_batch<K, FMT, LK, WIDE>(g, pb, ext, gx, gy, gz, v);
#pragma unroll
        for (int u = 0; u < K; ++u) add_sq<ACC32>(acc, accf, v[u]);
    };
    float4 xn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (wave == 0 && j0 < j1) xn = a.pts[min(j0 + lane, j1 - 1)];
    for (int jb = j0; jb < j1; jb += kWave) {
        const int cnt = min(kWave, j1 - jb);  // workgroup-uniform
        if (wave == 0) s_pts[lane] = xn;
        __syncthreads();
        if (wave == 0 && jb + kWave < j1) xn = a.pts[min(jb + kWave + lane, j1 - 1)];
        int u0 = 0;
        for (; u0 + U <= cnt; u0 += U) eval(std::integral_constant<int, U>{}, u0);
        for (; u0 < cnt; ++u0) eval(std::integral_constant<int, 1>{}, u0);
        __syncthreads();  // every wave's reads of the batch come before the next batch's write
    }
    // one term per point of the quarter (none for an empty quarter); the
    // no-Kahan ablation's binary32 sum is put on the grid per quarter
    if (live) {
        uint64_t sum;
        if constexpr (ACC32) sum = grid_of_f32_sum(accf);
        else sum = acc - (uint64_t)max(j1 - j0, 0) * kGridBase;
        a.partial[partial_index(pi, a.splits, split, sub)] = sum;
    }
}

// Wavefronts per workgroup of a particle-per-lane launch (its WG x 64
// particles share the staged points of one quarter-slice): 8 while that
// still leaves kPlWideMinBlocks workgroups or more (4 per CU), else 4 (the
// persistent batch kernel always runs 4).  On the 640x480 / 10240-particle
// room workload (1280 workgroups of 8) 8 waves took 92.8-93.0 ms over the
// bench's 275 particle-per-lane steps against 97.0-97.3 ms with 4 (16: 104.2
// ms); on 320x240 frames (640 workgroups of 8) and on 160x120 frames with
// 1024 particles (64) 8 waves were 7-10 % slower over whole sequences.
constexpr int kPlWaves = 8;
constexpr int kPlWideMinBlocks = 1024;

template <int P, int U, int FMT, int LK, bool FROM_STATE, bool WIDE, bool ACC32 = false, int WG = 4>
__global__ __launch_bounds__(P == kWave ? kWave * WG : 256) void k_fitness(FitLaunch a) {
    if constexpr (P == kWave) fitness_body_pl<U, FMT, LK, FROM_STATE, WIDE, ACC32, WG>(a, blockIdx.x);
    else fitness_body<P, U, FMT, LK, FROM_STATE, WIDE, ACC32>(a, blockIdx.x);
}

// work items of the persistent batch kernel (its workgroups: 4 particle
// groups and one slice (points across the lanes), or 4 groups of 64 and one
// quarter of a slice (one particle per lane)); also the workgroups of a
// points-across launch
int fitness_blocks(const FitLaunch& L, int P) {
    const int groups = (L.n + P - 1) / P;
    return (P == kWave ? (groups + 3) / 4 * kPartSub : (groups + 3) / 4) * L.splits;
}

__device__ inline int fitness_blocks_dev(const FitLaunch& L, int P) {
    const int groups = (L.n + P - 1) / P;
    return (P == kWave ? (groups + 3) / 4 * kPartSub : (groups + 3) / 4) * L.splits;
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
    if (P == 4 && U == 8) return batch_grid_shape<4, 8>(fmt, lk, requested);
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
           (P == 4 && U == 8) || (P == kWave && U == 8);
}

rose_status launch_fitness_batch(const FitLaunch* seqs_dev, const int* begin_dev, int count, int base, int end,
                                 int grid, int P, int U, int fmt, int lk, int* ctr_dev, hipStream_t s) {
    if (P == kWave && U == 8)
        launch_batch_shape<kWave, 8>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 8 && U == 4) launch_batch_shape<8, 4>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 4 && U == 8) launch_batch_shape<4, 8>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 8 && U == 2) launch_batch_shape<8, 2>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else if (P == 4 && U == 4) launch_batch_shape<4, 4>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    else launch_batch_shape<4, 2>(seqs_dev, begin_dev, count, base, end, grid, fmt, lk, ctr_dev, s);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

// fitness_eval second pass: F_i = sum of slices / m (m = 0: F = 1)
__global__ __launch_bounds__(256) void k_fitness_finish(const uint64_t* partial, int32_t n, int32_t splits,
                                                        int32_t m, float* F, float* rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t q = 0;
    const int S = splits * kPartSub;
    for (int k = 0; k < S; ++k) q += partial[(int64_t)i * S + k];
    const float f = (m > 0) ? (float)(((double)q * kGridScale) / (double)m) : 1.0f;
    F[i] = f;
    if (rho) rho[i] = (float)exp_rho(-(double)f);
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

// Process-wide default launch configuration (the tuner may change it); a
// handle with its own configuration (cfg_set) uses that instead.
// Switching-mode thresholds measured on the 640x480 room workload (1 cm
// voxels, 10240 particles): 8, 16, 32, 48, 64, 96 voxels at 3 m -> 0.709,
// 0.703, 0.618, 0.595, 0.632, 0.638 ms per fitness step (fixed (8, 4): 0.707
// ms, fixed (64, 8): 0.651 ms).  With one shared footprint for all six axes
// the crossover sits above the one measured with equal axis lengths (about
// 25 voxels): the largest axis overstates the spread of the others.
// Trilinear lookups (8 gathers per evaluation) cross over earlier: on the
// same workload 8, 16, 32, 48 voxels -> 2.099, 2.075, 2.055, 2.217 ms per
// step (4x2 alone: 2.100), so their default is 32.  The points-across
// shape of the switching mode: 4x2 (bench, 20 frames, three runs each:
// 3.698-3.706e11 evaluations/s against 3.632-3.634e11 for 4x4; 8x2 3.67e11,
// 2x4 3.63e11, 8x4 3.52e11, 4x8 3.46e11).
static const FitConfig kDefaultCfg = {4, 2, 0, 4, 2, {48.0f, 32.0f}, 3.0f};
static FitConfig g_cfg = kDefaultCfg;

FitConfig fit_config(const rose_tsdf* h) { return (h && h->cfg_set) ? h->cfg : g_cfg; }

void fit_launch_shape(const rose_tsdf* h, int lk, int* p, int* u, float* thr_vox, float* zref_m) {
    const FitConfig c = fit_config(h);
    if (c.sw) {
        // trilinear lookups (8 gathers per evaluation) keep (4, 2), deeper
        // shapes being register-bound there: 1.80 ms for 4x2 against 2.80
        // for 8x4 on a room frame
        const bool tri = lk == ROSE_LOOKUP_TRILINEAR;
        *p = tri ? 4 : c.wide_p;
        *u = tri ? 2 : c.wide_u;
        *thr_vox = c.thr_vox[tri ? 1 : 0];
    } else {
        *p = c.p;
        *u = c.u;
        *thr_vox = 0.0f;
    }
    *zref_m = c.zref;
}

template <int P, int U, int FMT, int LK, bool WIDE, int WG>
static void launch_pu_wg(const FitLaunch& L, unsigned blocks, hipStream_t s) {
    const dim3 threads(P == kWave ? kWave * WG : 256);
    if (L.T32)
        hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, false, WIDE, false, WG>), dim3(blocks), threads, 0, s, L);
    else if constexpr (FMT == ROSE_TSDF_F32 && !WIDE) {
        if (L.acc32)
            hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE, true, WG>), dim3(blocks), threads, 0, s, L);
        else
            hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE, false, WG>), dim3(blocks), threads, 0, s, L);
    } else
        hipLaunchKernelGGL((k_fitness<P, U, FMT, LK, true, WIDE, false, WG>), dim3(blocks), threads, 0, s, L);
}

template <int P, int U, int FMT, int LK, bool WIDE>
static void launch_pu(const FitLaunch& L, hipStream_t s) {
    // points across: 4 groups per workgroup and one slice; particle per
    // lane: WG groups of 64 per workgroup and one quarter-slice
    if constexpr (P == kWave) {
        const int groups = (L.n + kWave - 1) / kWave;
        const int wide = (groups + kPlWaves - 1) / kPlWaves * kPartSub * L.splits;
        if (wide >= kPlWideMinBlocks) {
            launch_pu_wg<P, U, FMT, LK, WIDE, kPlWaves>(L, (unsigned)wide, s);
            return;
        }
    }
    launch_pu_wg<P, U, FMT, LK, WIDE, 4>(L, (unsigned)fitness_blocks(L, P), s);
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
    else if (p == 4 && u == 8) launch_pu<4, 8, FMT, LK, false>(L, s);
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
        // switched: the points-across kernel (the given shape) above the
        // threshold, the particle-per-lane kernel at or below it; both write
        // the same partial-sum slices
        FitLaunch a = L, b = L;
        a.pl_side = 2;
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
    return (p == 2 && u == 4) || (p == 4 && u == 2) || (p == 4 && u == 4) || (p == 4 && u == 8) ||
           (p == 8 && u == 2) || (p == 8 && u == 4) || (p == kWave && (u == 4 || u == 8 || u == 16));
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

rose_status fitness_eval(rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                         rose_lookup lk, float* F_dev, float* rho_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && T_dev && F_dev && (pts_dev || m == 0), ROSE_E_ARG, "fitness_eval: NULL argument");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "fitness_eval: n = %d out of [1, %d]", n,
                 ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(m >= 0 && m <= ROSE_MAX_IMAGE_PIXELS, ROSE_E_ARG, "fitness_eval: m = %d out of range", m);
    ROSE_REQUIRE(lk == ROSE_LOOKUP_NEAREST || lk == ROSE_LOOKUP_TRILINEAR, ROSE_E_ARG, "fitness_eval: bad lookup");
    rose_tsdf* hm = h;
    int sp, su;
    float thr, zref;
    fit_launch_shape(h, lk, &sp, &su, &thr, &zref);
    const int splits = choose_splits(n, m, h->g.fmt, sp);
    // scratch: packed points and partial sums, owned by the handle
    if (hm->cap_points < m || !hm->pts) {
        if (hm->pts) ROSE_CHECK_HIP(hipFree(hm->pts));
        hm->pts = nullptr;
        const int64_t cap = m > 0 ? m : 1;
        ROSE_CHECK_HIP(hipMalloc(&hm->pts, sizeof(float4) * (size_t)cap));
        hm->cap_points = cap;
    }
    const int64_t need = (int64_t)n * splits * kPartSub;
    if (hm->cap_partial < need) {
        if (hm->partial) ROSE_CHECK_HIP(hipFree(hm->partial));
        hm->partial = nullptr;
        ROSE_CHECK_HIP(hipMalloc(&hm->partial, sizeof(uint64_t) * (size_t)need));
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
    L.shape_p = sp;
    L.shape_u = su;
    L.pl_thr = 0.0f;  // no device state: the switch needs the current axis lengths
    rose_status st = launch_fitness(L, s);
    if (st != ROSE_OK) return st;
    hipLaunchKernelGGL(k_fitness_finish, dim3((n + 255) / 256), dim3(256), 0, s, hm->partial, n, splits, m, F_dev,
                       rho_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free fitness
// fitness_eval_noalloc keeps its scratch -- the packed points and the
// (particle, slice) partial sums -- in one file-scope device array instead
// of the handle's grown buffers.  Each device holds its own copy for the
// life of the process; its address is looked up once per device, with that
// device current, and kept.  Every slot the kernels read is written earlier
// in the same call (the packing kernel writes the points, the fitness
// kernels every (particle, slice) sum), so nothing needs clearing; calls
// that overlap on one device share the array and race.
namespace rose {
constexpr int64_t kNoAllocPoints = 131072;    // 2 MiB of float4
constexpr int64_t kNoAllocPartials = 786432;  // 6 MiB of grid sums
struct NoAllocScratch {
    float4 pts[kNoAllocPoints];
    uint64_t partial[kNoAllocPartials];
};
static __device__ __align__(256) unsigned char scratch[sizeof(NoAllocScratch)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static NoAllocScratch* g_scratch_ptr[kMaxDevices] = {};

static rose_status noalloc_scratch(NoAllocScratch** out) {
    int dev = 0;
    ROSE_CHECK_HIP(hipGetDevice(&dev));
    ROSE_REQUIRE(dev >= 0 && dev < kMaxDevices, ROSE_E_DEVICE, "fitness_eval_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        ROSE_REQUIRE(e == hipSuccess && p != nullptr, ROSE_E_DEVICE,
                     "fitness_eval_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (NoAllocScratch*)p;
    }
    *out = g_scratch_ptr[dev];
    return ROSE_OK;
}
}  // namespace rose

extern "C" {

rose_status fitness_eval_noalloc(const rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                                 rose_lookup lk, float* F_dev, float* rho_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(h && T_dev && F_dev && (pts_dev || m == 0), ROSE_E_ARG, "fitness_eval_noalloc: NULL argument");
    ROSE_REQUIRE(n >= 1 && n <= ROSE_MAX_PARTICLES, ROSE_E_ARG, "fitness_eval_noalloc: n = %d out of [1, %d]", n,
                 ROSE_MAX_PARTICLES);
    ROSE_REQUIRE(m >= 0 && m <= kNoAllocPoints, ROSE_E_ARG, "fitness_eval_noalloc: m = %d out of [0, %lld]", m,
                 (long long)kNoAllocPoints);
    ROSE_REQUIRE(lk == ROSE_LOOKUP_NEAREST || lk == ROSE_LOOKUP_TRILINEAR, ROSE_E_ARG,
                 "fitness_eval_noalloc: bad lookup");
    int sp, su;
    float thr, zref;
    fit_launch_shape(h, lk, &sp, &su, &thr, &zref);
    const int splits = choose_splits(n, m, h->g.fmt, sp);
    ROSE_REQUIRE((int64_t)n * splits * kPartSub <= kNoAllocPartials, ROSE_E_ARG,
                 "fitness_eval_noalloc: %d particles x %d point slices x %d need more than the %lld partial sums of "
                 "the scratch",
                 n, splits, kPartSub, (long long)kNoAllocPartials);
    NoAllocScratch* sc = nullptr;
    rose_status st = noalloc_scratch(&sc);
    if (st != ROSE_OK) return st;
    if (m > 0) {
        hipLaunchKernelGGL(k_pack_points, dim3((m + 255) / 256), dim3(256), 0, s, pts_dev, m, sc->pts);
        ROSE_CHECK_HIP(hipGetLastError());
    }
    FitLaunch L{};
    L.g = h->g;
    L.pts = sc->pts;
    L.count_dev = nullptr;
    L.count = m;
    L.T32 = T_dev;
    L.n = n;
    L.splits = splits;
    L.lookup = lk;
    L.partial = sc->partial;
    L.shape_p = sp;
    L.shape_u = su;
    L.pl_thr = 0.0f;
    st = launch_fitness(L, s);
    if (st != ROSE_OK) return st;
    hipLaunchKernelGGL(k_fitness_finish, dim3((n + 255) / 256), dim3(256), 0, s, sc->partial, n, splits, m, F_dev,
                       rho_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

int32_t fitness_eval_noalloc_max_points(void) { return (int32_t)kNoAllocPoints; }

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

namespace rose {
// Shared by the process-wide and the per-handle setters.
static rose_status set_shape(FitConfig* c, int32_t p, int32_t u, const char* who) {
    if (p == 0 && u == 0) {
        c->sw = 1;
        return ROSE_OK;
    }
    ROSE_REQUIRE(fitness_shape_valid(p, u), ROSE_E_UNSUPPORTED, "%s: (%d, %d) is not a compiled shape", who, p, u);
    c->sw = 0;
    c->p = p;
    c->u = u;
    return ROSE_OK;
}

static rose_status set_switch(FitConfig* c, float vox, float zref, int32_t wide_p, int32_t wide_u, const char* who) {
    ROSE_REQUIRE(wide_p != kWave && fitness_shape_valid(wide_p, wide_u), ROSE_E_UNSUPPORTED,
                 "%s: (%d, %d) is not a compiled points-across shape", who, wide_p, wide_u);
    if (vox == 0.0f) {  // the default thresholds
        c->thr_vox[0] = kDefaultCfg.thr_vox[0];
        c->thr_vox[1] = kDefaultCfg.thr_vox[1];
        c->zref = kDefaultCfg.zref;
    } else {
        ROSE_REQUIRE(vox > 0.0f && vox <= 1.0e6f && zref >= 0.0f && zref <= 1.0e3f, ROSE_E_ARG,
                     "%s: threshold %g voxels / depth %g m out of range", who, (double)vox, (double)zref);
        c->thr_vox[0] = c->thr_vox[1] = vox;
        c->zref = zref;
    }
    c->wide_p = wide_p;
    c->wide_u = wide_u;
    return ROSE_OK;
}
}  // namespace rose

extern "C" rose_status rose_fitness_set_switch(float footprint_voxels, float reference_depth_m) {
    clear_error();
    return set_switch(&g_cfg, footprint_voxels, reference_depth_m, g_cfg.wide_p, g_cfg.wide_u,
                      "rose_fitness_set_switch");
}

extern "C" rose_status rose_fitness_set_switch_shape(int32_t particles_per_wave, int32_t points_per_lane) {
    clear_error();
    FitConfig c = g_cfg;
    rose_status st = set_switch(&c, 1.0f, 0.0f, particles_per_wave, points_per_lane, "rose_fitness_set_switch_shape");
    if (st != ROSE_OK) return st;
    g_cfg.wide_p = particles_per_wave;
    g_cfg.wide_u = points_per_lane;
    return ROSE_OK;
}

extern "C" rose_status rose_fitness_set_shape(int32_t particles_per_wave, int32_t points_per_lane) {
    clear_error();
    return set_shape(&g_cfg, particles_per_wave, points_per_lane, "rose_fitness_set_shape");
}

extern "C" rose_status tsdf_set_fitness_shape(rose_tsdf* h, int32_t particles_per_wave, int32_t points_per_lane) {
    clear_error();
    ROSE_REQUIRE(h != nullptr, ROSE_E_ARG, "tsdf_set_fitness_shape: NULL handle");
    if (particles_per_wave == -1 && points_per_lane == -1) {  // back to the process-wide default
        h->cfg_set = 0;
        return ROSE_OK;
    }
    FitConfig c = fit_config(h);
    rose_status st = set_shape(&c, particles_per_wave, points_per_lane, "tsdf_set_fitness_shape");
    if (st != ROSE_OK) return st;
    h->cfg = c;
    h->cfg_set = 1;
    return ROSE_OK;
}

extern "C" rose_status tsdf_set_fitness_switch(rose_tsdf* h, float footprint_voxels, float reference_depth_m,
                                               int32_t wide_particles, int32_t wide_points) {
    clear_error();
    ROSE_REQUIRE(h != nullptr, ROSE_E_ARG, "tsdf_set_fitness_switch: NULL handle");
    FitConfig c = fit_config(h);
    rose_status st = set_switch(&c, footprint_voxels, reference_depth_m, wide_particles, wide_points,
                                "tsdf_set_fitness_switch");
    if (st != ROSE_OK) return st;
    h->cfg = c;
    h->cfg_set = 1;
    return ROSE_OK;
}
