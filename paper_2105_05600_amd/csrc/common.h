// Internal definitions shared by the HIP translation units of librose.
//
// gfx950 (CDNA4): wave64, 160 KB LDS per CU.  All floating-point code is built
// with -ffp-contract=off: every fused multiply-add is an explicit fmaf / fma,
// so that the binary32 geometry (voxel and pixel choice) follows a fixed
// operation order.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstring>

#include "rose.h"

namespace rose {

constexpr int kWave = 64;

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

#define ROSE_CHECK_HIP(expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::rose::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                              __FILE__, __LINE__);                                        \
            return ROSE_E_DEVICE;                                                         \
        }                                                                                 \
    } while (0)

#define ROSE_REQUIRE(cond, code, ...)  \
    do {                               \
        if (!(cond)) {                 \
            ::rose::set_error(__VA_ARGS__); \
            return (code);             \
        }                              \
    } while (0)

// ----------------------------------------------- fitness launch configuration
struct FitConfig {
    int32_t p, u;           // fixed launch shape: particles per wave, points per lane per step
    int32_t sw;             // 1: switching mode (points-across above the footprint threshold,
                            // one particle per lane (64, 8) at or below it)
    int32_t wide_p, wide_u; // switching mode: the points-across shape (nearest lookups)
    float thr_vox[2];       // switching threshold by lookup (nearest, trilinear), voxels
    float zref;             // metres: depth at which a rotation axis length becomes a displacement
};

// -------------------------------------------------------------------- grid
struct Grid {
    int32_t nx, ny, nz;
    int32_t nbx, nby, nbz;      // bricks per axis (dimensions are multiples of 8)
    int32_t bstride_y;          // 64 nbx - 8     (brick_offset)
    int32_t bstride_z;          // 64 nbx nby - 64
    float vox, mu, w_max;
    float origin[3];
    int32_t fmt;  // rose_tsdf_fmt
    void* psi;
    void* wgt;
    // one bit per brick (brick-major order, 32 per word): set only while
    // every voxel of the brick decodes to exactly +1 (unobserved or free
    // space beyond the truncation band); cleared by fusion, rebuilt by
    // tsdf_create / tsdf_import / tsdf_rescan
    uint32_t* ones;
};

// Brick-major offset of voxel (i, j, k): bricks of 8x8x8 voxels in x-fastest
// brick order, voxels x-fastest inside a brick (brick index * 512 + in-brick
// offset), so that the voxels around a point share few cache lines (a
// 128-byte line holds an 8x4 patch of one z-slice) and few pages.  Written
// per axis: with i = 8a + b, i + 63 (i & ~7) = 512 a + b, and likewise
// 8 j + (64 nbx - 8)(j & ~7) and 64 k + (64 nbx nby - 64)(k & ~7), so the
// offset is three masks and five multiply-adds, every product a 24-bit
// multiply of in-volume indices (dimensions are at most 2048, brick
// strides below 2^22).  Callers pass in-volume indices or discard the
// offset.
__host__ __device__ inline uint32_t brick_offset(const Grid& g, uint32_t i, uint32_t j, uint32_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t a = __umul24(k & ~7u, (uint32_t)g.bstride_z) + __umul24(j & ~7u, (uint32_t)g.bstride_y);
    return a + __umul24(i & ~7u, 63u) + (k << 6) + (j << 3) + i;
#else
    const uint32_t b = ((k >> 3) * (uint32_t)g.nby + (j >> 3)) * (uint32_t)g.nbx + (i >> 3);
    return (b << 9) | ((k & 7u) << 6) | ((j & 7u) << 3) | (i & 7u);
#endif
}

// ------------------------------------------------------- TSDF value codecs
// F32: float psi, float weight.  F16: half psi (round to nearest even),
// u16 weight.  SN16: int16 psi = round(psi * 32767), u16 weight.
template <int FMT>
__device__ inline float load_psi(const void* base, uint32_t off) {
    if constexpr (FMT == ROSE_TSDF_F32) {
        return ((const float*)base)[off];
    } else if constexpr (FMT == ROSE_TSDF_F16) {
        return __half2float(((const __half*)base)[off]);
    } else {
        return (float)((const int16_t*)base)[off] * (1.0f / 32767.0f);
    }
}

template <int FMT>
__device__ inline void store_psi(void* base, uint32_t off, float v) {
    if constexpr (FMT == ROSE_TSDF_F32) {
        ((float*)base)[off] = v;
    } else if constexpr (FMT == ROSE_TSDF_F16) {
        ((__half*)base)[off] = __float2half_rn(v);
    } else {
        float s = rintf(fminf(fmaxf(v, -1.0f), 1.0f) * 32767.0f);
        ((int16_t*)base)[off] = (int16_t)s;
    }
}

template <int FMT>
__device__ inline float load_w(const void* base, uint32_t off) {
    if constexpr (FMT == ROSE_TSDF_F32) {
        return ((const float*)base)[off];
    } else {
        return (float)((const uint16_t*)base)[off];
    }
}

template <int FMT>
__device__ inline void store_w(void* base, uint32_t off, float v) {
    if constexpr (FMT == ROSE_TSDF_F32) {
        ((float*)base)[off] = v;
    } else {
        float c = rintf(fminf(fmaxf(v, 0.0f), 65535.0f));
        ((uint16_t*)base)[off] = (uint16_t)c;
    }
}

// ---------------------------------------------------------- pose algebra
// Binary64.  Quaternion (w, x, y, z), Hamilton product; a pose maps camera
// to world.
__host__ __device__ inline void quat_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__host__ __device__ inline void quat_prod(const double a[4], const double b[4], double c[4]) {
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    c[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// chart of the 6D state (q_x, q_y, q_z, x, y, z): quaternion
// (sqrt(1 - |u_123|^2), u_1, u_2, u_3) (imaginary part scaled to unit length
// and w = 0 when |u_123| > 1) and translation u_456.
__host__ __device__ inline void chart(const double u[6], double q[4], double t[3]) {
    const double s = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (s <= 1.0) {
        q[0] = sqrt(1.0 - s);
        q[1] = u[0];
        q[2] = u[1];
        q[3] = u[2];
    } else {
        const double n = sqrt(s);
        q[0] = 0.0;
        q[1] = u[0] / n;
        q[2] = u[1] / n;
        q[3] = u[2] / n;
    }
    t[0] = u[3];
    t[1] = u[4];
    t[2] = u[5];
}

// pose of a template particle: c * Delta(r (.) p)  -> 3x4 [R|t]
__host__ __device__ inline void particle_transform(const double qc[4], const double tc[3], const double r[6],
                                                   const float p[6], double T[12]) {
    double u[6], qd[4], td[3], q[4], R[9], Rc[9];
    for (int d = 0; d < 6; ++d) u[d] = r[d] * (double)p[d];
    chart(u, qd, td);
    quat_prod(qc, qd, q);
    quat_rot(q, R);
    quat_rot(qc, Rc);
    for (int i = 0; i < 3; ++i) {
        T[4 * i + 0] = R[3 * i + 0];
        T[4 * i + 1] = R[3 * i + 1];
        T[4 * i + 2] = R[3 * i + 2];
        const double rt = Rc[3 * i + 0] * td[0] + Rc[3 * i + 1] * td[1] + Rc[3 * i + 2] * td[2];
        T[4 * i + 3] = rt + tc[i];
    }
}

// MovePST of the centre: c <- c * Delta(u), quaternion renormalised, w >= 0
__host__ __device__ inline void retract(double qc[4], double tc[3], const double u[6]) {
    double qd[4], td[3], q[4], Rc[9], rt[3];
    chart(u, qd, td);
    quat_prod(qc, qd, q);
    quat_rot(qc, Rc);
    for (int i = 0; i < 3; ++i) rt[i] = Rc[3 * i + 0] * td[0] + Rc[3 * i + 1] * td[1] + Rc[3 * i + 2] * td[2];
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = (q[0] < 0.0) ? -1.0 : 1.0;
    for (int i = 0; i < 4; ++i) qc[i] = sg * q[i] / n;
    for (int i = 0; i < 3; ++i) tc[i] = rt[i] + tc[i];
}

__host__ __device__ inline void pose_matrix(const double q[4], const double t[3], double T[12]) {
    double R[9];
    quat_rot(q, R);
    for (int i = 0; i < 3; ++i) {
        T[4 * i + 0] = R[3 * i + 0];
        T[4 * i + 1] = R[3 * i + 1];
        T[4 * i + 2] = R[3 * i + 2];
        T[4 * i + 3] = t[i];
    }
}

// A = P^-1 C for rigid 3x4 transforms (P^-1 = [P_R^T | -P_R^T P_t])
__host__ __device__ inline void relative_transform(const double P[12], const double Cm[12], double A[12]) {
    double Pi[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Pi[4 * i + j] = P[4 * j + i];
        Pi[4 * i + 3] = -(P[0 * 4 + i] * P[3] + P[1 * 4 + i] * P[7] + P[2 * 4 + i] * P[11]);
    }
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = Pi[4 * i + 0] * Cm[0 * 4 + j] + Pi[4 * i + 1] * Cm[1 * 4 + j] + Pi[4 * i + 2] * Cm[2 * 4 + j];
            if (j == 3) s += Pi[4 * i + 3];
            A[4 * i + j] = s;
        }
    }
}

// camera->world transform folded with the voxel scaling, binary64, rounded
// once: V = [R / vox | (t - origin) / vox]
__host__ __device__ inline void fold_to_voxel(const double T[12], double vox, const float origin[3], float V[12]) {
    const double inv = 1.0 / vox;
    for (int c = 0; c < 3; ++c) {
        for (int j = 0; j < 3; ++j) V[4 * c + j] = (float)(T[4 * c + j] * inv);
        V[4 * c + 3] = (float)((T[4 * c + 3] - (double)origin[c]) * inv);
    }
}

// the binary32 rigid transform used everywhere: fmaf chain, x then y then z
__device__ inline float xf_row(float a0, float a1, float a2, float a3, float x, float y, float z) {
    return fmaf(a2, z, fmaf(a1, y, fmaf(a0, x, a3)));
}

// ------------------------------------------------------- device tracking state
struct DevState {
    double qc[4];
    double tc[3];
    double r[6];
    double r1[6];
    double Tprev[12];
    double rho_last;
    double thr;  // APS threshold carried between iterations (Eq. wafit)
    int32_t k;
    int32_t stopped;
    int32_t empty_streak;
    int32_t have_rho;
    int32_t n_points;
    int32_t n_overlap;
    int32_t status;
    int32_t pad;
    int32_t lvl_points[ROSE_MAX_LEVELS];  // valid samples per resolution level
    int32_t aps[ROSE_MAX_ITERS];
    int32_t n_overlap_iter[ROSE_MAX_ITERS];
    double rho_iter[ROSE_MAX_ITERS];
    double rho_centre[ROSE_MAX_ITERS];  // exact rho of c_{k-1} (particle 0) in iteration k
    double r_iter[ROSE_MAX_ITERS][6];   // axis lengths r_{k-1} of iteration k
};

// per-frame inputs of one tracked sequence
struct FrameIn {
    double qc[4], tc[3], r[6];  // PST centre c_0 and axis lengths r_0
    double Tprev[12];           // previous frame's final pose (overlap reference)
    const float* depth;         // current depth frame
    int32_t active;             // 0: nothing to do for this sequence
    int32_t pad;
};

// ------------------------------------------------- fitness sums on a grid
// Sums of psi^2 (Eq. ourlh) are exact on a grid of 2^-39: each term, exact in
// binary64 for a binary32 psi, is rounded once (to nearest, ties to even) to
// a multiple k 2^-39 and the integers k are added, so a sum does not depend
// on the order, the slicing or the launch shape that produced it.  The
// binary64 values in [2^13, 2^14) are spaced 2^-39 apart, so
// fma(d, d, 8192) = 8192 + k 2^-39 in one rounding and its bit pattern is
// kGridBase + k.  A term psi^2 = 1 (outside the grid) is kGridOne; k <= 2^39
// and at most 2^24 terms per sum keep every sum below 2^63.
constexpr uint64_t kGridBase = 0x40C0000000000000ull;  // bits of 8192.0
constexpr uint64_t kGridOne = 1ull << 39;
constexpr double kGridScale = 0x1p-39;

// kGridBase + k for the term v^2 (a per-lane accumulator adds these and
// subtracts kGridBase once per added term, modulo 2^64)
__device__ inline uint64_t grid_term_bits(float v) {
    const double d = (double)v;
    return (uint64_t)__double_as_longlong(fma(d, d, 8192.0));
}

// exp(x) for the likelihoods rho = exp(-F / tau) (Eq. pfolh): k = rint(x /
// ln 2), r = x - k ln 2 with ln 2 split in two binary64 parts (one fma
// each), exp(r) by its Taylor series to degree 13 by Horner's rule (one fma
// per step, |r| <= ln 2 / 2: truncation below 1e-17), scaled by 2^k.  Every
// step is a correctly rounded binary64 operation, so the result is a fixed
// function of x on any IEEE host or device.
__host__ __device__ inline double exp_rho(double x) {
    const double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;
    if (!(x > -1100.0)) return 0.0;  // also NaN -> 0 (never produced: F is finite)
    const double k = rint(x * 0x1.71547652b82fep0);  // x / ln 2
    double r = fma(-k, kLn2Hi, x);
    r = fma(-k, kLn2Lo, r);
    double fact = 1.0;
    for (int n = 2; n <= 13; ++n) fact *= (double)n;  // 13! = 6227020800, exact
    double p = 1.0 / fact;
    for (int n = 13; n >= 1; --n) {
        fact /= (double)n;          // (n-1)!, exact
        p = fma(p, r, 1.0 / fact);  // c_{n-1} = 1/(n-1)!
    }
    return ldexp(p, (int)k);
}

// --------------------------------------------------------- wave primitives
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, off, kWave);
    return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Order-preserving block compaction step: flag per thread -> exclusive
// position among flagged threads of the block; *total receives the count.
// lds must hold blockDim.x / 64 + 1 ints.  Uses two __syncthreads().
__device__ inline int block_scan_flag(int flag, int* lds, int* total) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const uint64_t m = __ballot(flag);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int in_wave = __popcll(m & lt);
    if (lane == 0) lds[wid] = __popcll(m);
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const int c = lds[w];
        base += (w < wid) ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return base + in_wave;
}

// ------------------------------------------------------------ host helpers
struct Scratch;  // defined in api.hip

}  // namespace rose

// Handle.  The TSDF buffers are the caller's; the tracking scratch below is
// owned by the handle and released by tsdf_destroy.
struct rose_tsdf {
    rose::Grid g;
    int device;
    rose::FitConfig cfg;  // own fitness launch configuration while cfg_set
    int32_t cfg_set;
    // tracking scratch (device)
    float4* pts;        // all valid subsampled points of the current frame
    float4* pts_o;      // overlap-compacted points
    uint64_t* partial;  // n_particles x splits partial sums of psi^2 (grid integers)
    float* F;           // n_particles fitness values of the last iteration
    rose::DevState* st; // device state of the current frame
    rose::DevState* st_host;  // pinned host copy
    rose::FrameIn* learn_in;  // pinned: the learned frame's proposal (c_0, r_0) and its finite flag
    int32_t* learn_ok;
    int64_t cap_points;
    int64_t cap_points_o;
    int64_t cap_partial;
    int64_t cap_particles;
    // comparison optimisers' scratch (swarm.hip), n particles
    float* sw_x;        // 2 x n x 6 states (current, next)
    float* sw_v;        // n x 6 velocities
    float* sw_p;        // n x 6 personal bests
    float* sw_pF;       // n personal best fitness values
    double* sw_C;       // n cumulative resampling weights
    void* sw_st;        // device search state
    void* sw_host;      // pinned host copy
    int64_t cap_swarm;
    // schedule orders of the PST templates tracked with this handle (fitness.hip)
    struct Order {
        const float* pst;
        int32_t n;
        int32_t* order;
    } orders[8];
    int32_t n_orders;
};

namespace rose {

// Fitness launch (fitness.hip).  Pose source: explicit binary32 transforms
// (T32 != nullptr) or the PST of the device tracking state (st, pst).
struct FitLaunch {
    Grid g;
    const float4* pts;
    const int32_t* count_dev;  // device point count, or nullptr to use `count`
    int32_t count;
    const float* T32;
    const DevState* st;
    const float* pst;
    const int32_t* order;      // schedule order of the template rows (n), or nullptr (index order)
    int32_t n;
    int32_t splits;
    int32_t lookup;
    int32_t shape_p, shape_u;  // particles per wave, points per lane per step
    int32_t acc32;             // 1: plain binary32 sums (ROSE_FLAG_NO_KAHAN), FROM_STATE binary32 volumes only
    // mapping switch (FROM_STATE launches): side 1 runs only while the
    // search footprint is at most pl_thr voxels, side 2 only above it; 0: always
    int32_t pl_side;
    float pl_thr;   // voxels
    float pl_zref;  // metres: depth at which a rotation axis length is turned into a displacement
    uint64_t* partial;         // n x splits x kPartSub grid integers (partial_index)
};

// Partial sums: every (particle, slice) owns kPartSub consecutive slots.  The
// particle-per-lane kernel's workgroups take a quarter of a slice for 256
// particles and each writes its quarter's sum to its own slot; the
// points-across kernel writes its slice's sum to the first slot and zeros to
// the others.  A particle's fitness is the sum of its splits x kPartSub
// consecutive slots (integers on the 2^-39 grid, so the order is free).
constexpr int kPartSub = 4;
__host__ __device__ inline int64_t partial_index(int64_t pi, int splits, int split, int sub) {
    return (pi * splits + split) * kPartSub + sub;
}
rose_status launch_fitness(const FitLaunch& L, hipStream_t s);

// The switching mode's footprint test: the largest translation axis length
// plus zref times the largest rotation axis length, at most thr voxels of
// size vox (axis lengths r: 3 rotation, then 3 translation).  Every kernel
// that takes the decision evaluates this same expression on the same state.
__host__ __device__ inline bool footprint_small(const double* r, float zref, float thr, float vox) {
    const double rr = fmax(fmax(r[0], r[1]), r[2]);
    const double rt = fmax(fmax(r[3], r[4]), r[5]);
    return (rt + (double)zref * rr) <= (double)thr * (double)vox;
}

// Schedule order of the first n rows of a PST template (cached per handle;
// the first request reads the template back, synchronising s).  nullptr
// (index order) when the handle's cache is full.
rose_status particle_order(rose_tsdf* h, const float* pst_dev, int32_t n, hipStream_t s, const int32_t** out);
// point slices for n particles in waves of P (the launch shape's first entry)
int choose_splits(int32_t n_particles, int64_t max_points, int32_t fmt, int P);
bool fitness_shape_valid(int p, int u);
// The effective launch configuration of a handle: its own (tsdf_set_fitness_*)
// or else the process-wide default (rose_fitness_set_*).
FitConfig fit_config(const rose_tsdf* h);
// Launch shape (and switch threshold, 0 = no switch) a handle's fitness
// launches use for lookup lk: the fixed shape, or in the switching mode the
// points-across side (its wide shape; (4, 2) for trilinear lookups).
void fit_launch_shape(const rose_tsdf* h, int lk, int* p, int* u, float* thr_vox, float* zref_m);
int fitness_blocks(const FitLaunch& L, int P);
bool batch_shape_valid(int p, int u);
int batch_grid(int P, int U, int fmt, int lk, int requested);
// ctr_dev: the group's 8 per-XCD work counters, zero at launch
rose_status launch_fitness_batch(const FitLaunch* seqs_dev, const int* begin_dev, int count, int base, int end,
                                 int grid, int P, int U, int fmt, int lk, int* ctr_dev, hipStream_t s);

// PST template rows 0..n-1 (tsdf.hip)
rose_status launch_pst_sample(int64_t n, uint64_t seed, float* out_dev, hipStream_t s);

// kernel timing (profile.hip)
enum { PROF_FITNESS = 0, PROF_UPDATE = 1, PROF_INTEGRATE = 2 };
bool prof_on();
int prof_begin(int kind, hipStream_t s);          // -1 when timing is off
void prof_end(int tok, hipStream_t s, double evals);
void prof_set_evals(int tok, double evals);

}  // namespace rose
