/*
 * rose_oracle.c -- plain, slow CPU oracle for PST pose search against a TSDF
 * (ROSEFusion, Zhang et al., ACM TOG 40(4) 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library, and it includes nothing from it.
 *
 * Every function is a direct transcription of the definition it cites
 * (section / equation of the paper), in plain loops.  Two of them may split
 * their outer loop over host threads (orc_set_threads): the fitness over
 * contiguous particle ranges and the fusion over z-slices of the volume.
 * Each particle's (each voxel's) arithmetic and point order are unchanged,
 * so the results do not depend on the thread count (pinned by the tests).
 *
 * Precision.  Two modes exist for the geometric steps whose floating-point
 * result decides an integer (which voxel, which pixel, inside or outside):
 *   ORC_F64 : everything in binary64 -- the definition itself;
 *   ORC_F32 : the decision is taken in binary32, the precision of the GPU
 *             kernels, with the operation order written next to each step,
 *             so that integer outcomes (voxel and pixel indices) can be
 *             compared bit for bit.
 * Sums of squared TSDF values: ORC_F64 adds them in binary64 with Neumaier
 * compensation; ORC_F32 adds them exactly on a 2^-39 grid (each term
 * rounded once to a multiple of 2^-39, the multiples added as integers), so
 * that the sum does not depend on the order of its terms.  The PST update
 * (Alg. 1 / Eqs. ebs, rsdir, rsinter, momentum, wafit) and pose algebra are
 * always binary64; the likelihood exp(-F / tau) is orc_exp below.
 *
 * Parity status of each function is stated in the oracle's README block in
 * oracle/__init__.py and in the design notes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* exp(x) for the likelihoods rho = exp(-F / tau) (Eq. pfolh), a fixed      */
/* function of x: Cody-Waite reduction x = k ln2 + r with k = rint(x / ln2) */
/* and ln2 given as a binary64 head and tail (one fma each), exp(r) from    */
/* its Taylor series sum_{n<=13} r^n / n! by Horner's rule (one fma per     */
/* step; |r| <= ln2 / 2, truncation error below 1e-17), then 2^k scaling.   */
/* Every step is one correctly rounded binary64 operation.                  */
/* ------------------------------------------------------------------------ */
double orc_exp(double x) {
    static const double ln2_head = 0x1.62e42fefa39efp-1;  /* ln 2 rounded to binary64 */
    static const double ln2_tail = 0x1.abc9e3b39803fp-56; /* ln 2 - ln2_head */
    static const double inv_ln2 = 0x1.71547652b82fep0;    /* 1 / ln 2 rounded */
    if (!(x > -1100.0)) return 0.0;                       /* exp underflows to 0 well before */
    double k = rint(x * inv_ln2);
    double r = fma(-k, ln2_head, x);
    r = fma(-k, ln2_tail, r);
    /* c[n] = 1 / n!  (n! is exact in binary64 for n <= 13) */
    double c[14];
    double f = 1.0;
    for (int n = 0; n <= 13; ++n) {
        if (n > 0) f *= (double)n;
        c[n] = 1.0 / f;
    }
    double p = c[13];
    for (int n = 12; n >= 0; --n) p = fma(p, r, c[n]);
    return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------------ */
/* Host threads for the two loops that may be split (see the header).  One  */
/* thread by default.                                                       */
/* ------------------------------------------------------------------------ */
#define ORC_MAX_THREADS 256
static int g_threads = 1;

void orc_set_threads(int32_t n) { g_threads = n < 1 ? 1 : (n > ORC_MAX_THREADS ? ORC_MAX_THREADS : n); }
int32_t orc_get_threads(void) { return g_threads; }

/* run fn(arg_t, t0, t1) for T contiguous ranges [t0, t1) of [0, n) */
typedef void (*orc_range_fn)(void* arg, int64_t t0, int64_t t1);
typedef struct {
    orc_range_fn fn;
    void* arg;
    int64_t t0, t1;
} orc_range_job;

static void* orc_range_main(void* p) {
    orc_range_job* j = (orc_range_job*)p;
    j->fn(j->arg, j->t0, j->t1);
    return NULL;
}

static void orc_parallel_ranges(orc_range_fn fn, void* arg, int64_t n) {
    int64_t T = g_threads;
    if (T > n) T = n;
    if (T <= 1) {
        fn(arg, 0, n);
        return;
    }
    orc_range_job jobs[ORC_MAX_THREADS];
    pthread_t tid[ORC_MAX_THREADS];
    int started[ORC_MAX_THREADS];
    for (int64_t t = 0; t < T; ++t) {
        jobs[t].fn = fn;
        jobs[t].arg = arg;
        jobs[t].t0 = n * t / T;
        jobs[t].t1 = n * (t + 1) / T;
    }
    /* threads 1..T-1 run beside the caller, which takes range 0; a thread  */
    /* that cannot be started runs its range on the caller afterwards       */
    for (int64_t t = 1; t < T; ++t) started[t] = pthread_create(&tid[t], NULL, orc_range_main, &jobs[t]) == 0;
    fn(arg, jobs[0].t0, jobs[0].t1);
    for (int64_t t = 1; t < T; ++t) {
        if (started[t]) pthread_join(tid[t], NULL);
        else fn(arg, jobs[t].t0, jobs[t].t1);
    }
}

#define ORC_F64 0
#define ORC_F32 1

#define ORC_LOOKUP_NEAREST 0
#define ORC_LOOKUP_TRILINEAR 1

/* flag bits of the tracker (ablation switches of Sec. 5.2, Tab. ablt-tsdf) */
#define ORC_NO_OVERLAP 1
#define ORC_NO_NORMALIZE 2
#define ORC_CENTRE_THRESHOLD 4
#define ORC_ISO_ONLY 8   /* rescaling ablation: isotropic part of Eq. rsinter only */
#define ORC_ANISO_ONLY 16 /* rescaling ablation: anisotropic part of Eq. rsinter only */
#define ORC_NO_KAHAN 32   /* TSDF-normalisation ablation: plain binary32 summation of psi^2 */

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11, */
/* "Parallel random numbers: as easy as 1, 2, 3").  Ten rounds of the       */
/* Philox S-box with the published multipliers and Weyl key increments.     */
/* ------------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, x0, &hi0, &lo0);
        mul128(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* PST template (Sec. 3.3 "pre-sample ... uniformly within the unit sphere  */
/* in the 6D state space"; Sec. 4 "PST pre-sampling").                      */
/* Row 0 is the origin (the PST centre itself).  Row i>0: attempt a = 0,1,..*/
/* draws one Philox block with counter (i, a, 0, 0) and key (seed, 0); six  */
/* 24-bit fields m_d are cut from the top of words 0..2 (bits 63..40 and    */
/* 39..16); a_d = 2 m_d + 1 - 2^24 (odd, |a_d| < 2^24); the draw is kept    */
/* iff sum a_d^2 <= 2^48, i.e. the point a*2^-24 lies in the closed unit    */
/* ball (exact integer test); p_d = a_d * 2^-24 (exact in binary32).        */
/* After 1024 rejected attempts the row is the zero vector.                 */
/* Returns the number of rows that hit the attempt cap.                     */
/* ------------------------------------------------------------------------ */
int orc_pst_sample(int32_t n, uint64_t seed, float* out) {
    int capped = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 6; ++d) out[6 * (size_t)i + d] = 0.0f;
        if (i == 0) continue;
        int ok = 0;
        for (uint64_t a = 0; a < 1024 && !ok; ++a) {
            uint64_t ctr[4] = {(uint64_t)i, a, 0, 0}, key[2] = {seed, 0}, w[4];
            orc_philox4x64_10(ctr, key, w);
            int64_t m[6];
            m[0] = (int64_t)(w[0] >> 40);
            m[1] = (int64_t)((w[0] >> 16) & 0xFFFFFF);
            m[2] = (int64_t)(w[1] >> 40);
            m[3] = (int64_t)((w[1] >> 16) & 0xFFFFFF);
            m[4] = (int64_t)(w[2] >> 40);
            m[5] = (int64_t)((w[2] >> 16) & 0xFFFFFF);
            int64_t s = 0, av[6];
            for (int d = 0; d < 6; ++d) {
                av[d] = 2 * m[d] + 1 - (1LL << 24);
                s += av[d] * av[d];
            }
            if (s <= (1LL << 48)) {
                for (int d = 0; d < 6; ++d) out[6 * (size_t)i + d] = (float)ldexp((double)av[d], -24);
                ok = 1;
            }
        }
        if (!ok) ++capped;
    }
    return capped;
}

/* ------------------------------------------------------------------------ */
/* 6D Poisson-disk PST (Sec. 4 "PST pre-sampling": the template is a 6D     */
/* Poisson-disk sample of the unit ball).  Dart throwing: the candidates   */
/* are rows 1, 2, ... of orc_pst_sample(seed) (uniform in the unit ball);  */
/* the origin is accepted first; a candidate is accepted iff its squared   */
/* distance to every point accepted before it is >= r_min^2.  Distances    */
/* are taken on the sampler's integer lattice (p = a 2^-24, a odd integers */
/* below 2^24), where sum (a - b)^2 < 6 * 2^50 is exact in int64; the      */
/* threshold is d2 = ceil(r_min^2 2^48) evaluated in binary64.             */
/* Stops when n points are accepted or max_cand candidates were drawn.     */
/* Returns the number of accepted rows (n on success); rows past it are 0; */
/* *drawn = the number of candidates drawn.                                */
/* ------------------------------------------------------------------------ */
int32_t orc_pst_poisson(int32_t n, uint64_t seed, double r_min, int32_t max_cand, float* out, int32_t* drawn) {
    const int64_t d2 = (int64_t)ceil(r_min * r_min * 281474976710656.0);
    float* cand = (float*)malloc(sizeof(float) * 6 * ((size_t)max_cand + 1));
    int64_t* acc = (int64_t*)malloc(sizeof(int64_t) * 6 * (size_t)(n > 0 ? n : 1));
    orc_pst_sample(max_cand + 1, seed, cand);
    for (size_t e = 0; e < 6 * (size_t)n; ++e) out[e] = 0.0f;
    int32_t count = 0;
    if (n > 0) {
        for (int d = 0; d < 6; ++d) acc[d] = 0;
        count = 1;
    }
    int32_t c = 1;
    for (; c <= max_cand && count < n; ++c) {
        int64_t a[6];
        for (int d = 0; d < 6; ++d) a[d] = (int64_t)ldexp((double)cand[6 * (size_t)c + d], 24);
        int far = 1;
        for (int32_t k = 0; k < count && far; ++k) {
            int64_t s = 0;
            for (int d = 0; d < 6; ++d) {
                const int64_t df = a[d] - acc[6 * (size_t)k + d];
                s += df * df;
            }
            far = (s >= d2);
        }
        if (!far) continue;
        for (int d = 0; d < 6; ++d) {
            acc[6 * (size_t)count + d] = a[d];
            out[6 * (size_t)count + d] = cand[6 * (size_t)c + d];
        }
        ++count;
    }
    *drawn = c - 1;
    free(cand);
    free(acc);
    return count;
}

/* ------------------------------------------------------------------------ */
/* Pose algebra, binary64.  A pose is (q, t): unit quaternion q = (w,x,y,z) */
/* (Hamilton convention) and translation t; it maps camera to world,        */
/* X = R(q) x + t (Eq. unproj).                                             */
/* ------------------------------------------------------------------------ */
void orc_quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
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

void orc_quat_mul(const double a[4], const double b[4], double c[4]) {
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    c[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

static void rot_apply(const double R[9], const double v[3], double o[3]) {
    for (int i = 0; i < 3; ++i) o[i] = R[3 * i + 0] * v[0] + R[3 * i + 1] * v[1] + R[3 * i + 2] * v[2];
}

/* The 6D state of Sec. 3.3, s = (q_x, q_y, q_z, x, y, z), read as a local  */
/* chart: u -> Delta(u) with quaternion (sqrt(1-|u_123|^2), u1, u2, u3) and */
/* translation (u4, u5, u6).  If |u_123| > 1 the imaginary part is scaled   */
/* to unit length and w = 0.                                                */
void orc_chart_delta(const double u[6], double q[4], double t[3]) {
    double s = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (s <= 1.0) {
        q[0] = sqrt(1.0 - s); q[1] = u[0]; q[2] = u[1]; q[3] = u[2];
    } else {
        double n = sqrt(s);
        q[0] = 0.0; q[1] = u[0] / n; q[2] = u[1] / n; q[3] = u[2] / n;
    }
    t[0] = u[3]; t[1] = u[4]; t[2] = u[5];
}

/* MovePST (Alg. 1; Sec. 3.3 "PST move": not a vector addition in SE(3)).   */
/* Reading: the PST lives in the chart at the current centre c and a chart  */
/* point u denotes the pose c * Delta(u) (right composition, i.e. a motion  */
/* expressed in the centre camera's own frame).                            */
/* c * Delta(u): q = q_c (x) q_D, t = R(q_c) t_D + t_c.  The centre update */
/* renormalises q and keeps w >= 0.                                         */
void orc_pose_retract(const double qc[4], const double tc[3], const double u[6], double qo[4], double to[3]) {
    double qd[4], td[3], Rc[9], rt[3], q[4];
    orc_chart_delta(u, qd, td);
    orc_quat_mul(qc, qd, q);
    orc_quat_to_rot(qc, Rc);
    rot_apply(Rc, td, rt);
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double sg = (q[0] < 0.0) ? -1.0 : 1.0;
    for (int i = 0; i < 4; ++i) qo[i] = sg * q[i] / n;
    for (int i = 0; i < 3; ++i) to[i] = rt[i] + tc[i];
}

/* Pose of particle i (Alg. 1 MovePST + RescalePST applied to the stored    */
/* unit template, Sec. 4 "GPU implementation"): u = r (.) p_i, pose =       */
/* c * Delta(u).  Rotation matrix R(q_c (x) q_D) (product not renormalised),*/
/* translation R(q_c) t_D + t_c.  Output as a 3x4 row-major [R|t].          */
void orc_particle_pose(const double qc[4], const double tc[3], const double r[6], const float p[6], double T[12]) {
    double u[6], qd[4], td[3], q[4], R[9], Rc[9], rt[3];
    for (int d = 0; d < 6; ++d) u[d] = r[d] * (double)p[d];
    orc_chart_delta(u, qd, td);
    orc_quat_mul(qc, qd, q);
    orc_quat_to_rot(q, R);
    orc_quat_to_rot(qc, Rc);
    rot_apply(Rc, td, rt);
    for (int i = 0; i < 3; ++i) {
        T[4 * i + 0] = R[3 * i + 0];
        T[4 * i + 1] = R[3 * i + 1];
        T[4 * i + 2] = R[3 * i + 2];
        T[4 * i + 3] = rt[i] + tc[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Depth unprojection (Eq. unproj) on a stride-s pixel grid (Sec. 4,        */
/* "stride-based downsampling").  Point index j follows row-major order of  */
/* the sampled pixels (v = 0, s, 2s..; u = 0, s, 2s..).  z <= 0 (or not a   */
/* number) is "no measurement" and yields no point.                         */
/*   F64: x = (u - cx) z / fx, y = (v - cy) z / fy, in binary64, rounded to */
/*        binary32 for storage.                                             */
/*   F32: x = (((float)u - cx) * z) / fx, same for y, binary32.             */
/* Returns the point count M; pts receives M*3 floats.                      */
/* ------------------------------------------------------------------------ */
int orc_unproject(const float* depth, int32_t W, int32_t H, float fx, float fy, float cx, float cy,
                  int32_t stride, int prec, float* pts) {
    int m = 0;
    for (int32_t v = 0; v < H; v += stride) {
        for (int32_t u = 0; u < W; u += stride) {
            float z = depth[(size_t)v * W + u];
            if (!(z > 0.0f)) continue;
            if (prec == ORC_F32) {
                pts[3 * m + 0] = (((float)u - cx) * z) / fx;
                pts[3 * m + 1] = (((float)v - cy) * z) / fy;
            } else {
                pts[3 * m + 0] = (float)(((double)u - (double)cx) * (double)z / (double)fx);
                pts[3 * m + 1] = (float)(((double)v - (double)cy) * (double)z / (double)fy);
            }
            pts[3 * m + 2] = z;
            ++m;
        }
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Rigid transform of a camera point by a 3x4 binary64 transform A.         */
/*   F64: binary64 A x + a.                                                 */
/*   F32: A is rounded once to binary32 (A32), then for each output row c:  */
/*        fmaf(A32[c][2], z, fmaf(A32[c][1], y, fmaf(A32[c][0], x, a32[c]))) */
/* ------------------------------------------------------------------------ */
static void xform_point(const double A[12], const float* A32, const float x[3], int prec, double o[3]) {
    if (prec == ORC_F32) {
        for (int c = 0; c < 3; ++c) {
            float acc = fmaf(A32[4 * c + 0], x[0], A32[4 * c + 3]);
            acc = fmaf(A32[4 * c + 1], x[1], acc);
            acc = fmaf(A32[4 * c + 2], x[2], acc);
            o[c] = (double)acc;
        }
    } else {
        for (int c = 0; c < 3; ++c)
            o[c] = A[4 * c + 0] * x[0] + A[4 * c + 1] * x[1] + A[4 * c + 2] * x[2] + A[4 * c + 3];
    }
}

static void round_xform(const double A[12], float A32[12]) {
    for (int i = 0; i < 12; ++i) A32[i] = (float)A[i];
}

/* inverse of a rigid 3x4 [R|t]: [R^T | -R^T t] */
void orc_rigid_inverse(const double T[12], double Ti[12]) {
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Ti[4 * i + j] = T[4 * j + i];
        Ti[4 * i + 3] = -(T[0 * 4 + i] * T[3] + T[1 * 4 + i] * T[7] + T[2 * 4 + i] * T[11]);
    }
}

/* C = A B for 3x4 rigid transforms */
void orc_rigid_mul(const double A[12], const double B[12], double C[12]) {
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = A[4 * i + 0] * B[0 * 4 + j] + A[4 * i + 1] * B[1 * 4 + j] + A[4 * i + 2] * B[2 * 4 + j];
            if (j == 3) s += A[4 * i + 3];
            C[4 * i + j] = s;
        }
    }
}

void orc_pose_to_mat(const double q[4], const double t[3], double T[12]) {
    double R[9];
    orc_quat_to_rot(q, R);
    for (int i = 0; i < 3; ++i) {
        T[4 * i + 0] = R[3 * i + 0]; T[4 * i + 1] = R[3 * i + 1]; T[4 * i + 2] = R[3 * i + 2];
        T[4 * i + 3] = t[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Overlap set O_k (Eq. validness, Sec. 4): a point x of the current frame  */
/* is kept iff, moved by the current centre pose T_c into the world and     */
/* back into frame t-1 by T_prev^-1, it lies in front of that camera        */
/* (z' > 0) and projects inside the image: 0 <= fx x'/z' + cx <= W-1 and    */
/* 0 <= fy y'/z' + cy <= H-1 (continuous pixel coordinates).                */
/*   F32: A = T_prev^-1 T_c in binary64, rounded once; x' by xform_point;    */
/*        px = fmaf(fx, x' / z', cx), py = fmaf(fy, y' / z', cy).           */
/* Optional stricter reading of "in the previous depth image" (prev_depth  */
/* non-NULL, the H x W depth frame t-1): the pixel nearest to (px, py),    */
/* u = floor(px + 1/2), v = floor(py + 1/2) (in binary32 for F32), must     */
/* also hold a valid depth (> 0).                                          */
/* Writes mask[j] in {0,1}; returns |O_k|.                                   */
/* ------------------------------------------------------------------------ */
int orc_overlap(const float* pts, int32_t m, const double Tc[12], const double Tprev[12],
                float fx, float fy, float cx, float cy, int32_t W, int32_t H, const float* prev_depth, int prec,
                uint8_t* mask) {
    double Ti[12], A[12];
    float A32[12];
    orc_rigid_inverse(Tprev, Ti);
    orc_rigid_mul(Ti, Tc, A);
    round_xform(A, A32);
    int n = 0;
    for (int32_t j = 0; j < m; ++j) {
        double o[3];
        xform_point(A, A32, pts + 3 * (size_t)j, prec, o);
        int keep;
        if (prec == ORC_F32) {
            float xp = (float)o[0], yp = (float)o[1], zp = (float)o[2];
            if (!(zp > 0.0f)) { keep = 0; }
            else {
                float px = fmaf(fx, xp / zp, cx);
                float py = fmaf(fy, yp / zp, cy);
                keep = (px >= 0.0f && px <= (float)(W - 1) && py >= 0.0f && py <= (float)(H - 1));
                if (keep && prev_depth) {
                    const int32_t u = (int32_t)floorf(px + 0.5f), v = (int32_t)floorf(py + 0.5f);
                    keep = prev_depth[(size_t)v * W + u] > 0.0f;
                }
            }
        } else {
            if (!(o[2] > 0.0)) { keep = 0; }
            else {
                double px = fx * (o[0] / o[2]) + cx;
                double py = fy * (o[1] / o[2]) + cy;
                keep = (px >= 0.0 && px <= (double)(W - 1) && py >= 0.0 && py <= (double)(H - 1));
                if (keep && prev_depth) {
                    const int32_t u = (int32_t)floor(px + 0.5), v = (int32_t)floor(py + 0.5);
                    keep = prev_depth[(size_t)v * W + u] > 0.0f;
                }
            }
        }
        mask[j] = (uint8_t)keep;
        n += keep;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* TSDF lookup.  psi is the normalised TSDF (value / truncation, in [-1,1]),*/
/* stored linearly as psi[(k*ny + j)*nx + i]; voxel (i,j,k) covers          */
/* origin + [i, i+1) * vox along each axis, centre at (i + 1/2) * vox.      */
/* Unobserved voxels hold +1; a query outside the grid reads +1 (a penalty, */
/* never an exclusion).                                                     */
/*   voxel coordinate g = (X - origin) / vox.                               */
/*   NEAREST: the voxel containing X, i.e. floor(g).                        */
/*   TRILINEAR: interpolation between the 8 voxel centres around X,         */
/*   h = g - 1/2, i0 = floor(h); if any of the 8 corners is outside the     */
/*   grid the value is +1.                                                  */
/* In F32 mode g is computed by one binary32 transform (xform_point) whose  */
/* matrix is [R/vox | (t - origin)/vox] folded in binary64 and rounded once;*/
/* h = g - 0.5f in binary32; interpolation weights f = h - i0 in binary32.  */
/* The interpolation itself and the squares are summed in binary64.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float* psi;
    int32_t nx, ny, nz;
    double vox;
    double origin[3];
} orc_grid;

static double grid_at(const orc_grid* g, int64_t i, int64_t j, int64_t k) {
    return (double)g->psi[((size_t)k * g->ny + (size_t)j) * g->nx + (size_t)i];
}

static double lookup(const orc_grid* g, const double gv[3], int lk) {
    const int32_t n[3] = {g->nx, g->ny, g->nz};
    if (lk == ORC_LOOKUP_NEAREST) {
        int64_t id[3];
        for (int c = 0; c < 3; ++c) {
            if (!(gv[c] >= 0.0 && gv[c] < (double)n[c])) return 1.0;
            id[c] = (int64_t)floor(gv[c]);
            if (id[c] >= n[c]) return 1.0;
        }
        return grid_at(g, id[0], id[1], id[2]);
    }
    /* trilinear */
    int64_t i0[3];
    double f[3];
    for (int c = 0; c < 3; ++c) {
        double h = gv[c];
        if (!(h >= 0.0 && h < (double)(n[c] - 1))) return 1.0;
        i0[c] = (int64_t)floor(h);
        if (i0[c] + 1 >= n[c]) return 1.0;
        f[c] = h - (double)i0[c];
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                acc += w * grid_at(g, i0[0] + dx, i0[1] + dy, i0[2] + dz);
            }
    return acc;
}

/* voxel-space coordinate of a camera point under pose T (3x4, binary64) */
static void voxel_coord(const orc_grid* g, const double T[12], const float* V32, const float x[3], int prec,
                        int lk, double gv[3]) {
    if (prec == ORC_F32) {
        double o[3];
        xform_point(T /*unused in F32*/, V32, x, ORC_F32, o);
        for (int c = 0; c < 3; ++c) {
            float gc = (float)o[c];
            if (lk == ORC_LOOKUP_TRILINEAR) {
                float h = gc - 0.5f;
                float fl = floorf(h);
                /* store integer part and binary32 fraction exactly: i0 + f */
                float fr = h - fl;
                gv[c] = (double)fl + (double)fr; /* exact: both parts fit in binary64 */
                /* keep the binary32 fraction as the weight (see lookup) */
            } else {
                gv[c] = (double)gc;
            }
        }
    } else {
        double X[3];
        for (int c = 0; c < 3; ++c)
            X[c] = T[4 * c + 0] * x[0] + T[4 * c + 1] * x[1] + T[4 * c + 2] * x[2] + T[4 * c + 3];
        for (int c = 0; c < 3; ++c) {
            gv[c] = (X[c] - g->origin[c]) / g->vox;
            if (lk == ORC_LOOKUP_TRILINEAR) gv[c] -= 0.5;
        }
    }
}

/* fold the voxel scaling into a camera->world transform (binary64), then    */
/* round once to binary32: V = [R / vox | (t - origin) / vox]               */
static void fold_voxel(const orc_grid* g, const double T[12], float V32[12]) {
    double inv = 1.0 / g->vox;
    for (int c = 0; c < 3; ++c) {
        for (int j = 0; j < 3; ++j) V32[4 * c + j] = (float)(T[4 * c + j] * inv);
        V32[4 * c + 3] = (float)((T[4 * c + 3] - g->origin[c]) * inv);
    }
}

/* ------------------------------------------------------------------------ */
/* Fitness (Eq. ourlh with the overlap normalisation of Eq. normallh):      */
/*   S_i = sum_{j in O} psi(T_i x_j)^2, F_i = S_i / |O|  (|O| > 0),          */
/*   rho_i = exp(-F_i / tau).  |O| = 0 gives F_i = 1.                        */
/* T: n transforms, 3x4 row-major camera->world, binary64.                   */
/* The sum follows Sec. 4 "GPU implementation" (sums of many floating-point */
/* numbers taken with compensation, Kahan summation):                       */
/*  ORC_F64: binary64 with Neumaier compensation (Kahan-Babuska-Neumaier);  */
/*  ORC_F32: exact on a 2^-39 grid -- every term v^2 (exact in binary64 for */
/*           a binary32 v) rounded to the nearest multiple of 2^-39 (ties   */
/*           to even), the integers added exactly (below 2^63 for up to     */
/*           2^24 terms), S = (their sum) 2^-39 rounded once to binary64.   */
/*           The result does not depend on the order of the terms; its      */
/*           error is at most m 2^-40 absolute.                              */
/* mask may be NULL (all points).  normalize=0 returns S_i instead of F_i.   */
/* ------------------------------------------------------------------------ */
static void neumaier_add(double* s, double* c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

/* v^2 on the 2^-39 grid: nearest integer (ties to even) to v^2 2^39 */
static uint64_t grid_term(double v) { return (uint64_t)nearbyint(ldexp(v * v, 39)); }

/* plain32 != 0 ("No Kahan" of the Sec. 5 TSDF-normalisation ablation): the  */
/* sum is taken directly in binary32 in point order, acc = fmaf(v, v, acc)  */
/* with v rounded to binary32, i.e. one rounding per added term and no      */
/* compensation; S = acc.                                                   */
typedef struct {
    const orc_grid* g;
    const float* pts;
    int32_t m;
    const uint8_t* mask;
    const double* T;
    int32_t lk, prec, normalize, plain32, cnt;
    double* F;
} orc_fitness_job;

/* particles [i0, i1) of one orc_fitness_ex call */
static void fitness_range(void* arg, int64_t i0, int64_t i1) {
    const orc_fitness_job* a = (const orc_fitness_job*)arg;
    for (int64_t i = i0; i < i1; ++i) {
        const double* Ti = a->T + 12 * (size_t)i;
        float V32[12];
        fold_voxel(a->g, Ti, V32);
        double s = 0.0, c = 0.0;
        float acc = 0.0f;
        uint64_t q = 0;
        for (int32_t j = 0; j < a->m; ++j) {
            if (a->mask != NULL && !a->mask[j]) continue;
            double gv[3];
            voxel_coord(a->g, Ti, V32, a->pts + 3 * (size_t)j, a->prec, a->lk, gv);
            double v;
            if (a->lk == ORC_LOOKUP_TRILINEAR) {
                /* gv already holds h = g - 1/2; lookup() treats it as h */
                v = lookup(a->g, gv, ORC_LOOKUP_TRILINEAR);
            } else {
                v = lookup(a->g, gv, ORC_LOOKUP_NEAREST);
            }
            if (a->plain32) {
                const float vf = (float)v;
                acc = fmaf(vf, vf, acc);
            } else if (a->prec == ORC_F32) {
                q += grid_term(v);
            } else {
                neumaier_add(&s, &c, v * v);
            }
        }
        double S = a->plain32 ? (double)acc : (a->prec == ORC_F32 ? ldexp((double)q, -39) : s + c);
        if (!a->normalize) a->F[i] = S;
        else a->F[i] = (a->cnt > 0) ? S / (double)a->cnt : 1.0;
    }
}

void orc_fitness_ex(const float* psi, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                    const float* pts, int32_t m, const uint8_t* mask, const double* T, int32_t n, int32_t lk,
                    int prec, int normalize, int plain32, double* F) {
    orc_grid g = {psi, nx, ny, nz, (double)vox, {origin[0], origin[1], origin[2]}};
    int32_t cnt = 0;
    for (int32_t j = 0; j < m; ++j) cnt += (mask == NULL || mask[j]);
    orc_fitness_job job = {&g, pts, m, mask, T, lk, prec, normalize, plain32, cnt, F};
    orc_parallel_ranges(fitness_range, &job, (int64_t)(n > 0 ? n : 0));
}

void orc_fitness(const float* psi, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                 const float* pts, int32_t m, const uint8_t* mask, const double* T, int32_t n, int32_t lk,
                 int prec, int normalize, double* F) {
    orc_fitness_ex(psi, nx, ny, nz, vox, origin, pts, m, mask, T, n, lk, prec, normalize, 0, F);
}

/* Voxel indices of each (particle, point) pair under NEAREST lookup, for   */
/* bit-exact index checks: idx[i*m + j] = linear voxel index (k*ny+j)*nx+i, */
/* or -1 when outside the grid.  F32 mode only (the kernel's precision).    */
void orc_voxel_indices(int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3], const float* pts,
                       int32_t m, const double* T, int32_t n, int64_t* idx) {
    orc_grid g = {NULL, nx, ny, nz, (double)vox, {origin[0], origin[1], origin[2]}};
    const int32_t dims[3] = {nx, ny, nz};
    for (int32_t i = 0; i < n; ++i) {
        float V32[12];
        fold_voxel(&g, T + 12 * (size_t)i, V32);
        for (int32_t j = 0; j < m; ++j) {
            double o[3];
            xform_point(NULL, V32, pts + 3 * (size_t)j, ORC_F32, o);
            int64_t id[3];
            int inside = 1;
            for (int c = 0; c < 3; ++c) {
                float gc = (float)o[c];
                if (!(gc >= 0.0f && gc < (float)dims[c])) { inside = 0; break; }
                id[c] = (int64_t)floorf(gc);
                if (id[c] >= dims[c]) { inside = 0; break; }
            }
            idx[(size_t)i * m + j] = inside ? ((id[2] * ny + id[1]) * nx + id[0]) : -1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* PST update of one iteration (the steps of Alg. 1 after the APS loop):  */
/*  rho_prev = rho(s*_{k-1}), the APS threshold, given by the caller.       */
/*  APS = { i : rho_i > rho_prev }, rho_i = exp(-F_i / tau) in binary64.    */
/*  Non-empty APS (Eqs. ebs, wafit, rsdir, rsinter):                        */
/*     w_i = rho_i - rho_prev, W = sum w_i;                                 */
/*     u* = sum w_i u_i / W  (u_i = r (.) p_i, chart of c_{k-1});            */
/*     rho~ = sum w_i rho_i / W;  v = u* - 0 = u*;                           */
/*     rhat_d = (1 - rho~) |v_d| / ||v|| + eps   (||v|| = 0: 1/sqrt6 per d); */
/*     c_k = c_{k-1} * Delta(u*).                                           */
/*  Empty APS (Sec. 4 "PST update", second corner case):                    */
/*     rhat = 2 (1 - rho_prev) 1/||1||; c unchanged.                         */
/*  TSDF not built (first corner case): rhat = 0.5 * 1, c unchanged.        */
/*  Momentum (Eq. momentum): r_k = beta r_{k-1} + (1 - beta) rhat.          */
/*  Rescaling ablation (Sec. 5 ablation of Eq. rsinter, flags):             */
/*     ORC_ISO_ONLY:   the attractor direction |v|/||v|| is replaced by the */
/*                     isotropic unit vector 1/sqrt6: rhat = (1-rho~)/sqrt6 */
/*                     + eps;                                               */
/*     ORC_ANISO_ONLY: the isotropic factor (1 - rho~) is dropped:          */
/*                     rhat = |v|/||v|| + eps.                              */
/*  Both concern the non-empty branch only.                                 */
/* Sums in binary64 with Neumaier compensation.                              */
/* Returns the APS size; outputs r_out, q_out/t_out (new centre), rho~      */
/* (rho_prev when the APS is empty) and u* (zeros when empty).              */
/* ------------------------------------------------------------------------ */
int orc_pst_update(const double* F, const float* pst, int32_t n, const double r_in[6], const double qc[4],
                   const double tc[3], double tau, double beta, double eps, int32_t tsdf_built, double rho_thr,
                   double r_out[6], double q_out[4], double t_out[3], double* rho_tilde, double u_star[6],
                   int32_t flags) {
    const double inv_sqrt6 = 1.0 / sqrt(6.0);
    double rhat[6];
    int aps = 0;
    for (int d = 0; d < 6; ++d) u_star[d] = 0.0;
    memcpy(q_out, qc, 4 * sizeof(double));
    memcpy(t_out, tc, 3 * sizeof(double));
    if (!tsdf_built) {
        for (int d = 0; d < 6; ++d) rhat[d] = 0.5;
        *rho_tilde = 0.5;
    } else {
        double rho_prev = rho_thr;
        double sw = 0, cw = 0, sr = 0, cr = 0, su[6] = {0}, cu[6] = {0};
        for (int32_t i = 0; i < n; ++i) {
            double rho = orc_exp(-F[i] / tau);
            if (!(rho > rho_prev)) continue;
            ++aps;
            double w = rho - rho_prev;
            neumaier_add(&sw, &cw, w);
            neumaier_add(&sr, &cr, w * rho);
            for (int d = 0; d < 6; ++d) neumaier_add(&su[d], &cu[d], w * (r_in[d] * (double)pst[6 * (size_t)i + d]));
        }
        if (aps > 0) {
            double W = sw + cw;
            double nv = 0.0;
            for (int d = 0; d < 6; ++d) {
                u_star[d] = (su[d] + cu[d]) / W;
                nv += u_star[d] * u_star[d];
            }
            nv = sqrt(nv);
            double rt = (sr + cr) / W;
            *rho_tilde = rt;
            const double iso = (flags & ORC_ANISO_ONLY) ? 1.0 : (1.0 - rt);
            for (int d = 0; d < 6; ++d) {
                const double dir = (nv > 0.0 && !(flags & ORC_ISO_ONLY)) ? fabs(u_star[d]) / nv : inv_sqrt6;
                rhat[d] = iso * dir + eps;
            }
            orc_pose_retract(qc, tc, u_star, q_out, t_out);
        } else {
            *rho_tilde = rho_prev;
            for (int d = 0; d < 6; ++d) rhat[d] = 2.0 * (1.0 - rho_prev) * inv_sqrt6;
        }
    }
    for (int d = 0; d < 6; ++d) r_out[d] = beta * r_in[d] + (1.0 - beta) * rhat[d];
    return aps;
}

/* ------------------------------------------------------------------------ */
/* One frame of Alg. 1 (PFO with PST), plain host loop.                      */
/* Inputs: normalised TSDF psi (linear), depth of frame t (HxW, metres),    */
/* optionally the depth of frame t-1 (prev_depth, NULL: the overlap test is */
/* image bounds only; see orc_overlap), intrinsics, stride, PST template    */
/* (n x 6, row 0 = origin), previous final                                  */
/* pose s^{t-1}_* (q_prev, t_prev), PST initialisation c_0 (q_init, t_init) */
/* and r_0 (r_init) (Sec. 4 "PST initialization": c_0 = s^{t-1}_*,          */
/* r_0 = r_1^{t-1}).                                                         */
/* Loop k = 1..max_iters: overlap O_k with c_{k-1} (Eq. validness), fitness */
/* of all particles (Eq. normallh), PST update (orc_pst_update).            */
/* Stop (Sec. 4 "Convergence criteria", when early_stop != 0): the APS is   */
/* empty in two consecutive iterations, or every |u*_d| < stop_tol.          */
/* In F32 mode, F_i is rounded to binary32 before the APS decision (the     */
/* kernel stores F in binary32).                                             */
/* Outputs: final centre (pose of frame t), r_1 (axis lengths after the     */
/* first iteration, carried to frame t+1), rho~ of the last non-empty       */
/* iteration (rho_prev if none), iteration count, per-iteration APS sizes   */
/* and rho~, point count, last overlap count; optional (NULL: not written)  */
/* per-iteration |O_k|, the centre's exact fitness exp(-F_0/tau) and the    */
/* APS threshold used.                                                      */
/* Returns 0, or -4 when the frame has no valid point.                      */
/*                                                                          */
/* Multi-resolution PST (Sec. 4 "Multi-resolution PST"; levels >= 2): the  */
/* paper alternates a few (PST size, depth subsampling) pairs across the   */
/* iterations.  Iteration k uses level (k - 1) mod levels: the particles    */
/* are the first level_n[l] rows of the template (an i.i.d. template's     */
/* prefix is itself a uniform template) and the points are the frame       */
/* subsampled with stride level_stride[l].  Everything else (centre, axis  */
/* lengths, APS threshold, stop rules) carries across levels unchanged.    */
/* A level with no valid sample has F = 1 for every particle; -4 only when */
/* no level has a valid sample.  levels <= 1: one level (n, stride).       */
/* ------------------------------------------------------------------------ */
#define ORC_MAX_LEVELS 4
typedef struct {
    int32_t max_iters, early_stop, stride, lookup, flags, prec;
    int32_t levels, level_n[ORC_MAX_LEVELS], level_stride[ORC_MAX_LEVELS];
    double beta, eps, tau, stop_tol;
} orc_track_params;

int orc_track_frame(const float* psi, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                    const float* depth, const float* prev_depth, int32_t W, int32_t H, float fx, float fy,
                    float cx, float cy, const float* pst, int32_t n, const double q_prev[4],
                    const double t_prev[3], const double q_init[4], const double t_init[3],
                    const double r_init[6], int32_t tsdf_built,
                    const orc_track_params* P, double q_out[4], double t_out[3], double r1_out[6],
                    double* rho_out, int32_t* iters_out, int32_t* aps_sizes, double* rho_iter,
                    int32_t* n_points_out, int32_t* n_overlap_last, int32_t* n_overlap_iter,
                    double* rho_centre_iter, double* thr_iter) {
    const int32_t L = (P->levels > 1) ? P->levels : 1;
    if (L > ORC_MAX_LEVELS) return -1;
    int32_t lv_n[ORC_MAX_LEVELS], lv_m[ORC_MAX_LEVELS];
    float* lv_pts[ORC_MAX_LEVELS];
    int32_t m_all = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t st = (L > 1) ? P->level_stride[l] : P->stride;
        lv_n[l] = (L > 1) ? P->level_n[l] : n;
        if (st < 1 || lv_n[l] < 1 || lv_n[l] > n) {
            for (int32_t e = 0; e < l; ++e) free(lv_pts[e]);
            return -1;
        }
        const int32_t cap = ((H + st - 1) / st) * ((W + st - 1) / st);
        lv_pts[l] = (float*)malloc(sizeof(float) * 3 * (size_t)(cap > 0 ? cap : 1));
        lv_m[l] = orc_unproject(depth, W, H, fx, fy, cx, cy, st, P->prec, lv_pts[l]);
        if (lv_m[l] > m_all) m_all = lv_m[l];
    }
    uint8_t* mask = (uint8_t*)malloc((size_t)(m_all > 0 ? m_all : 1));
    double* T = (double*)malloc(sizeof(double) * 12 * (size_t)n);
    double* F = (double*)malloc(sizeof(double) * (size_t)n);
    const float* pts = lv_pts[0];
    int32_t m = lv_m[0];
    *n_points_out = m;
    memcpy(r1_out, r_init, 6 * sizeof(double));
    double qc[4], tc[3], r[6], Tprev[12];
    memcpy(qc, q_init, sizeof qc);
    memcpy(tc, t_init, sizeof tc);
    memcpy(r, r_init, sizeof r);
    orc_pose_to_mat(q_prev, t_prev, Tprev);
    int rc = 0;
    int32_t k = 0, empty_streak = 0, nO = 0;
    double thr = 0.0;
    double rho_last = 0.5;
    int have_rho = 0;
    if (m_all == 0 && tsdf_built) {
        rc = -4;
        goto done;
    }
    for (k = 1; k <= P->max_iters; ++k) {
        double r_new[6], q_new[4], t_new[3], rt, us[6];
        pts = lv_pts[(k - 1) % L];
        m = lv_m[(k - 1) % L];
        n = lv_n[(k - 1) % L];
        if (tsdf_built) {
            double Tc[12];
            orc_pose_to_mat(qc, tc, Tc);
            if (P->flags & ORC_NO_OVERLAP) {
                for (int32_t j = 0; j < m; ++j) mask[j] = 1;
                nO = m;
            } else {
                nO = orc_overlap(pts, m, Tc, Tprev, fx, fy, cx, cy, W, H, prev_depth, P->prec, mask);
            }
            for (int32_t i = 0; i < n; ++i) orc_particle_pose(qc, tc, r, pst + 6 * (size_t)i, T + 12 * (size_t)i);
            orc_fitness_ex(psi, nx, ny, nz, vox, origin, pts, m, mask, T, n, P->lookup, P->prec,
                           !(P->flags & ORC_NO_NORMALIZE), (P->flags & ORC_NO_KAHAN) != 0, F);
            if (P->prec == ORC_F32)
                for (int32_t i = 0; i < n; ++i) F[i] = (double)(float)F[i];
        }
        /* APS threshold rho(s*_{k-1}).  Sec. 4 never evaluates the fitness of  */
        /* a best state: it stands in the weighted APS average of Eq. wafit.   */
        /* So from k = 2 on the threshold is that average, carried from the    */
        /* last non-empty iteration; at k = 1 (s*_0 = c_0, no average yet) it  */
        /* is the centre's own fitness (template row 0 sits at c_0).           */
        /* ORC_CENTRE_THRESHOLD: the centre's exact fitness at every k.        */
        double centre = tsdf_built ? orc_exp(-F[0] / P->tau) : 0.5;
        double thr_k = (k == 1 || (P->flags & ORC_CENTRE_THRESHOLD)) ? centre : thr;
        int aps = orc_pst_update(F, pst, n, r, qc, tc, P->tau, P->beta, P->eps, tsdf_built, thr_k, r_new, q_new,
                                 t_new, &rt, us, P->flags);
        thr = (aps > 0) ? rt : thr_k;
        if (k - 1 < 32) {
            aps_sizes[k - 1] = aps;
            rho_iter[k - 1] = rt;
            if (n_overlap_iter) n_overlap_iter[k - 1] = tsdf_built ? nO : 0;
            if (rho_centre_iter) rho_centre_iter[k - 1] = centre;
            if (thr_iter) thr_iter[k - 1] = thr_k;
        }
        memcpy(r, r_new, sizeof r);
        memcpy(qc, q_new, sizeof qc);
        memcpy(tc, t_new, sizeof tc);
        if (k == 1) memcpy(r1_out, r, sizeof r);
        if (!tsdf_built) { rho_last = 0.5; have_rho = 1; break; }
        if (aps > 0) {
            rho_last = rt; have_rho = 1;
            empty_streak = 0;
            if (P->early_stop) {
                int small = 1;
                for (int d = 0; d < 6; ++d) small &= (fabs(us[d]) < P->stop_tol);
                if (small) break;
            }
        } else {
            if (!have_rho) rho_last = rt;
            ++empty_streak;
            if (P->early_stop && empty_streak >= 2) break;
        }
    }
    if (k > P->max_iters) k = P->max_iters;
done:
    memcpy(q_out, qc, sizeof qc);
    memcpy(t_out, tc, sizeof tc);
    *rho_out = rho_last;
    *iters_out = (rc == 0) ? k : 0;
    *n_overlap_last = nO;
    for (int32_t l = 0; l < L; ++l) free(lv_pts[l]);
    free(mask); free(T); free(F);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Volumetric depth fusion (Curless-Levoy / KinectFusion framework that     */
/* Sec. 3 builds on; the paper gives no formula -- projective running       */
/* average, the reading stated in the design notes).  For every voxel with */
/* centre X = origin + (i + 1/2) vox:                                        */
/*   x_c = T^-1 X (camera frame); skip if z_c <= 0;                          */
/*   pixel u = floor(fx x_c / z_c + cx + 1/2), v likewise (nearest pixel);  */
/*   skip if outside the image or D(u,v) <= 0;                              */
/*   sdf = D(u,v) - z_c; skip if sdf < -mu;                                 */
/*   d = min(1, sdf / mu);                                                   */
/*   psi <- (W psi + d) / (W + 1);  W <- min(W + 1, w_max).                  */
/* psi and W are linear [k][j][i] arrays (binary32 storage).                */
/*   F32: A = [R^T vox | R^T (origin + vox/2 - t)] folded in binary64 and  */
/*        rounded once; x_c = xform_point(A, (i, j, k)); u = floor(fmaf(fx, */
/*        x_c / z_c, cx) + 0.5f); sdf = D - z_c; d = fminf(1, sdf / mu);     */
/*        psi' = fmaf(W, psi, d) / (W + 1) -- all binary32.                  */
/*   F64: the same in binary64, stored rounded to binary32.                 */
/* Returns the number of voxels updated.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    float *psi, *wgt;
    int32_t nx, ny, nz;
    float vox, mu, w_max;
    const float* origin;
    const float* depth;
    int32_t W, H;
    float fx, fy, cx, cy;
    const double* R;
    const double* t;
    const float* A32;
    int prec;
    int64_t* updated; /* per z-slice */
} orc_integrate_job;

/* z-slices [k0, k1) of one orc_integrate call */
static void integrate_range(void* arg, int64_t k0, int64_t k1) {
    const orc_integrate_job* a = (const orc_integrate_job*)arg;
    const int32_t nx = a->nx, ny = a->ny, W = a->W, H = a->H;
    const float fx = a->fx, fy = a->fy, cx = a->cx, cy = a->cy, mu = a->mu;
    const double vx = (double)a->vox;
    for (int64_t k = k0; k < k1; ++k) {
        int64_t updated = 0;
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                size_t id = ((size_t)k * ny + j) * nx + i;
                if (a->prec == ORC_F32) {
                    float vi[3] = {(float)i, (float)j, (float)k};
                    double o[3];
                    xform_point(NULL, a->A32, vi, ORC_F32, o);
                    float xc = (float)o[0], yc = (float)o[1], zc = (float)o[2];
                    if (!(zc > 0.0f)) continue;
                    float pu = floorf(fmaf(fx, xc / zc, cx) + 0.5f);
                    float pv = floorf(fmaf(fy, yc / zc, cy) + 0.5f);
                    if (!(pu >= 0.0f && pu < (float)W && pv >= 0.0f && pv < (float)H)) continue;
                    float D = a->depth[(size_t)pv * W + (size_t)pu];
                    if (!(D > 0.0f)) continue;
                    float sdf = D - zc;
                    if (sdf < -mu) continue;
                    float d = fminf(1.0f, sdf / mu);
                    float w0 = a->wgt[id];
                    a->psi[id] = fmaf(w0, a->psi[id], d) / (w0 + 1.0f);
                    a->wgt[id] = fminf(w0 + 1.0f, a->w_max);
                } else {
                    double X[3] = {a->origin[0] + (i + 0.5) * vx, a->origin[1] + (j + 0.5) * vx,
                                   a->origin[2] + (k + 0.5) * vx};
                    double xc[3];
                    for (int r = 0; r < 3; ++r) {
                        double s = 0.0;
                        for (int c = 0; c < 3; ++c) s += a->R[3 * c + r] * (X[c] - a->t[c]);
                        xc[r] = s;
                    }
                    if (!(xc[2] > 0.0)) continue;
                    double pu = floor(fx * (xc[0] / xc[2]) + cx + 0.5);
                    double pv = floor(fy * (xc[1] / xc[2]) + cy + 0.5);
                    if (!(pu >= 0.0 && pu < (double)W && pv >= 0.0 && pv < (double)H)) continue;
                    double D = a->depth[(size_t)pv * W + (size_t)pu];
                    if (!(D > 0.0)) continue;
                    double sdf = D - xc[2];
                    if (sdf < -(double)mu) continue;
                    double d = fmin(1.0, sdf / (double)mu);
                    double w0 = a->wgt[id];
                    a->psi[id] = (float)((w0 * (double)a->psi[id] + d) / (w0 + 1.0));
                    a->wgt[id] = (float)fmin(w0 + 1.0, (double)a->w_max);
                }
                ++updated;
            }
        a->updated[k] = updated;
    }
}

int64_t orc_integrate(float* psi, float* wgt, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                      float mu, float w_max, const float* depth, int32_t W, int32_t H, float fx, float fy, float cx,
                      float cy, const double q[4], const double t[3], int prec) {
    double R[9];
    orc_quat_to_rot(q, R);
    double A[12];
    float A32[12];
    double vx = (double)vox;
    for (int r = 0; r < 3; ++r) {
        /* row r of R^T is column r of R */
        for (int c = 0; c < 3; ++c) A[4 * r + c] = R[3 * c + r] * vx;
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += R[3 * c + r] * ((double)origin[c] + 0.5 * vx - t[c]);
        A[4 * r + 3] = s;
    }
    round_xform(A, A32);
    int64_t* per_slice = (int64_t*)calloc((size_t)(nz > 0 ? nz : 1), sizeof(int64_t));
    orc_integrate_job job = {psi, wgt, nx, ny, nz, vox, mu, w_max, origin, depth, W, H,
                             fx, fy, cx, cy, R, t, A32, prec, per_slice};
    orc_parallel_ranges(integrate_range, &job, (int64_t)(nz > 0 ? nz : 0));
    int64_t updated = 0;
    for (int32_t k = 0; k < nz; ++k) updated += per_slice[k];
    free(per_slice);
    return updated;
}

/* ------------------------------------------------------------------------ */
/* Low-resolution raycast of the TSDF (the model rendered at a pose; input  */
/* of the learned proposal).  For pixel (u, v) of the given intrinsics the  */
/* ray is x(z) = T (z (u - cx)/fx, z (v - cy)/fy, z), z = z-depth.  It is   */
/* sampled at z_k = near + k * step (k = 0, 1, ..) while z_k <= far, with   */
/* trilinear psi (any corner outside the grid: +1).  The first pair of      */
/* consecutive samples with psi_k > 0 >= psi_{k+1}, both inside the          */
/* truncation band (|psi| < 1), gives the depth by linear interpolation     */
/* z* = z_k + step psi_k / (psi_k - psi_{k+1}); no such pair: 0.            */
/* Binary64 throughout.                                                     */
/* ------------------------------------------------------------------------ */
void orc_raycast(const float* psi, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                 const double q[4], const double t[3], int32_t W, int32_t H, double fx, double fy, double cx,
                 double cy, double near_z, double far_z, double step, float* depth_out) {
    orc_grid g = {psi, nx, ny, nz, (double)vox, {origin[0], origin[1], origin[2]}};
    double R[9];
    orc_quat_to_rot(q, R);
    for (int32_t v = 0; v < H; ++v)
        for (int32_t u = 0; u < W; ++u) {
            double dc[3] = {((double)u - cx) / fx, ((double)v - cy) / fy, 1.0}, dw[3];
            rot_apply(R, dc, dw);
            double prev = 0.0, zprev = 0.0, out = 0.0;
            int have = 0;
            for (int64_t k = 0;; ++k) {
                double z = near_z + (double)k * step;
                if (z > far_z) break;
                double gv[3];
                for (int c = 0; c < 3; ++c) gv[c] = (t[c] + z * dw[c] - g.origin[c]) / g.vox - 0.5;
                double s = lookup(&g, gv, ORC_LOOKUP_TRILINEAR);
                if (have && prev > 0.0 && s <= 0.0 && prev < 1.0 && s > -1.0) {
                    out = zprev + step * prev / (prev - s);
                    break;
                }
                prev = s;
                zprev = z;
                have = 1;
            }
            depth_out[(size_t)v * W + u] = (float)out;
        }
}

/* ------------------------------------------------------------------------ */
/* Comparison optimisers of the Sec. 5 ablation of the optimisation         */
/* strategy: vanilla PFO (particle filter optimisation as in Sec. 3.1,      */
/* without particle swarm guidance) and PSO (particle swarm optimisation,   */
/* no template), on the same fitness (Eq. normallh) and particle count as   */
/* PFO with PST.  The paper names both without parameters; the readings:   */
/*  * State space: the chart at the frame's initial pose c_0 = s^{t-1}_*;   */
/*    particle x in R^6 (binary32) denotes the pose c_0 * Delta(x).          */
/*  * Start: x_i = (float)(r_init_d * p_i,d) from the PST template, i.e.    */
/*    the initial particle set of PFO with PST at axis lengths r_init.       */
/*  * Iteration k = 1..K: O_k is the overlap set (Eq. validness) of the     */
/*    best state so far s*_{k-1} (s*_0 = c_0); F_i is the fitness of         */
/*    c_0 * Delta(x_i) over O_k (rounded to binary32 in F32 mode); the best  */
/*    state is replaced when min_i F_i (lowest index on ties) is strictly    */
/*    below F*.  Then, for k < K, one step of the method.                    */
/*  * Vanilla PFO step (Eqs. proposal, weight, pfolh): after resampling the */
/*    weights are uniform, so the new weight is the likelihood of Eq. pfolh */
/*    with g(s*) the best objective found so far, w_i = exp(-(F_i - F*)/tau);*/
/*    systematic resampling with one offset u_k in [0, 1); Gaussian proposal */
/*    around each resampled particle, Sigma = diag(sigma^2) fixed.           */
/*  * PSO step (inertia-weight PSO with a global best, the empirical study  */
/*    the paper cites for PSO): personal bests, inertia weight linear from   */
/*    w_start (k = 1) to w_end (k = K), acceleration coefficients c1, c2,    */
/*    velocity clamp vmax, velocities starting at 0.                         */
/*  * Output: s^t = c_0 * Delta(x*) (orc_pose_retract), rho = exp(-F* / tau). */
/* Random numbers are inputs: PFO takes K x n x 6 standard normals and K    */
/* offsets, PSO K x n x 12 uniforms (r1 in columns 0-5, r2 in 6-11); the    */
/* draws of step k (after iteration k) are row k - 1.                       */
/* ------------------------------------------------------------------------ */
#define ORC_SWARM_PFO 0
#define ORC_SWARM_PSO 1

/* Systematic resampling of n particles with weights                        */
/* w_i = exp(-(F_i - F_best)/tau): C_i = w_0 + ... + w_i (binary64, in      */
/* index order); the ancestor of slot m is the first i with                 */
/* C_i > ((m + u)/n) C_{n-1} (n - 1 if none).                               */
void orc_pfo_resample(const double* F, int32_t n, double F_best, double tau, double u, int32_t* anc) {
    double* Cs = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        acc += orc_exp(-(F[i] - F_best) / tau);
        Cs[i] = acc;
    }
    int32_t i = 0;
    for (int32_t m = 0; m < n; ++m) {
        const double t = (((double)m + u) / (double)n) * Cs[n - 1];
        while (i < n - 1 && !(Cs[i] > t)) ++i;
        anc[m] = i;
    }
    free(Cs);
}

/* PSO velocity and position step for n particles (x, v, p: n x 6; g: 6;   */
/* R: n x 12 uniforms), binary32 in this order per coordinate d:           */
/*   a = (c1 * r1) * (p - x);  b = (c2 * r2) * (g - x);                    */
/*   v = ((w * v) + a) + b;  v = min(max(v, -vmax), vmax);  x = x + v.      */
void orc_pso_move(float* x, float* v, const float* p, const float* g, const float* R, int32_t n, float w, float c1,
                  float c2, const float vmax[6]) {
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 6; ++d) {
            const size_t e = 6 * (size_t)i + d;
            const float r1 = R[12 * (size_t)i + d], r2 = R[12 * (size_t)i + 6 + d];
            const float t1 = c1 * r1, t2 = c2 * r2;
            const float d1 = p[e] - x[e], d2 = g[d] - x[e];
            const float a = t1 * d1, b = t2 * d2;
            float vv = w * v[e];
            vv = vv + a;
            vv = vv + b;
            vv = fminf(fmaxf(vv, -vmax[d]), vmax[d]);
            v[e] = vv;
            x[e] = x[e] + vv;
        }
    }
}

typedef struct {
    int32_t method, iters, stride, lookup, flags, prec;
    double tau;
    double r_init[6], sigma[6];
    double w_start, w_end, c1, c2;
    double vmax[6];
} orc_swarm_params;

/* One frame of either comparison optimiser.  Returns 0, -1 for bad         */
/* parameters, -4 when the frame has no valid point (pose unchanged).       */
/* Per iteration k (index k - 1): rho_best = exp(-F* / tau) after the         */
/* iteration, rho_mean = mean_i exp(-F_i/tau), best_index = the particle    */
/* that improved F* (-1 if none), n_overlap = |O_k|.                         */
int orc_swarm_frame(const float* psi, int32_t nx, int32_t ny, int32_t nz, float vox, const float origin[3],
                    const float* depth, int32_t W, int32_t H, float fx, float fy, float cx, float cy,
                    const float* pst, int32_t n, const double q_prev[4], const double t_prev[3],
                    const orc_swarm_params* P, const float* draws, const float* offsets, double q_out[4],
                    double t_out[3], double* rho_out, double* rho_best, double* rho_mean, int32_t* best_index,
                    int32_t* n_overlap, int32_t* n_points_out) {
    memcpy(q_out, q_prev, 4 * sizeof(double));
    memcpy(t_out, t_prev, 3 * sizeof(double));
    *n_points_out = 0;
    if (n < 1 || P->iters < 1 || P->iters > 32 || P->stride < 1 ||
        (P->method != ORC_SWARM_PFO && P->method != ORC_SWARM_PSO))
        return -1;
    const int32_t K = P->iters;
    const int32_t cap = ((H + P->stride - 1) / P->stride) * ((W + P->stride - 1) / P->stride);
    float* pts = (float*)malloc(sizeof(float) * 3 * (size_t)(cap > 0 ? cap : 1));
    const int32_t m = orc_unproject(depth, W, H, fx, fy, cx, cy, P->stride, P->prec, pts);
    *n_points_out = m;
    if (m == 0) {
        free(pts);
        return -4;
    }
    uint8_t* mask = (uint8_t*)malloc((size_t)m);
    double* T = (double*)malloc(sizeof(double) * 12 * (size_t)n);
    double* F = (double*)malloc(sizeof(double) * (size_t)n);
    float* x = (float*)malloc(sizeof(float) * 6 * (size_t)n);
    float* xn = (float*)malloc(sizeof(float) * 6 * (size_t)n);
    float* v = (float*)calloc(6 * (size_t)n, sizeof(float));
    float* pb = (float*)malloc(sizeof(float) * 6 * (size_t)n);
    double* pF = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    const double ones[6] = {1, 1, 1, 1, 1, 1};
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 6; ++d) x[6 * (size_t)i + d] = (float)(P->r_init[d] * (double)pst[6 * (size_t)i + d]);
        pF[i] = INFINITY;
    }
    double Tprev[12];
    orc_pose_to_mat(q_prev, t_prev, Tprev);
    double qb[4], tb[3], Fb = INFINITY;
    float xb[6] = {0, 0, 0, 0, 0, 0};
    memcpy(qb, q_prev, sizeof qb);
    memcpy(tb, t_prev, sizeof tb);
    float sig[6], vmx[6];
    for (int d = 0; d < 6; ++d) {
        sig[d] = (float)P->sigma[d];
        vmx[d] = (float)P->vmax[d];
    }
    for (int32_t k = 1; k <= K; ++k) {
        double Tb[12];
        orc_pose_to_mat(qb, tb, Tb);
        int32_t nO;
        if (P->flags & ORC_NO_OVERLAP) {
            for (int32_t j = 0; j < m; ++j) mask[j] = 1;
            nO = m;
        } else {
            nO = orc_overlap(pts, m, Tb, Tprev, fx, fy, cx, cy, W, H, NULL, P->prec, mask);
        }
        for (int32_t i = 0; i < n; ++i) orc_particle_pose(q_prev, t_prev, ones, x + 6 * (size_t)i, T + 12 * (size_t)i);
        orc_fitness(psi, nx, ny, nz, vox, origin, pts, m, mask, T, n, P->lookup, P->prec,
                    !(P->flags & ORC_NO_NORMALIZE), F);
        if (P->prec == ORC_F32)
            for (int32_t i = 0; i < n; ++i) F[i] = (double)(float)F[i];
        int32_t imin = 0;
        double srho = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            if (F[i] < F[imin]) imin = i;
            srho += orc_exp(-F[i] / P->tau);
        }
        best_index[k - 1] = -1;
        if (F[imin] < Fb) {
            double u[6];
            Fb = F[imin];
            for (int d = 0; d < 6; ++d) {
                xb[d] = x[6 * (size_t)imin + d];
                u[d] = (double)xb[d];
            }
            orc_pose_retract(q_prev, t_prev, u, qb, tb);
            best_index[k - 1] = imin;
        }
        rho_best[k - 1] = orc_exp(-Fb / P->tau);
        rho_mean[k - 1] = srho / (double)n;
        n_overlap[k - 1] = nO;
        if (k == K) break;
        if (P->method == ORC_SWARM_PFO) {
            orc_pfo_resample(F, n, Fb, P->tau, (double)offsets[k - 1], anc);
            const float* N = draws + (size_t)(k - 1) * n * 6;
            for (int32_t i = 0; i < n; ++i)
                for (int d = 0; d < 6; ++d) {
                    const float step = sig[d] * N[6 * (size_t)i + d];
                    xn[6 * (size_t)i + d] = x[6 * (size_t)anc[i] + d] + step;
                }
            float* tmp = x;
            x = xn;
            xn = tmp;
        } else {
            for (int32_t i = 0; i < n; ++i)
                if (F[i] < pF[i]) {
                    pF[i] = F[i];
                    memcpy(pb + 6 * (size_t)i, x + 6 * (size_t)i, 6 * sizeof(float));
                }
            const double w = P->w_start + (P->w_end - P->w_start) * (double)(k - 1) / (double)(K - 1);
            orc_pso_move(x, v, pb, xb, draws + (size_t)(k - 1) * n * 12, n, (float)w, (float)P->c1, (float)P->c2,
                         vmx);
        }
    }
    memcpy(q_out, qb, sizeof qb);
    memcpy(t_out, tb, sizeof tb);
    *rho_out = orc_exp(-Fb / P->tau);
    free(pts); free(mask); free(T); free(F); free(x); free(xn); free(v); free(pb); free(pF); free(anc);
    return 0;
}
