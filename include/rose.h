/*
 * rose.h -- C ABI of the MI355X (gfx950) PST pose-search library.
 *
 * The library implements the per-frame camera tracking of ROSEFusion
 * (Zhang, Zhu, Ma, Xu -- "ROSEFusion: Random Optimization for Online Dense
 * Reconstruction under Fast Camera Motion", ACM TOG 40(4), 2021): particle
 * filter optimisation with a particle swarm template (PST) against a TSDF
 * volume (Sec. 3.3, Alg. 1, Sec. 4), and the volumetric depth fusion it
 * builds on (Sec. 3, "volumetric depth fusion framework").
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Every call returns a rose_status and never throws.  Arguments are
 *   validated before anything is enqueued; on a non-OK status nothing was
 *   enqueued and rose_last_error() holds a text for the calling thread.
 * - "_dev" pointers are device pointers (HIP device memory, e.g. the storage
 *   of a torch tensor on the GPU).  All other pointers are host pointers.
 *   Buffers belong to the caller; the library never frees caller memory.
 * - Work is enqueued on the given stream `s` (0 = the null stream) and is
 *   asynchronous unless stated otherwise.
 * - Poses map camera to world: X = R x + t (Eq. unproj).  Quaternions are
 *   (w, x, y, z), Hamilton convention, unit length.  Lengths are metres.
 * - Camera frame: x right, y down, z forward; depth is z-depth in metres,
 *   0 (or any value that is not > 0) marks a missing measurement.
 * - The TSDF stores psi = (signed distance / truncation), clamped to
 *   [-1, 1]; unobserved voxels hold +1 with weight 0, and a query outside the
 *   grid reads +1 (a penalty, never an exclusion).
 */
#ifndef ROSE_H
#define ROSE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROSE_OK = 0,
    ROSE_E_ARG = -1,         /* a NULL/negative/out-of-range argument */
    ROSE_E_SHAPE = -2,       /* sizes inconsistent or above a documented limit */
    ROSE_E_DEVICE = -3,      /* a HIP runtime call failed */
    ROSE_E_STATE = -4,       /* the call cannot run in the current state (e.g. no valid depth) */
    ROSE_E_UNSUPPORTED = -5  /* valid request that this build does not implement */
} rose_status;

typedef enum { ROSE_TSDF_F32 = 0, ROSE_TSDF_F16 = 1, ROSE_TSDF_SN16 = 2 } rose_tsdf_fmt;
typedef enum { ROSE_LOOKUP_NEAREST = 0, ROSE_LOOKUP_TRILINEAR = 1 } rose_lookup;

/* pso_track_frame flags: the ablation switches of Sec. 5.2 (Tab. ablt-tsdf) */
#define ROSE_FLAG_NO_OVERLAP 1   /* O_k := every valid point (Eq. validness skipped) */
#define ROSE_FLAG_NO_NORMALIZE 2 /* fitness = exp(-sum psi^2 / tau) (Eq. ourlh) instead of Eq. normallh */
/* APS threshold rho(s*_{k-1}): Sec. 4 never evaluates the fitness of a best
 * state and uses the weighted APS average of Eq. wafit in its place; by
 * default the threshold is therefore that average, carried from the last
 * non-empty iteration (at k = 1, the centre's own fitness: template row 0
 * sits at c_0).  With this flag: the centre's exact fitness at every k. */
#define ROSE_FLAG_CENTRE_THRESHOLD 4
/* Rescaling ablation (Sec. 5 ablation of Eq. rsinter; at most one of the
 * two): ISO_ONLY replaces the attractor direction |v|/||v|| by the isotropic
 * unit vector 1/sqrt6, rhat = (1 - rho~)/sqrt6 + eps; ANISO_ONLY drops the
 * isotropic factor, rhat = |v|/||v|| + eps.  Non-empty APS only. */
#define ROSE_FLAG_ISO_ONLY 8
#define ROSE_FLAG_ANISO_ONLY 16
/* "No Kahan" of the TSDF-normalisation ablation (Sec. 5): each particle's
 * sum of psi^2 is taken directly in binary32 -- with points across the
 * lanes, per lane a running fmaf sum over its points, then a butterfly sum
 * over the wavefront; with one particle per lane, a running fmaf sum over
 * each quarter of a slice, the four added in order -- instead of in
 * binary64 over exact squares; the 8-64 slice totals are still added in
 * binary64.  Binary32 volumes below 4 GB only (ROSE_E_UNSUPPORTED otherwise);
 * not supported by pso_batch_*. */
#define ROSE_FLAG_NO_KAHAN 32

#define ROSE_MAX_ITERS 32
#define ROSE_MAX_LEVELS 4
#define ROSE_MAX_PARTICLES 65536
#define ROSE_MAX_IMAGE_PIXELS (4096 * 4096)

typedef struct {
    float fx, fy, cx, cy;   /* pinhole intrinsics in pixels */
    int32_t width, height;  /* image size; depth images are row-major height x width */
} rose_camera;

typedef struct {
    double q[4]; /* unit quaternion (w, x, y, z) */
    double t[3]; /* translation, metres */
} rose_pose;

typedef struct rose_tsdf rose_tsdf; /* opaque; host-side metadata plus small device scratch */
typedef struct rose_mlp rose_mlp;   /* opaque; learned-proposal network scratch (see below) */

/* Text of the last non-OK status of the calling thread ("" if none). */
const char* rose_last_error(void);
/* Library version string. */
const char* rose_version(void);

/* ------------------------------------------------------------------ TSDF */
/* Bytes of device memory the caller provides for a TSDF of nx*ny*nz voxels
 * in format `fmt`; which = 0 for the psi buffer, 1 for the weight buffer.
 * F32: 4 + 4 bytes per voxel; F16 and SN16: 2 + 2 (u16 weight).  Returns 0
 * for invalid sizes (each dimension a positive multiple of 8, <= 2048). */
size_t tsdf_bytes(int32_t nx, int32_t ny, int32_t nz, rose_tsdf_fmt fmt, int32_t which);

/* Create a TSDF handle over caller-owned device buffers psi_dev and
 * weight_dev (sizes from tsdf_bytes) and enqueue their initialisation to
 * psi = +1, weight = 0 on `s`.  Voxel (i,j,k) covers
 * origin + [i, i+1) * voxel_m (and likewise in y, z); its centre is at
 * origin + (i + 1/2) * voxel_m.  trunc_m is the truncation distance mu;
 * w_max caps the running-average weight (the fusion framework of Sec. 3:
 * Curless & Levoy 1996, KinectFusion 2011).  The buffer layout is internal
 * (8x8x8 bricks, brick-major); use tsdf_export / tsdf_import for a linear
 * view.  Errors:
 * ROSE_E_ARG (NULL pointer, non-positive voxel/truncation, w_max < 1),
 * ROSE_E_SHAPE (dimensions), ROSE_E_DEVICE. */
rose_status tsdf_create(int32_t nx, int32_t ny, int32_t nz, float voxel_m, float trunc_m, const float origin_m[3],
                        rose_tsdf_fmt fmt, float w_max, void* psi_dev, void* weight_dev, hipStream_t s,
                        rose_tsdf** out);

/* Release the handle and its device scratch.  NULL is a no-op.  Never frees
 * the caller's psi/weight buffers.  Synchronises the handle's scratch. */
rose_status tsdf_destroy(rose_tsdf* h);

/* Fuse one depth frame (height x width float32, metres) taken at camera pose
 * T_wc into the TSDF (projective running average, one weight per frame):
 * for every voxel whose centre X maps to camera coordinates x_c = T^-1 X
 * with z_c > 0 and a nearest pixel (u, v) = (floor(fx x_c/z_c + cx + 1/2),
 * floor(fy y_c/z_c + cy + 1/2)) inside the image with depth D > 0:
 * sdf = D - z_c; if sdf >= -mu: d = min(1, sdf/mu),
 * psi <- (W psi + d)/(W + 1), W <- min(W + 1, w_max).
 * The geometry is evaluated in binary32 in the operation order of the
 * library's numerics notes (folded voxel->camera transform, fmaf chain,
 * correctly rounded division).  Errors: ROSE_E_ARG, ROSE_E_SHAPE. */
rose_status tsdf_integrate(rose_tsdf* h, const float* depth_dev, const rose_camera* cam, const rose_pose* T_wc,
                           hipStream_t s);

/* Copy the TSDF to / from linear float32 buffers laid out [k][j][i]
 * (i fastest), nx*ny*nz elements each: psi decoded to float, weight as
 * float.  tsdf_import encodes into the handle's format (round to nearest
 * even for F16; round(psi * 32767) clamped for SN16; weights rounded and
 * clamped to [0, 65535] for u16).  weight_lin_dev may be NULL in
 * tsdf_import: weights then become 1 where psi < 1 and 0 elsewhere. */
rose_status tsdf_export(const rose_tsdf* h, float* psi_lin_dev, float* weight_lin_dev, hipStream_t s);
/* The handle keeps one bit per 8x8x8 brick, set while every voxel of the
 * brick holds exactly +1; the fitness kernels skip the reads of such
 * bricks (the value is known), fusion clears bits and tsdf_create /
 * tsdf_import rebuild them.  After writing the psi buffer in any other way,
 * call tsdf_rescan (asynchronous on s) before the next fitness call.
 * ROSE_E_ARG for a NULL handle. */
rose_status tsdf_rescan(rose_tsdf* h, hipStream_t s);

/* Particle schedule orders.  The first track call with a PST template on a
 * handle reads the template back once and caches the order in which the
 * fitness kernels take its rows (similar rotations together, for cache
 * reuse), keyed by the template's device pointer and row count, up to 8
 * templates per handle; further templates run in index order.  Results do
 * not depend on the order, only speed does: a template rewritten in place,
 * or new template data at the address of a freed one (as a caching
 * allocator hands out), keeps the old order.  tsdf_forget_templates drops
 * the cache (it waits for the device to be idle and frees the orders;
 * batches created on the handle hold the old orders and must be created
 * again); tsdf_template_orders returns the number cached. */
rose_status tsdf_forget_templates(rose_tsdf* h);
int32_t tsdf_template_orders(const rose_tsdf* h);
rose_status tsdf_import(rose_tsdf* h, const float* psi_lin_dev, const float* weight_lin_dev, hipStream_t s);

/* -------------------------------------------------------------- PST (a1) */
/* Pre-sample the particle swarm template (Sec. 3.3; Sec. 4 "PST
 * pre-sampling"): n particles uniform in the closed unit 6-ball, written as
 * n x 6 float32 (q_x, q_y, q_z, x, y, z) to out_dev.  Row 0 is the origin
 * (the PST centre).  Row i > 0 takes the first accepted attempt a of:
 * Philox4x64-10 (Salmon et al., SC 2011) block with counter (i, a, 0, 0),
 * key (seed, 0); m_0..m_5 = bits 63..40 and 39..16 of words 0, 1, 2;
 * a_d = 2 m_d + 1 - 2^24; accept iff sum a_d^2 <= 2^48 (exact integers);
 * p_d = a_d * 2^-24 (exact).  1024 rejected attempts give the zero row.
 * Errors: ROSE_E_ARG (n < 1 or > ROSE_MAX_PARTICLES, NULL). */
rose_status pst_sample(int32_t n, uint64_t seed, float* out_dev, hipStream_t s);

/* 6D Poisson-disk PST template (Sec. 4 "PST pre-sampling" samples the
 * template as a 6D Poisson disk) by dart throwing over pst_sample's stream:
 * the candidates are rows 1, 2, ... of pst_sample(max_candidates + 1, seed)
 * (written to work_dev, (max_candidates + 1) x 6 floats); row 0 (origin) is
 * accepted first; a candidate is accepted iff its squared distance to every
 * point accepted before it is >= r_min^2, decided exactly on the sampler's
 * lattice (threshold ceil(r_min^2 2^48) in units of 2^-48).  Stops at n rows
 * or after max_candidates candidates.  out_dev: n x 6, accepted rows in
 * acceptance order, the rest 0.  result_dev (2 int32): rows accepted (n on
 * success), candidates drawn.  r_min in [0, 2]; r_min = 0 gives
 * pst_sample's template.  1 <= n <= ROSE_MAX_PARTICLES; max_candidates in
 * [0, 2^24].  Asynchronous on s. */
rose_status pst_poisson(int32_t n, uint64_t seed, double r_min, int32_t max_candidates, float* work_dev,
                        float* out_dev, int32_t* result_dev, hipStream_t s);

/* Particle poses (Alg. 1 MovePST + RescalePST applied on the fly to the
 * stored unit template, Sec. 4 "GPU implementation"): for each row p_i,
 * u = r (.) p_i and pose_i = c * Delta(u), Delta(u) = (quaternion
 * (sqrt(1 - |u_123|^2), u_1, u_2, u_3), translation u_456).  Writes
 * n x 12 binary64 [R|t] row-major to T_dev.  Diagnostic view of the pose
 * build that pso_track_frame performs inside its fitness kernel. */
rose_status pst_particle_poses(const rose_pose* centre, const double r[6], const float* pst_dev, int32_t n,
                               double* T_dev, hipStream_t s);

/* --------------------------------------------------------- fitness (a5) */
/* Fitness of n arbitrary poses over m camera-frame points (Eq. ourlh with
 * the normalisation of Eq. normallh over the given points):
 * F_i = (1/m) sum_j psi(R_i x_j + t_i)^2 and rho_i = exp(-F_i) (tau = 1).
 * pts_dev: m x 3 float32; T_dev: n x 12 float32 row-major [R|t]
 * camera->world; F_dev: n float32; rho_dev: n float32 or NULL.  m = 0 gives
 * F = 1.  The voxel is chosen in binary32 from a transform folded with the
 * voxel scale in binary64 and rounded once; squares are summed in binary64.
 * Limits: n <= ROSE_MAX_PARTICLES, m <= ROSE_MAX_IMAGE_PIXELS.  The call
 * packs the points into, and sums into, scratch owned by the handle (grown
 * on demand, freed by tsdf_destroy), hence the non-const handle. */
rose_status fitness_eval(rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                         rose_lookup lk, float* F_dev, float* rho_dev, hipStream_t s);

/* fitness_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results (bit for bit) from the same kernels, but the packed
 * points and the partial sums live in a fixed scratch array of the library
 * (8 MiB per device, held from the first call on that device until the
 * process ends) instead of the handle's scratch; the handle is not changed.
 * No allocation, no free, no allocating library call.  Limits: m <=
 * fitness_eval_noalloc_max_points() (131072), and n times the point slices
 * the launch uses at most 196608 (ROSE_E_ARG otherwise, before anything is
 * enqueued).  Calls that overlap on one device share the scratch and race:
 * serialise them (one stream, or events).  Errors as fitness_eval, plus
 * ROSE_E_DEVICE when the scratch address cannot be obtained. */
rose_status fitness_eval_noalloc(const rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                                 rose_lookup lk, float* F_dev, float* rho_dev, hipStream_t s);
int32_t fitness_eval_noalloc_max_points(void);

/* Diagnostic: the NEAREST voxel of every (pose, point) pair of fitness_eval
 * as a linear index (k*ny + j)*nx + i, or -1 outside the grid; idx_dev is
 * n x m int64. */
rose_status fitness_voxel_indices(const rose_tsdf* h, const float* pts_dev, int32_t m, const float* T_dev, int32_t n,
                                  int64_t* idx_dev, hipStream_t s);

/* ------------------------------------------------- points (a2) / overlap (a3) */
/* Stride-s unprojection (Eq. unproj; Sec. 4 stride-based downsampling):
 * pixels (u, v) = (0, s, 2s, ..) x (0, s, 2s, ..) with depth z > 0 give
 * x = (((float)u - cx) z / fx, ((float)v - cy) z / fy, z) (binary32),
 * written as count x 3 float32 to pts_dev (capacity ceil(H/s) * ceil(W/s)
 * points); the count goes to *count_dev (int32).  order 0: row-major sample
 * order; order 1: 8x8-sample tiles in row-major tile order (the order the
 * tracker uses internally, for cache-line sharing of the TSDF gathers). */
rose_status depth_unproject(const float* depth_dev, const rose_camera* cam, int32_t stride, int32_t order,
                            float* pts_dev, int32_t* count_dev, hipStream_t s);

/* Overlap mask (Eq. validness): mask_dev[j] = 1 iff point j, moved to the
 * world by `centre` and into the previous camera by prev^-1, has z' > 0 and
 * projects inside [0, W-1] x [0, H-1] (binary32, continuous pixel
 * coordinates).  m points, m x 3 float32.
 * prev_depth_dev: NULL (the test is image bounds only), or the depth image
 * of frame t-1 (H x W float32, device, caller-owned, read only) for the
 * stricter reading of "inside the previous depth image": the pixel nearest to
 * the projection, (floor(px + 1/2), floor(py + 1/2)) in binary32, must also
 * hold a depth > 0. */
rose_status overlap_mask(const float* pts_dev, int32_t m, const rose_pose* centre, const rose_pose* prev,
                         const rose_camera* cam, const float* prev_depth_dev, uint8_t* mask_dev, hipStream_t s);

/* --------------------------------------- learned-proposal inputs (a10) */
/* Render the TSDF at camera pose T_wc through the given (low-resolution)
 * intrinsics: for each pixel the ray is sampled at z = near + k step
 * (z-depth) with trilinear psi; the first pair of consecutive samples with
 * psi_k > 0 >= psi_{k+1}, both within the truncation band (|psi| < 1),
 * gives z* = z_k + step psi_k / (psi_k - psi_{k+1}); none: 0.  Binary64
 * geometry.  depth_out_dev: height x width float32.  At most 2^20 pixels
 * and 1e6 steps per ray. */
rose_status tsdf_raycast(const rose_tsdf* h, const rose_pose* T_wc, const rose_camera* cam, double near_m,
                         double far_m, double step_m, float* depth_out_dev, hipStream_t s);

/* Feature vector of the learned proposal (dim >= w*h + 6 floats):
 * element i < w*h (low-res pixel (u, v), row-major) is the depth residual
 * clamp(D(scale u + scale/2, scale v + scale/2) - render(u, v), -0.5, 0.5)
 * where both depths are > 0, else 0; the next 6 are `velocity` (the previous
 * inter-frame motion in the chart of Sec. 3.3); the rest are 0.
 * depth_dev: full-resolution frame (cam); render_dev: tsdf_raycast output
 * (cam_low). */
rose_status proposal_features(const float* depth_dev, const rose_camera* cam, const float* render_dev,
                              const rose_camera* cam_low, int32_t scale, const double velocity[6], int32_t dim,
                              float* features_dev, hipStream_t s);

/* ---------------------------------------------------- per-frame tracking */
typedef struct {
    int32_t max_iters;  /* 1..ROSE_MAX_ITERS (paper: 20) */
    int32_t early_stop; /* 1: stop on two consecutive empty APS or |u*_d| < stop_tol for all d */
    int32_t stride;     /* depth subsampling stride, >= 1 */
    int32_t lookup;     /* rose_lookup */
    int32_t flags;      /* ROSE_FLAG_* */
    int32_t levels;     /* 0 or 1: one resolution (n_particles, stride); 2..ROSE_MAX_LEVELS: the schedule below */
    double beta;        /* momentum of Eq. momentum (paper: 0.1) */
    double eps;         /* epsilon of Eq. rsinter (paper: 1e-3) */
    double tau;         /* temperature of Eq. pfolh (paper: 1) */
    double stop_tol;    /* stop tolerance (paper: 1e-6) */
    /* Multi-resolution PST (Sec. 4 "Multi-resolution PST"): iteration k uses
     * level (k - 1) mod levels, i.e. the first level_n[l] template rows
     * (1 <= level_n[l] <= n_particles) and the frame subsampled with stride
     * level_stride[l] (>= 1); centre, axis lengths, APS threshold and stop
     * rules carry across levels.  A level without valid samples evaluates
     * F = 1 for every particle.  The paper's (1024, 1/8), (3072, 1/16),
     * (10240, 1/32) read as pixel fractions are strides 3, 4, 6.  Ignored when
     * levels <= 1; not supported by pso_batch_* or the learned frame. */
    int32_t level_n[ROSE_MAX_LEVELS];
    int32_t level_stride[ROSE_MAX_LEVELS];
} rose_track_params;

typedef struct {
    rose_pose pose;      /* in: s^{t-1}_* (previous final pose); out: s^t_* */
    double r[6];         /* in: r_0 = r_1^{t-1}; out: r_1^t (axis lengths after iteration 1) */
    double rho;          /* out: approximated fitness (Eq. wafit) of the last non-empty iteration */
    int32_t tsdf_built;  /* in: 0 for the first frame (Sec. 4 corner case 1) */
    int32_t frame;       /* incremented by each successful call */
} rose_track_state;

typedef struct {
    int32_t iters;          /* iterations run */
    int32_t n_points;       /* valid subsampled points (of level 0 under a multi-resolution schedule) */
    int32_t n_overlap_last; /* |O_k| of the last iteration */
    int32_t status;         /* pso_batch_track: per-sequence status (ROSE_E_STATE: no valid depth) */
    int32_t aps_size[ROSE_MAX_ITERS];
    int32_t n_overlap[ROSE_MAX_ITERS]; /* |O_k| per iteration */
    double rho_iter[ROSE_MAX_ITERS];   /* rho~ per iteration (rho of the centre when the APS is empty) */
    int32_t n_particles[ROSE_MAX_ITERS]; /* particles evaluated per iteration */
    double rho_centre[ROSE_MAX_ITERS];   /* exact rho of the centre c_{k-1} (particle 0) in iteration k */
    double r_iter[ROSE_MAX_ITERS][6];    /* axis lengths r_{k-1} that scale the template in iteration k */
    int32_t fit_mode[ROSE_MAX_ITERS];    /* fitness kernel that did the work in iteration k: 0 one fixed launch
                                          * shape; switching mode: 1 points across the lanes, 2 one particle
                                          * per lane (pso_track_frame; 0 elsewhere) */
} rose_track_stats;

/* One frame of Alg. 1 (PFO with PST) on the device.
 * depth_dev: the current depth frame (cam->height x cam->width float32).
 * prev_depth_dev: NULL, or the previous depth frame (same size, device,
 * read only) for the stricter overlap test of overlap_mask (a point of O_k
 * must also land on a valid pixel of frame t-1).
 * pst_dev: n_particles x 6 template from pst_sample (row 0 = origin).
 * init_centre: PST centre c_0 (NULL: state->pose, i.e. c_0 = s^{t-1}_*);
 * init_r: r_0 (NULL: state->r).  The overlap set always reprojects into the
 * previous frame's camera at state->pose.
 * Every iteration k: O_k with the centre c_{k-1}; fitness of every particle
 * pose c_{k-1} * Delta(r_{k-1} (.) p_i) (Eq. normallh); APS = particles with
 * fitness above rho(s*_{k-1}) (see ROSE_FLAG_CENTRE_THRESHOLD); CompBestState (Eq. ebs),
 * approximated best fitness (Eq. wafit), CompAxisLength (Eqs. rsdir,
 * rsinter with |v_d|, momentum), MovePST (c_k = c_{k-1} * Delta(u*)) and the
 * corner cases of Sec. 4.  The whole loop runs on the device; the call
 * synchronises `s` once at the end and then fills state/stats.  The first
 * call with a template (pointer and particle count) on a handle also reads
 * the template back once to derive the order in which wavefronts take the
 * particles (similar rotations together, for cache reuse); results do not
 * depend on that order.
 * state->tsdf_built == 0: no fitness is evaluated; r_1 = beta r_0 +
 * (1-beta) 0.5 and the pose is kept.  Returns ROSE_E_STATE (state
 * unchanged) when the frame has no valid point.
 * Limits: n_particles <= ROSE_MAX_PARTICLES; image <= ROSE_MAX_IMAGE_PIXELS.
 * A handle must not be used by two streams at once. */
rose_status pso_track_frame(rose_tsdf* h, const float* depth_dev, const float* prev_depth_dev,
                            const rose_camera* cam, const float* pst_dev, int32_t n_particles,
                            const rose_track_params* p, const rose_pose* init_centre, const double* init_r,
                            rose_track_state* state, rose_track_stats* stats, hipStream_t s);

/* ------------------------------------------- comparison optimisers */
/* The two optimisers that Sec. 5 (ablation of the optimisation strategy)
 * compares PFO with PST against: vanilla PFO (Sec. 3.1: Gaussian proposal,
 * Eq. proposal; weights by the likelihood of Eq. pfolh, Eq. weight;
 * resampling) and PSO (inertia-weight particle swarm optimisation with a
 * global best).  Both use the fitness of Eq. normallh and the same particle
 * count.  The paper gives neither method's parameters; the definitions:
 *  - state: x in R^6 (binary32) in the chart at c_0 = state->pose, i.e. the
 *    pose c_0 * Delta(x); start x_i = (float)(r_init_d * p_i,d) from the PST
 *    template rows p_i (the initial particle set of PFO with PST);
 *  - iteration k = 1..iters: O_k = overlap set (Eq. validness) of the best
 *    state so far s*_{k-1} (s*_0 = c_0); F_i = fitness of c_0 * Delta(x_i)
 *    over O_k, kept in binary32; the best state becomes the particle with
 *    the smallest F_i (lowest index on ties) if that is below F*; then, for
 *    k < iters, one step of the method;
 *  - vanilla PFO step: w_i = exp(-(F_i - F*) / tau) (uniform weights after
 *    the previous resampling, so Eq. weight is Eq. pfolh with g(s*) = F*);
 *    systematic resampling, C_i = w_0 + .. + w_i, the ancestor of slot m is
 *    the first i with C_i > ((m + u_k) / n) C_{n-1}; proposal
 *    x'_m = x_{a_m} + sigma (.) z_{k,m} (product and sum rounded to binary32);
 *  - PSO step: personal best p_i (F_i below the particle's best so far);
 *    w_k = w_start + (w_end - w_start)(k - 1)/(iters - 1);
 *    v = ((w_k v + (c1 r1)(p_i - x)) + (c2 r2)(x* - x)) clamped to
 *    [-vmax, vmax], x = x + v, binary32 in this order, v starting at 0;
 *  - result: state->pose = c_0 * Delta(x*) (quaternion renormalised),
 *    state->rho = exp(-F* / tau), state->frame + 1; state->r is untouched.
 * Random numbers are inputs (device buffers, float32): PFO normals_dev
 * iters x n x 6 standard normals z and offsets_dev iters uniforms u_k in
 * [0, 1); PSO uniforms_dev iters x n x 12 (r1 in columns 0-5, r2 in 6-11).
 * Row k - 1 serves the step after iteration k (the last row is not read).
 * flags: ROSE_FLAG_NO_OVERLAP and ROSE_FLAG_NO_NORMALIZE (others: E_ARG).
 * state->tsdf_built == 0: nothing to search, the pose is kept (OK).  No
 * valid depth sample: ROSE_E_STATE, state unchanged.  The search runs on
 * the device and the call synchronises `s` once at the end.  Scratch
 * (108 bytes per particle) is owned by the handle. */
typedef struct {
    int32_t iters;      /* 1..ROSE_MAX_ITERS */
    int32_t stride;     /* depth subsampling stride (>= 1) */
    int32_t lookup;     /* rose_lookup */
    int32_t flags;      /* ROSE_FLAG_NO_OVERLAP | ROSE_FLAG_NO_NORMALIZE */
    double tau;         /* temperature (> 0; paper: 1) */
    double r_init[6];   /* axis lengths of the initial set (>= 0) */
    double sigma[6];    /* vanilla PFO: standard deviation of the proposal per axis (>= 0) */
    double w_start, w_end; /* PSO: inertia weight at the first and last iteration */
    double c1, c2;      /* PSO: acceleration towards the personal and the global best */
    double vmax[6];     /* PSO: velocity clamp per axis (>= 0) */
} rose_swarm_params;

typedef struct {
    int32_t iters;                       /* iterations run */
    int32_t n_points;                    /* valid subsampled points */
    int32_t n_overlap[ROSE_MAX_ITERS];   /* |O_k| */
    int32_t best_index[ROSE_MAX_ITERS];  /* particle that improved F* in iteration k, -1 if none */
    double rho_best[ROSE_MAX_ITERS];     /* exp(-F* / tau) after iteration k */
    double rho_mean[ROSE_MAX_ITERS];     /* mean over the particles of exp(-F_i / tau) in iteration k */
} rose_swarm_stats;

rose_status vanilla_pfo_track_frame(rose_tsdf* h, const float* depth_dev, const rose_camera* cam,
                                    const float* pst_dev, int32_t n_particles, const rose_swarm_params* p,
                                    const float* normals_dev, const float* offsets_dev, rose_track_state* state,
                                    rose_swarm_stats* stats, hipStream_t s);
rose_status plain_pso_track_frame(rose_tsdf* h, const float* depth_dev, const rose_camera* cam, const float* pst_dev,
                                  int32_t n_particles, const rose_swarm_params* p, const float* uniforms_dev,
                                  rose_track_state* state, rose_swarm_stats* stats, hipStream_t s);

/* Chart of Sec. 3.3 between two poses: u = (imaginary part of the
 * quaternion of a^-1 b with w >= 0, translation of a^-1 b), so that
 * b = a * Delta(u) (rose_chart_exp).  Host functions. */
rose_status rose_chart_log(const rose_pose* a, const rose_pose* b, double u[6]);
rose_status rose_chart_exp(const rose_pose* a, const double u[6], rose_pose* out);

/* ----------------------------------------- learned proposal frame (a11, a13) */
typedef struct {
    int32_t low_w, low_h, scale; /* residual grid (40 x 30) and its subsampling of the frame (16 at 640x480) */
    int32_t feature_dim;         /* network input size (>= low_w * low_h + 6; 1216) */
    double kappa;                /* r_0 = kappa * exp(l), clamped to [r_min, r_max] */
    double r_min, r_max;
    double delta;                /* fall back when rho < previous rho - delta */
    double near_m, far_m, step_m;/* raycast range and step */
    int32_t iters;               /* iterations of the learned run (0: p->max_iters; the fallback uses p) */
    int32_t reserved;
} rose_learned_params;

/* One frame with the learned PST proposal: render the model at the previous
 * pose (tsdf_raycast), build the residual features (proposal_features with
 * `velocity`), run the network (rose_mlp_forward, B = 1) for (mu, l); centre
 * the small template at c_0 = s^{t-1} * Delta(mu) with axis lengths
 * r_0 = kappa exp(l) and run pso_track_frame.  The result is kept unless the
 * network output is not finite or the final fitness falls below the previous
 * frame's state->rho - delta; then plain pso_track_frame with the plain
 * template runs from the unchanged state (fallback, *fallback_out = 1).
 * work_dev: >= low_w*low_h + feature_dim + 12 floats of device scratch.
 * Synchronises `s`. */
rose_status pso_track_frame_learned(rose_tsdf* h, const float* depth_dev, const rose_camera* cam,
                                    const float* pst_small_dev, int32_t n_small, const float* pst_plain_dev,
                                    int32_t n_plain, rose_mlp* mlp, const float* mlp_params_dev, float* work_dev,
                                    const double velocity[6], const rose_track_params* p,
                                    const rose_learned_params* lp, rose_track_state* state, rose_track_stats* stats,
                                    int32_t* fallback_out, hipStream_t s);

/* ------------------------------------------------- batched tracking (a14) */
/* Many independent sequences (each its own TSDF handle, camera, template,
 * particle count and parameters) tracked in lockstep, one frame step per
 * pso_batch_track call, with the same per-sequence semantics as
 * pso_track_frame.  Per frame step the device work is: one unprojection /
 * overlap launch (one workgroup per sequence), then per iteration one
 * persistent fitness launch per group over the sequences that share it, the
 * fitness launches of pso_track_frame for each sequence that has its own
 * (see rose_batch_set_own_launch), one slice-reduction launch and one update
 * launch, then one launch copying the states to pinned host memory; with
 * use_graph != 0 and a non-null stream it is captured into a HIP graph on
 * the first call and replayed afterwards (new inputs are read from pinned
 * host memory; a change of a handle's scratch pointers makes the next call
 * capture again).  The persistent launches run the first handle's launch
 * shape when the batch is created -- the fixed shape set by
 * rose_fitness_set_shape or tsdf_set_fitness_shape if it is (4,2), (8,2),
 * (4,4), (8,4), (4,8) or (64,8), in the switching mode its points-across
 * shape, otherwise (4,2) -- one per iteration and per group of sequences
 * that share a storage format and lookup; their workgroups take work items
 * from one counter per XCD, cleared by the kernel before each fitness
 * round.
 * Creation reads each template back once to derive the particle schedule
 * order (as pso_track_frame does).  Volumes must be below 4 GB.  The handles
 * must stay alive while the batch exists; tracking one through another path
 * between batch steps is allowed (the batch re-reads the handles' scratch
 * pointers before each step). */
typedef struct rose_batch rose_batch;
rose_status pso_batch_create(int32_t count, rose_tsdf* const* tsdfs, const rose_camera* cams,
                             const float* const* pst_devs, const int32_t* n_particles,
                             const rose_track_params* params, int32_t use_graph, rose_batch** out);
/* depth_devs[count]; init_centres (count poses) and init_rs (count x 6) may be
 * NULL (each sequence then starts from its state, as in pso_track_frame);
 * states[count] in/out; stats[count] (nullable) receive per-sequence status.
 * Synchronises `s` once. */
rose_status pso_batch_track(rose_batch* b, const float* const* depth_devs, const rose_pose* init_centres,
                            const double* init_rs, rose_track_state* states, rose_track_stats* stats,
                            hipStream_t s);
rose_status pso_batch_destroy(rose_batch* b);
/* Which sequences of a batch created afterwards take launches of their own:
 * those whose handle runs the switching mode (rose_fitness_set_shape(0, 0)
 * or tsdf_set_fitness_switch) and whose iteration holds at least min_evals
 * particle x point evaluations (n_particles x ceil(width / stride) x
 * ceil(height / stride)).  They run pso_track_frame's fitness launches
 * (both kernels, the one for the current search footprint chosen on the
 * device; stats fit_mode reports it) inside the batch's stream or graph, in
 * sequence order; the persistent launches have no particle-per-lane side
 * and serve the others.  Process-wide, host-only; default 8388608 (2^23);
 * 0: every switching-mode sequence; ROSE_E_ARG if min_evals < 0.  Results
 * do not depend on it. */
rose_status rose_batch_set_own_launch(int64_t min_evals);

/* Batched learned frame step: for every sequence of batch b whose model
 * exists, the learned proposal of pso_track_frame_learned (raycast at the
 * previous pose, features with velocities[6 i .. 6 i + 5], one forward of the
 * network over all sequences, B = count <= the network's max_batch), then
 * one pso_batch_track step of b (its templates and parameters drive the
 * learned runs: create b with the small templates and the learned-run
 * iteration count) from the proposed centres and axis lengths.  A sequence
 * whose proposal is not finite, whose frame has no valid depth, or whose
 * final fitness falls below its previous state->rho - delta is tracked again
 * by plain pso_track_frame from its unchanged state with pst_plain_devs[i],
 * n_plain[i], plain_params[i] (fallback_out[i] = 1; stats[i].status carries
 * that call's status).  Sequences without a model (tsdf_built = 0) take the
 * batch's first-frame step.  work_dev: count x (low_w low_h + feature_dim +
 * 12) floats.  The results equal pso_track_frame_learned per sequence.
 * Synchronises s. */
rose_status pso_batch_track_learned(rose_batch* b, const float* const* depth_devs, rose_mlp* mlp,
                                    const float* mlp_params_dev, float* work_dev, const double* velocities,
                                    const rose_learned_params* lp, const float* const* pst_plain_devs,
                                    const int32_t* n_plain, const rose_track_params* plain_params,
                                    rose_track_state* states, rose_track_stats* stats, int32_t* fallback_out,
                                    hipStream_t s);

/* ------------------------------------------- learned proposal network */
/* A 3-layer perceptron in -> hid (GELU) -> hid (GELU) -> 12, output
 * (mu in R^6, log-scale l in R^6) of the PST centre increment and axis
 * lengths.  Parameters: one caller-owned float32 device buffer of
 * rose_mlp_param_count() elements laid out [W1 (in x hid), b1, W2
 * (hid x hid), b2, W3 (hid x 12), b3], y = x W + b.  The GEMMs run on the
 * matrix cores with BF16 operands (round to nearest even) and FP32
 * accumulation; GELU is the exact erf form.  The handle owns activation
 * scratch for up to max_batch rows.  out_dim must be 12. */
int64_t rose_mlp_param_count(int32_t in_dim, int32_t hidden, int32_t out_dim);
rose_status rose_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t max_batch, rose_mlp** out);
rose_status rose_mlp_destroy(rose_mlp* m);
/* out_dev: B x 12 float32; X_dev: B x in float32 (row-major). */
rose_status rose_mlp_forward(rose_mlp* m, const float* params_dev, const float* X_dev, int32_t B, float* out_dev,
                             hipStream_t s);
/* Heteroscedastic Gaussian NLL, mean over the batch of
 * sum_d [(y_d - mu_d)^2 / (2 exp(2 l_d)) + l_d]; targets Y_dev B x 6.  Writes
 * the gradient w.r.t. every parameter to grads_dev (same layout) and the
 * loss to loss_dev[0] (device float). */
rose_status rose_mlp_loss_grad(rose_mlp* m, const float* params_dev, const float* X_dev, const float* Y_dev,
                               int32_t B, float* grads_dev, float* loss_dev, hipStream_t s);
/* Adam (Kingma & Ba 2015), elementwise on FP32 master weights; step is the
 * 1-based step count used for the bias corrections. */
rose_status rose_mlp_adam(int64_t n, float* params_dev, const float* grads_dev, float* m_dev, float* v_dev,
                          int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t s);
/* The BF16 matrix-core GEMM on its own: C(m, n) = sum_k A(m, k) B(k, n) with
 * A(m, k) = A_dev[m sam + k sak], B(k, n) = B_dev[k sbk + n sbn],
 * C(m, n) = C_dev[m ldc + n]. */
rose_status rose_gemm_bf16(int32_t M, int32_t N, int32_t K, const float* A_dev, int64_t sam, int64_t sak,
                           const float* B_dev, int64_t sbk, int64_t sbn, float* C_dev, int64_t ldc, hipStream_t s);

/* Launch configuration of the fitness kernel.  A handle uses its own
 * configuration once one was set on it (tsdf_set_fitness_shape / _switch),
 * and the process-wide default (rose_fitness_set_*) otherwise; the defaults
 * are read when a call starts.  Neither kind of setting may change while a
 * call that uses it runs on another thread.
 *
 * Shape: particles per wavefront and points per lane per loop step.
 * Compiled shapes: (2, 4), (4, 2) (default), (4, 4), (4, 8), (8, 2), (8, 4)
 * -- points across the lanes, P particles per wave -- and (64, 4), (64, 8),
 * (64, 16) -- one particle per lane, U points looked up per step.  (0, 0)
 * selects the switching mode: pso_track_frame, the learned tracker and the
 * plain fallbacks run the switching mode's points-across shape (default
 * (4, 2), for both lookups) while the search footprint (see
 * rose_fitness_set_switch) is above the threshold and (64, 8) at or below
 * it, decided on the device each iteration from the current axis lengths;
 * fitness_eval and the comparison optimisers run the points-across shape.
 * Other values give ROSE_E_UNSUPPORTED.  The batched tracker runs the first
 * handle's shape (in the switching mode its points-across shape) when it
 * is (4, 2), (8, 2), (4, 4), (4, 8), (8, 4) or (64, 8), else (4, 2).
 * Results do not depend on the shape (the fitness sums are exact). */
rose_status rose_fitness_set_shape(int32_t particles_per_wave, int32_t points_per_lane);

/* Threshold of the switching mode (process-wide default): the footprint of
 * an iteration is max(r_4, r_5, r_6) + reference_depth_m * max(r_1, r_2,
 * r_3) (translation axis lengths plus rotation axis lengths turned into a
 * displacement at the reference depth), in units of the volume's voxel
 * size; at or below footprint_voxels the particle-per-lane kernel runs.
 * Defaults: 48 voxels for nearest lookups, 32 for trilinear ones, at 3 m;
 * a call sets the threshold for both lookups; footprint_voxels = 0 restores
 * the defaults (reference_depth_m ignored).  ROSE_E_ARG unless
 * footprint_voxels is 0 or in (0, 1e6] with 0 <= reference_depth_m <= 1e3.
 * Host-only. */
rose_status rose_fitness_set_switch(float footprint_voxels, float reference_depth_m);
/* The switching mode's points-across shape (process-wide default (4, 2));
 * any compiled shape with fewer than 64 particles per wave, else
 * ROSE_E_UNSUPPORTED. */
rose_status rose_fitness_set_switch_shape(int32_t particles_per_wave, int32_t points_per_lane);

/* The same settings for one handle (fitness_eval, pso_track_frame and the
 * calls built on them with that handle): the shape as in
 * rose_fitness_set_shape, (-1, -1) returning the handle to the process-wide
 * default; the switch threshold as in rose_fitness_set_switch together with
 * the switching mode's points-across shape.  The first call copies the
 * current process-wide default and then changes it.  ROSE_E_ARG (NULL
 * handle, thresholds out of range), ROSE_E_UNSUPPORTED (shapes). */
rose_status tsdf_set_fitness_shape(rose_tsdf* h, int32_t particles_per_wave, int32_t points_per_lane);
rose_status tsdf_set_fitness_switch(rose_tsdf* h, float footprint_voxels, float reference_depth_m,
                                    int32_t wide_particles, int32_t wide_points);

/* ------------------------------------------------------- kernel timing */
/* When enabled (process-wide), pso_track_frame and tsdf_integrate bracket
 * each fitness, update and integration launch with HIP events recorded on
 * the call's stream; rose_profile_read resolves the pending events
 * (synchronising on them), adds their elapsed times to the totals and
 * returns the totals; rose_profile_reset clears them.  Timing perturbs the
 * launch stream slightly and is meant for measurement runs. */
typedef struct {
    double fitness_ms;      /* summed duration of fitness kernel launches */
    int64_t fitness_launches;
    double fitness_evals;   /* summed particle x point evaluations of those launches */
    double update_ms;       /* per-iteration update kernels (APS, PST move/rescale, overlap) */
    int64_t update_launches;
    double integrate_ms;
    int64_t integrate_launches;
} rose_profile;

rose_status rose_profile_enable(int32_t on);
rose_status rose_profile_reset(void);
rose_status rose_profile_read(rose_profile* out);
/* Durations (ms) of the fitness launches timed since the last reset, in
 * launch order: copies min(cap, count) of them to ms_out (host memory) and
 * sets *count_out to the count.  Resolves pending events like
 * rose_profile_read. */
rose_status rose_profile_fitness_launches(float* ms_out, int64_t cap, int64_t* count_out);

/* ------------------------------------------------------------ measurement */
/* Gather-rate probe (the roofline of the fitness kernel's TSDF reads): a
 * launch of `blocks` workgroups of 256 lanes (blocks a positive multiple of
 * 8), each lane issuing iters * rose_gather_peak_loads_per_lane()
 * independent 4-byte loads, every load from a pseudo-random 128-byte line of
 * one of 8 regions of region_lines lines (a power of two <= 2^26), region
 * b mod 8 for workgroup b (one region per XCD).  buf_dev must hold
 * 8 * region_lines * 32 floats (E_SHAPE otherwise); sink_dev (blocks floats)
 * is never written for finite buffer contents.  Asynchronous on s; the
 * caller times it with events on s.  Not part of the method: bench.py uses
 * it to state the kernel's gather roofline. */
rose_status rose_gather_peak(const float* buf_dev, int64_t buf_elems, int32_t region_lines, int32_t blocks,
                             int32_t iters, uint32_t seed, float* sink_dev, hipStream_t s);
int32_t rose_gather_peak_loads_per_lane(void);

/* L2 -> CU read bandwidth probe (the measured P_L2 of the fitness kernel's
 * gather roofline, R_gather = P_L2 / bytes per TSDF element): `blocks`
 * workgroups of 256 lanes (a positive multiple of 8) each sweep, `sweeps`
 * times, one of 8 regions of region_f4 float4 values (a power of two in
 * [1024, 2^24]; region b mod 8 for workgroup b, one per XCD) with coalesced
 * 16-byte loads.  A region that fits the L2 (2 MiB) and exceeds a CU's L1
 * makes every load after the first sweep an L2 hit.  Bytes read =
 * blocks * sweeps * region_f4 * 16.  buf_dev: 8 * region_f4 * 4 floats,
 * 16-byte aligned (E_SHAPE / E_ARG otherwise); sink_dev (blocks floats) is
 * never written for finite contents.  Asynchronous on s.  Not part of the
 * method. */
rose_status rose_l2_read_peak(const float* buf_dev, int64_t buf_elems, int32_t region_f4, int32_t blocks,
                              int32_t sweeps, float* sink_dev, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* ROSE_H */
