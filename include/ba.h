/* ba.h - C-ABI of the MI355X bundle-adjustment library (libba_mi355x.so).
 *
 * What the library computes (paper, Sec. 4.3 "Iterative Triangulation and
 * Mapping"): Levenberg-Marquardt bundle adjustment of SE(3) camera poses and
 * 3D points that minimises C = 1/2 sum_k rho(||r_k||^2) over observations k of
 * point j in camera i, with the reprojection residual of Sec. 4.3,
 *     r_k = pi(K_i (R_i X_j + t_i)) - z_k,   pi(x, y, z) = (x/z, y/z),
 * rho the Huber loss on the squared norm (huber_delta > 0) or rho(s) = s,
 * and arbitrary camera subsets held fixed (Sec. 4.3, fixed-pose designation).
 * Each iteration linearises, forms the per-camera, per-point and camera-point
 * Hessian blocks, eliminates the points (Schur complement onto the reduced
 * camera system), solves that system with block-Jacobi preconditioned CG and
 * back-substitutes the points.  The pose-only entry refines single poses
 * against a fixed map (the localization mode of Sec. 6.4.2).
 *
 * Conventions
 *  - Poses are world -> camera: P_c = R X + t, R from the unit quaternion
 *    (qw, qx, qy, qz), Hamilton convention.  A quaternion whose norm differs
 *    from 1 by more than 1e-6 is rejected; otherwise it is renormalised.
 *  - Pixels: origin at the top-left image corner, u to the right, v down.
 *  - Updates: T <- Exp(xi) T with xi = (rho, phi) in se(3); points additive.
 *  - Ownership: every input is copied during the call that receives it; the
 *    caller may free its arrays afterwards.  Outputs go to caller buffers.
 *    Handles belong to the caller until destroyed.
 *  - Errors: every entry returns an int status (BA_OK = 0, negative on error).
 *    Validation happens before any side effect.  ba_last_error() returns a
 *    thread-local message for the last failing call on this thread.
 *    Non-convergence is not an error: it is reported in ba_report.status.
 *  - Threading: a ba_problem handle must not be used from two threads at once.
 *    All ba_server_* calls are thread-safe.
 *  - Streams: hip_stream may be NULL (the library then creates its own stream)
 *    or a hipStream_t owned by the caller (for example PyTorch's current
 *    stream); the library never destroys a caller's stream.
 */
#ifndef BA_MI355X_H
#define BA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BA_OK 0
#define BA_EINVAL (-1)   /* invalid argument or problem description            */
#define BA_ENOMEM (-2)   /* device allocation failed, or request exceeds budget  */
#define BA_EDEVICE (-3)  /* HIP runtime error                                   */
#define BA_ESTATE (-4)   /* call not valid in the object's current state        */

/* precision modes */
#define BA_PREC_F64 0    /* everything in FP64 (parity build)                                */
#define BA_PREC_F32 1    /* FP32 projection/Jacobians/Schur/SpMV; FP64 state, dot products,
                            cost and gain reductions and 6x6 preconditioner inverses        */
#define BA_PREC_F16J 2   /* as F32, Jacobians stored in FP16 (FP32 accumulation)             */
#define BA_PREC_BF16J 3  /* as F32, Jacobians stored in BF16 (FP32 accumulation)             */

/* ba_report.status */
#define BA_STATUS_OK 0
#define BA_STATUS_DAMPING 1    /* lambda ended at its upper clamp (1e16)     */
#define BA_STATUS_NUMERICAL 2  /* the cost became non-finite                  */
#define BA_STATUS_PCG_SYNC 3   /* the resident PCG's grid barrier timed out (its workgroups
                                  were not all resident at once): the solve stopped with the
                                  step rejected; solve without BA_FLAG_PCG_RESIDENT         */

typedef struct { double fx, fy, cx, cy; } ba_intrinsics;         /* pinhole, no distortion  */
typedef struct { double qw, qx, qy, qz, tx, ty, tz; } ba_pose;   /* world -> camera         */
typedef struct { int32_t cam, pt; double u, v; } ba_obs;         /* one 2D observation      */

typedef struct {
  int32_t max_iters;      /* LM iterations (accepted and rejected both count), >= 1      */
  int32_t pcg_max_iters;  /* products with S per linear solve, >= 1                      */
  double pcg_rel_tol;     /* stop when ||r||_2 <= tol * ||b||_2                           */
  double lambda0;         /* initial LM damping, > 0                                      */
  double huber_delta;     /* <= 0: plain least squares; > 0: Huber threshold in pixels    */
  int32_t precision;      /* BA_PREC_*                                                    */
  int32_t flags;          /* BA_FLAG_* bits, 0 for the defaults                           */
  /* Prior terms of the objective (paper Sec. 4.3: absolute pose constraint, Eq. abs;
     sequential constraint, Eq. seq), read as squared Frobenius norms of 3x4 pose
     differences and added to C as 1/2 weight * e:
       e_a(i)   = ||[R_i | t_i] - [R_i0 | t_i0]||^2 for every camera,
       e_c(i,j) = ||A_ij - A_ij0||^2, A_ij = T_i T_j^-1, for j = i + k, k = 1..prior_seq_k
     in the caller's camera order; T_0 are the poses given to ba_create.  Weights 0
     (the defaults) disable a term.  Not robustified. */
  double prior_abs;       /* lambda_a >= 0                                                  */
  double prior_seq;       /* lambda_c >= 0                                                  */
  int32_t prior_seq_k;    /* 1..64 when prior_seq > 0 (default 1: adjacent frames)          */
  int32_t reserved;       /* 0                                                              */
} ba_options;

/* ba_options.flags bits.
   BA_FLAG_NO_GRAPH: enqueue the kernels of every solve one by one instead of
   replaying a HIP graph captured on the first solve.
   BA_FLAG_PAIR_LISTS: form the Schur complement from per-block observation-pair
   lists (one wavefront per block of S) instead of point chunks staged in LDS.
   The pair-list form is also used whenever one point has more free-camera
   observations than a chunk holds (2048; 1024 in BA_PREC_F64). */
#define BA_FLAG_NO_GRAPH 2
#define BA_FLAG_PAIR_LISTS 4
/* BA_FLAG_PCG_WIDE: run the PCG with 32 reduced-system rows per workgroup (half a
   wave per row) whatever the problem size, when the tile's columns fit in LDS.  By
   default that layout is used only for more than 8192 free cameras. */
#define BA_FLAG_PCG_WIDE 8
/* BA_FLAG_PCG_RESIDENT: run each linear solve of a single-problem solve as ONE launch
   whose workgroups stay resident and meet at a grid barrier once per iteration, instead
   of one launch per iteration: each workgroup keeps its S blocks and preconditioner rows
   in registers for the whole solve, and no launch gaps remain.  The iterates are the
   same, bit for bit.  Used when every workgroup of the solve fits on the device at once
   (at most one 1024-thread workgroup per CU for 4-row tiles) and a tile's columns fit one
   sweep (at most 170); otherwise ignored (ba_problem_info.pcg_resident reports it).  The
   barrier needs the CUs to itself: do not run two such solves at the same time, nor
   other long kernels beside one.  A barrier that times out (about a second) stops the
   solve with status BA_STATUS_PCG_SYNC instead of waiting forever. */
#define BA_FLAG_PCG_RESIDENT 16
/* BA_FLAG_PCG_COOPERATIVE: with BA_FLAG_PCG_RESIDENT, start the resident solve as a
   cooperative launch, so the runtime itself places every workgroup at once (or fails the
   launch) instead of relying on the occupancy count alone; for callers that share the
   device with other work.  Costs about 20 us per linear solve on an idle device.  No
   effect without BA_FLAG_PCG_RESIDENT or where the resident form does not fit. */
#define BA_FLAG_PCG_COOPERATIVE 64
/* BA_FLAG_DENSE_SCHUR: form the Schur complement in its dense co-visibility form, used
   by default when at most 1024 cameras are free, a point is seen by at least a quarter
   of them on average, the observation pairs outnumber 32 per block of S and at least
   half of the free-camera pairs share a point (scenes where every camera sees most
   points).  S is held dense; for each observation the 6x3 block
   Z = W V*^-1/2 (with the Cholesky factor of the point's damped block) is formed on
   the fly, and S = U* - sum Z Z^T is accumulated tile by tile on the matrix cores
   (MFMA in the compute type; FP16 / BF16 operands in BA_PREC_F16J / BA_PREC_BF16J), so
   no per-pair lists are stored.  The flag forces the form for any problem of at most
   1024 free cameras; BA_FLAG_PAIR_LISTS excludes it.  Not used for vehicle rigs. */
#define BA_FLAG_DENSE_SCHUR 32

typedef struct {
  int32_t iters;          /* iterations run                                               */
  int32_t accepted;       /* accepted steps                                               */
  int32_t status;         /* BA_STATUS_*                                                  */
  int32_t n_masked;       /* observations with depth <= 1e-6 at the final state           */
  double cost0;           /* C at the initial state                                       */
  double cost;            /* C at the final state                                         */
  double rms_px;          /* sqrt(sum ||r||^2 / N) over unmasked observations in the problem */
  double lambda;          /* damping after the last iteration                             */
  double *iter_cost;      /* caller buffer of max_iters + 1 entries, or NULL: C_0..C_n    */
  int32_t *pcg_iters;     /* caller buffer of max_iters entries, or NULL                  */
  double solve_ms;        /* device time of the iteration loop (HIP events)               */
  double setup_ms;        /* host symbolic analysis + upload time                         */
} ba_report;

typedef struct {                 /* one problem; all pointers are host memory          */
  int32_t n_cams;
  const ba_intrinsics *K;        /* n_cams entries, or 1 entry shared (K_per_cam = 0)  */
  int32_t K_per_cam;
  const ba_pose *poses;          /* n_cams initial poses                               */
  const uint8_t *cam_fixed;      /* n_cams flags (1 = held fixed), or NULL for none    */
  int32_t n_pts;
  const double *points_xyz;      /* 3 * n_pts initial points                           */
  int64_t n_obs;
  const ba_obs *obs;             /* n_obs observations, any order; each (cam, pt) at most once */
} ba_problem_desc;

typedef struct ba_problem ba_problem;
typedef struct ba_server ba_server;

/* Library version string. */
const char *ba_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *ba_last_error(void);
/* Fill *opt with the defaults: 10 iterations, PCG 50 / 1e-6, lambda0 1e-4,
   no robust loss, BA_PREC_F32. */
void ba_default_options(ba_options *opt);

/* Validate and copy a problem, run the symbolic analysis (observation order,
   Hessian-block and reduced-camera-system sparsity, pair lists of the Schur
   complement) and upload it to the current HIP device.  BA_EINVAL: index out
   of range, non-finite input, bad quaternion, duplicate (cam, pt), n_obs = 0,
   every camera fixed, or bad options.  BA_ENOMEM: device allocation failed. */
int ba_create(const ba_problem_desc *d, const ba_options *opt, void *hip_stream,
              ba_problem **out);
/* Run opt->max_iters LM iterations from the current state (lambda reset to
   lambda0) and wait for them.  The state after the call is the last accepted one. */
int ba_solve(ba_problem *p);
/* Enqueue the iterations on the problem's stream and return; ba_wait blocks.  The
   solve's report (state, final evaluation, per-iteration costs and PCG counts) is
   copied into page-locked memory of the problem behind the solve, so that after
   ba_wait a report from ba_get_result needs no device traffic.  The first call
   allocates that buffer (BA_ENOMEM or BA_EDEVICE if it cannot). */
int ba_solve_async(ba_problem *p);
int ba_wait(ba_problem *p);
/* Restore the poses and points given to ba_create (device-side copy; the
   structure, buffers and options are kept) and put every observation back in
   the problem.  The next solve starts from them. */
int ba_reset(ba_problem *p);

/* ---------------------------------------------------------------- iterative refinement
   The alternation of BA and triangulation of paper Sec. 4.3 ("Iterative
   Triangulation and Mapping"): after each BA round, observations whose
   reprojection error exceeds the outlier threshold leave the problem and the
   points that lost observations are triangulated again from the ones that
   remain; a first stage uses a robust loss and a relaxed threshold, a second no
   loss and a strict one.  Each stage runs `rounds` times: a solve of
   opt->max_iters LM iterations from the current state (lambda reset to lambda0)
   with the stage's loss, then the culling step at the accepted state:
     - an active observation stays iff its depth is > 1e-6 and ||r_k|| <= cull_px
       (FP64 residual from the stored pixels);
     - a point that lost an observation is re-triangulated by the multi-view
       midpoint method (the X minimising the summed squared distances to its
       observation rays, Sec. 4.3's midpoint variant), in FP64, from its active
       observations; if fewer than two remain, the 3x3 system is singular
       (determinant <= 1e-12) or the new point is not in front of every camera
       that observes it, all its observations leave the problem instead.
   Observations out of the problem contribute nothing to C, the Hessian blocks or
   the gradient and are not counted as masked.  ba_reset puts them back.
   BA_EINVAL: n_stages < 1, rounds < 1, stages NULL, a non-finite huber_delta, or
   a cull_px that is not positive and finite (checked before any side effect).
   hist: NULL or n_stages * rounds entries, stage-major.  After the call,
   ba_get_result returns the final state; its report is that of the last solve,
   with n_masked and rms_px evaluated again at the final state over the
   observations still in the problem.  With profiling on and the "cull" kernel
   selected, ba_get_kernel_times reports the culling launches of the call (HIP
   events around each) and, for the other kernels, the last solve's times. */
#define BA_TRI_MIDPOINT 0  /* the multi-view midpoint (Sec. 4.3)                            */
#define BA_TRI_DLT 1       /* the DLT of Eq. dlt in its classical homogeneous form: rows
                              x P_3 - P_1, y P_3 - P_2 in normalized coordinates, X~ the
                              unit minimiser of ||A X~|| (smallest eigenvector of A^T A by
                              Jacobi rotations, FP64), X = X~[:3] / X~[3]; fails when
                              |X~[3]| <= 1e-12                                              */
typedef struct {
  double huber_delta;     /* the stage's loss: <= 0 none, > 0 Huber threshold in pixels  */
  double cull_px;         /* outlier threshold on ||r_k|| in pixels, > 0                 */
  int32_t triangulation;  /* BA_TRI_* method of the stage's re-triangulation             */
  int32_t reserved;
} ba_refine_stage;
typedef struct {
  int32_t stage, round;
  int32_t iters, status;  /* of the round's solve                                        */
  double cost;            /* C at the end of the round's solve (before its culling)      */
  int64_t n_active_obs;   /* observations in the problem after the round's culling       */
  int32_t n_active_pts;   /* points with at least one observation in the problem         */
  int32_t reserved;
} ba_refine_round;
int ba_refine(ba_problem *p, int32_t n_stages, const ba_refine_stage *stages, int32_t rounds,
              ba_refine_round *hist);
/* n_obs flags in the caller's observation order: 1 = in the problem. */
int ba_get_active(const ba_problem *p, uint8_t *active_out);
/* Batched triangulation from scratch (the triangulation step of Sec. 4.3, one thread
   per point): every point of d from all its observations, with the cameras held at
   d->poses, by BA_TRI_MIDPOINT or BA_TRI_DLT, in FP64.  points_out (3 * n_pts) receives
   the point, or d->points_xyz's value (NaN when that is NULL) where ok_out is 0: fewer
   than two observations, a degenerate system, or a point not in front of every camera
   that observes it.  d->points_xyz may be NULL; the other inputs are validated as by
   ba_create.  device_ms (may be NULL): the kernel's device time. */
int ba_triangulate(const ba_problem_desc *d, int32_t method, void *hip_stream, double *points_out,
                   uint8_t *ok_out, double *device_ms);
/* RANSAC triangulation per track (Sec. 4.3), as ba_triangulate plus outlier rejection:
   hypothesis h = 0 .. n_hyp - 1 of a track of n observations (in the caller's order)
   takes the pair a = h mod n, b = (a + 1 + (h div n) mod (n - 1)) mod n, a fixed schedule
   that lists every ordered pair once within n (n - 1) hypotheses; the two-ray midpoint
   scores the observations in front of their camera with a reprojection error of at most
   tau_px; the first hypothesis with the most inliers wins, and with at least two the
   point is triangulated from them by `method`.  inlier_out: n_obs flags in the caller's
   order (all 0 on a failed track).  BA_EINVAL also for tau_px not positive and finite or
   n_hyp outside 1..4096. */
int ba_triangulate_ransac(const ba_problem_desc *d, int32_t method, double tau_px, int32_t n_hyp, void *hip_stream,
                          double *points_out, uint8_t *ok_out, uint8_t *inlier_out, double *device_ms);
/* Copy the current state and the report of the last solve.  NULL outputs are
   skipped.  poses_out: n_cams entries; points_out: 3 * n_pts doubles. */
int ba_get_result(const ba_problem *p, ba_pose *poses_out, double *points_out, ba_report *rep);
/* Sizes found by the symbolic analysis. */
typedef struct {
  int32_t n_cams, n_free_cams, n_pts, n_obs;
  int64_t n_pairs;        /* observation pairs (k_a, k_b), a < b, both cameras free   */
  int32_t n_up_blocks;    /* upper off-diagonal 6x6 blocks of the reduced system       */
  int32_t nnzb;           /* stored 6x6 blocks of S (both triangles and the diagonal)  */
  int32_t n_free_obs;     /* observations in free cameras                             */
  int32_t precision;
  int32_t schur_form;     /* 1: point chunks staged in LDS, 0: per-block pair lists,
                             2: dense co-visibility form                             */
  int32_t n_chunks;       /* point chunks (chunk form)                                 */
  int64_t n_entries;      /* (chunk, block) partial sums (chunk form)                  */
  int32_t pcg_rows;       /* reduced-system rows per PCG workgroup: 4; for at least
                             1024 free cameras 16, or 32 beyond 8192 free cameras
                             (4 again where a tile's columns would not fit in LDS)     */
  int32_t pcg_resident;   /* 1: BA_FLAG_PCG_RESIDENT was asked for and the problem fits it;
                             2: the same, started as a cooperative launch                  */
} ba_problem_info;
int ba_get_info(const ba_problem *p, ba_problem_info *out);
/* The symbolic analysis of ba_create alone, for planning: validates d and opt as
   ba_create does and fills *info (the sizes ba_get_info would report; pcg_resident is
   1 only where a device is present to check residency) and *bytes (the device bytes
   ba_create would allocate, the server's admission charge).  Uploads nothing and needs
   no device: with none present, the Schur form is chosen as for a gfx950 device.
   info and bytes may be NULL. */
int ba_analyse(const ba_problem_desc *d, const ba_options *opt, ba_problem_info *info, int64_t *bytes);
/* Device bytes held by the problem (the admission byte model of the server). */
int64_t ba_problem_bytes(const ba_problem *p);
void ba_destroy(ba_problem *p);

/* Per-kernel device time of the last solve, summed over the timed launches
   (HIP events recorded on the problem's stream around each timed launch).
   ba_set_profiling(p, mask, stride) selects the kernels (bit i of mask = kernel
   i in the order ba_get_kernel_times reports them; -1 all, 0 off) and times
   every stride-th launch of each (events between launches cost time, so a
   stride keeps the measured solve close to an unmeasured one).  The PCG step
   kernel ("pcg_cg") is timed once per run of launches (one run per LM
   iteration) and reports that run's launch count.  Profiled solves are
   enqueued launch by launch, except when pcg_cg alone is selected: then each
   LM iteration replays three graphs (before, during and after the PCG run)
   with the events between them. */
int ba_set_profiling(ba_problem *p, int32_t mask, int32_t stride);
/* Test hook for the time-out path of BA_FLAG_PCG_RESIDENT: the number of polls of the
   other workgroups' flags after which the resident PCG's grid barrier gives up
   (default 1048576, about a second).  With 0 every barrier gives up at once, so every
   workgroup of the launch exits at its first barrier, the LM iteration rejects its
   step, and the solve ends with status BA_STATUS_PCG_SYNC and iters = that
   iteration's number.  Applies from the next solve on; BA_EINVAL for polls < 0. */
int ba_set_barrier_polls(ba_problem *p, int32_t polls);
/* Test export of one LM iteration's intermediate quantities, for element-wise
   checks of the linearisation, the Schur complement (paper Sec. 4.3; the reduced
   camera system of the method), the PCG solution and the back-substitution.  Runs one
   LM iteration from the current state as a solve with max_iters = 1 would (lambda =
   lambda0), leaves the problem in the state that solve leaves, and copies out, in
   FP64 (values of the compute type widened), into the caller's buffers (NULL skips):
     S_rowptr   n_free_cams + 1    block rows of S (free cameras in the caller's order)
     S_col      nnzb               free-camera column of each stored block
     S          36 nnzb            the damped reduced system S = U* - W V*^-1 W^T,
                                   every stored 6x6 block (both triangles), row-major
     b          6 n_free_cams      right-hand side -g_c + W V*^-1 g_p
     gc         6 n_free_cams      camera gradient J_c^T W r (with the prior terms)
     dc         6 n_free_cams      the PCG solution (the camera step)
     gp         3 n_pts            point gradient, caller's point order
     dp         3 n_pts            the back-substituted point step (trial point minus
                                   point, in FP64)
     r          2 n_obs            sqrt(w) r per observation, caller's order, as stored
                                   for the Schur complement (0 in fixed cameras)
     Jc, Jp     12 n_obs, 6 n_obs  sqrt(w) J_c and sqrt(w) J_p (row-major 2x6, 2x3) as
                                   rebuilt from the stored record (0 in fixed cameras)
   lambda, pcg_iters and accepted report the iteration.  BA_EINVAL for a vehicle-rig
   problem; BA_ESTATE while a solve is in flight. */
typedef struct {
  double lambda;
  int32_t pcg_iters, accepted;
  int32_t *S_rowptr, *S_col;
  double *S, *b, *gc, *dc, *gp, *dp, *r, *Jc, *Jp;
} ba_debug_iteration;
int ba_debug_iteration_export(ba_problem *p, ba_debug_iteration *out);
int ba_get_kernel_times(const ba_problem *p, int32_t max_kernels, const char **names,
                        double *ms, int32_t *launches, int32_t *n_out);

/* ---------------------------------------------------------------- pose graphs
   Pose-graph optimisation (paper Sec. 4.2): nodes are poses, edges carry a measured
   relative pose.  Sequential constraints (Eq. seq), loop-closure constraints and
   extrinsic constraints between the cameras of one rig (Eq. extrinsic) all have the
   error e = T_i T_j^-1 - M_ij over the 3x4 upper parts, and the objective
   sum_e e^T Omega_e e is read with Omega_e diagonal: w_rot on the nine rotation
   entries, w_trans on the three translation entries, with the factor 1/2 of C.
   A node is a camera (camera-frame mode) or a vehicle rig (vehicle-rig mode, where
   the rig's cameras follow from fixed extrinsics and extrinsic edges do not arise);
   the solver does not distinguish them.  The problem runs through the same
   Levenberg-Marquardt iteration, reduced-system assembly and block-Jacobi PCG as
   bundle adjustment, with no points: ba_solve, ba_solve_async / ba_wait, ba_reset,
   ba_get_result (points_out ignored; n_masked and rms_px are 0), ba_get_info,
   profiling and ba_destroy apply; ba_refine does not (BA_EINVAL).
   Options: max_iters, pcg_*, lambda0, precision and flags as for BA; prior_abs > 0
   adds the absolute prior on every node (anchored at the given poses); huber_delta
   must be <= 0 and prior_seq 0.
   BA_EINVAL: fewer than 2 nodes or 1 edge, a node index out of range, an edge from a
   node to itself, two edges between the same two nodes (either direction), a bad
   quaternion (node pose or measurement), weights not finite and >= 0 or both 0,
   every node fixed, or bad options. */
#define BA_EDGE_SEQUENTIAL 0
#define BA_EDGE_LOOP 1
#define BA_EDGE_EXTRINSIC 2
typedef struct {
  int32_t i, j;           /* nodes: the edge measures A_ij = T_i T_j^-1                   */
  int32_t type;           /* BA_EDGE_*: where the measurement came from (not used)        */
  int32_t reserved;
  ba_pose meas;           /* measured A_ij as (quaternion, t) of [R | t]                 */
  double w_rot, w_trans;  /* weights of the rotation and translation entries             */
} ba_pose_edge;
typedef struct {                 /* host memory                                          */
  int32_t n_nodes;
  const ba_pose *poses;          /* n_nodes initial poses (world -> node)               */
  const uint8_t *node_fixed;     /* n_nodes flags (1 = held fixed), or NULL              */
  int64_t n_edges;
  const ba_pose_edge *edges;
} ba_pose_graph_desc;
int ba_pose_graph_create(const ba_pose_graph_desc *g, const ba_options *opt, void *hip_stream,
                         ba_problem **out);

/* ---------------------------------------------------------------- vehicle rigs
   Extrinsic refinement in the vehicle-rig configuration (paper Sec. 4.4): the pose
   of rig camera c at frame f is the composition T_(f,c) = E_c T_v(f) of the camera's
   extrinsic E_c = T_c^v (vehicle -> camera, shared by every frame) and the vehicle pose
   T_v(f) (world -> vehicle), and both are unknowns next to the points.  C gains
     1/2 prior_ext sum_c ||E_c - E_c,init||^2                 (Sec. 4.4 absolute prior)
     1/2 prior_rig sum_pairs ||E_c E_d^-1 - E_c,init E_d,init^-1||^2
   (the rigidity constraint of Eq. extrinsic between rig cameras, which in this
   configuration depends on the extrinsics alone), as 3x4 Frobenius norms.  Updates:
   T_v <- Exp(xi_v) T_v, E_c <- Exp(xi_e) E_c.  The reprojection terms, loss, masking,
   damping schedule and PCG are those of BA; the Marquardt diagonal is that of the rig
   unknowns.  Without prior_ext (or a fixed extrinsic) the rig keeps a gauge: the
   vehicle frame is only defined up to a rigid motion shared by the extrinsics.
   ba_solve, ba_solve_async / ba_wait, ba_reset, ba_get_info, profiling and ba_destroy
   apply; ba_get_result returns the composed camera poses (n_frames * n_rig, camera
   f * n_rig + c), ba_rig_get_result the vehicle poses and extrinsics; ba_refine does
   not apply (BA_EINVAL).
   Options as for BA; prior_abs and prior_seq must be 0 (the rig's priors are given
   here).  BA_EINVAL: n_frames < 1, n_rig outside 1..16, a camera, frame or point index
   out of range, a duplicate (frame, camera, point), a bad quaternion, non-finite data,
   negative or non-finite prior weights, a rigidity pair of one camera with itself or
   given twice, nothing free, or bad options. */
#define BA_RIG_MAX_CAMS 16
typedef struct { int32_t frame, cam, pt, reserved; double u, v; } ba_rig_obs;
typedef struct {                 /* host memory                                           */
  int32_t n_frames, n_rig;
  const ba_intrinsics *K;        /* n_rig, one per rig camera                             */
  const ba_pose *vehicle_poses;  /* n_frames initial world -> vehicle poses               */
  const ba_pose *extrinsics;     /* n_rig initial vehicle -> camera poses (T_c^v)         */
  const uint8_t *vehicle_fixed;  /* n_frames flags, or NULL                               */
  const uint8_t *extrinsic_fixed; /* n_rig flags, or NULL                                  */
  int32_t n_pts;
  const double *points_xyz;      /* 3 * n_pts                                             */
  int64_t n_obs;
  const ba_rig_obs *obs;
  double prior_ext;              /* lambda_e >= 0                                          */
  double prior_rig;              /* lambda_r >= 0                                          */
  int32_t n_rig_pairs;
  const int32_t *rig_pairs;      /* 2 * n_rig_pairs rig camera indices                    */
} ba_rig_desc;
int ba_rig_create(const ba_rig_desc *r, const ba_options *opt, void *hip_stream, ba_problem **out);
/* vehicles_out: n_frames, extrinsics_out: n_rig, points_out: 3 * n_pts; NULL skips. */
int ba_rig_get_result(const ba_problem *p, ba_pose *vehicles_out, ba_pose *extrinsics_out, double *points_out,
                      ba_report *rep);

/* ---------------------------------------------------------------- pose-only */
typedef struct {                 /* one localization request (host memory)             */
  ba_intrinsics K;
  ba_pose pose0;                 /* initial world -> camera pose                       */
  int32_t n;                     /* correspondences, 1 .. BA_POSE_MAX_CORR              */
  const double *X;               /* 3n map points (world)                              */
  const double *uv;              /* 2n pixels                                          */
} ba_pose_request;
#define BA_POSE_MAX_CORR 4096

/* Gauss-Newton on each pose with the map fixed: opt->max_iters iterations of
   delta = -H^-1 g (6x6 FP64 Cholesky), T <- Exp(delta) T, Huber weights from
   opt->huber_delta; no damping.  All requests run in one launch.  status_out[r]
   is 0, or 1 if some iteration met a non-positive-definite H (that update is
   skipped).  cost_out[r] = C at the final pose.  Any output may be NULL. */
int ba_pose_batch(int32_t n_req, const ba_pose_request *reqs, const ba_options *opt,
                  void *hip_stream, ba_pose *poses_out, int32_t *status_out, double *cost_out,
                  double *device_ms);
/* For callers that cannot allocate device memory (serving loops and harnesses that
   forbid hipMalloc): ba_pose_batch with the same requests, options, kernel and
   outputs, but the requests are staged in a fixed device array of
   BA_POSE_NOALLOC_MAX_BYTES that the library holds, on every device it runs on, until
   the process ends.  The call allocates and frees no device memory.  Staging takes
   160 bytes per request and 32 bytes per correspondence (each part rounded up to
   256 bytes); a call that needs more fails with BA_ENOMEM before any device work.
   hip_stream NULL: the current device's null stream.  The call returns once its
   results are on the host.  All calls on one device share its array: calls that
   overlap in time there (from two threads) race and give undefined results. */
#define BA_POSE_NOALLOC_MAX_BYTES 100663296  /* 96 MiB */
int ba_pose_batch_noalloc(int32_t n_req, const ba_pose_request *reqs, const ba_options *opt,
                          void *hip_stream, ba_pose *poses_out, int32_t *status_out, double *cost_out);

/* ---------------------------------------------------------------- serving
   Continuous batching: submitted problems wait in a queue; a scheduler thread
   admits them in submission order while a slot is free and their device bytes fit
   the budget (a later problem that fits may go ahead of one that does not, up to 16
   times, after which admission waits for the one passed over), and
   advances every admitted problem by one LM iteration per batched launch
   sequence; a finished problem retires, frees its bytes and its slot, and the
   next queued one joins the running batch.  Pose-only requests run in batched
   pose launches between LM steps.  All problems of a server use the server's
   precision.  Results do not depend on which other problems share a batch. */
typedef struct {
  double p50_ms, p99_ms;   /* submit -> result-ready latency                            */
  double solves_per_s;     /* completed / (last completion - first submission)           */
  int64_t done, queued, active;
  int64_t bytes_in_use, peak_bytes;
} ba_server_stats_t;

int ba_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int32_t precision,
                     void *hip_stream, ba_server **out);
/* Check the sizes and options, copy the problem and queue it; its symbolic analysis
   runs on the server's own threads, so the call returns after the copy.  BA_ENOMEM
   here when the problem's observation, point and camera arrays alone exceed the
   budget.  A problem whose content is invalid (as ba_create rejects it) or whose
   analysed device bytes exceed the budget fails its ticket: ba_server_wait returns
   BA_EINVAL or BA_ENOMEM.  *ticket identifies it in ba_server_wait. */
int ba_server_submit(ba_server *s, const ba_problem_desc *d, const ba_options *opt,
                     int64_t *ticket);
int ba_server_submit_pose(ba_server *s, const ba_pose_request *req, const ba_options *opt,
                          int64_t *ticket);
/* Block until the ticket finishes and copy its result (each ticket once).
   For pose tickets, points_out is ignored and rep->iters/status/cost are set. */
int ba_server_wait(ba_server *s, int64_t ticket, ba_pose *poses_out, double *points_out,
                   ba_report *rep);
int ba_server_stats(ba_server *s, ba_server_stats_t *out);
/* Cancel queued requests, finish active ones, free everything. */
void ba_server_destroy(ba_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BA_MI355X_H */
