// Internal layout shared by the host runtime and the gfx950 kernels.
//
// One problem lives in one device allocation.  Kernels never see a problem
// directly: they receive a table of ProbDev descriptors and a list of tiles
// (problem index, tile index), so one launch advances any mix of problems by
// the same stage of the Levenberg-Marquardt iteration.  A single solve is the
// batch of one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bax {

constexpr int kPtTile = 256;     // points per point-major tile (one workgroup), at most
constexpr int kPtTileLong = 32;  // ... for problems whose points have long tracks
constexpr int kPtTileFill = 2048;  // fewer full tiles than this (8 per CU): half-size tiles
constexpr int kObsChunk = 256;   // observations processed per pass inside a point tile (one per thread)
constexpr int kPcgRows = 4;      // reduced-camera-system rows per PCG tile, dense rows
constexpr int kPcgRowsSparse = 16;  // rows per PCG tile when rows hold few blocks
constexpr int kPcgRowsMax = 32;     // ... and when there are more than 512 such tiles
constexpr int kRigSeg = 32;         // contributions per segment of a rig block's list
constexpr int kCamTile = 256;    // cameras per camera-update tile
constexpr int kOffWaves = 4;     // upper S blocks per off-diagonal workgroup (one wave each)
constexpr int kPoseThreads = 256;
// Point-chunk Schur form: a chunk is at most kChPts points (F64: half) whose free
// observations (at most chunk_obs_cap) are staged in LDS by one workgroup of
// kChThreads threads (F64: half).
constexpr int kChPts = 256;
constexpr int kChThreads = 1024;
constexpr int kChSubItems = 32;  // items per chunk entry (one thread each)
constexpr int kEntSlice = 64;    // chunk entries whose items are interleaved (one wavefront's)
inline int chunk_obs_cap(int precision) { return precision == 0 ? 1024 : precision == 1 ? 1984 : 1600; }
inline int chunk_pts_cap(int precision) { return precision == 0 ? kChPts / 2 : kChPts; }
inline int chunk_cam_cap(int precision) { return precision == 0 ? 128 : 256; }
// LDS bytes of one chunk workgroup: per observation two rows of 8 T (f[7], e[0];
// Q[6], Q g_p[2]) and e[1] -- or, with 16-bit storage, the FP32 gradient
// contribution (6 T) in place of e; per point V*^-1 (6 T); per camera R (9 T)
// and its index.
inline size_t chunk_lds_bytes(int precision) {
  const size_t T = precision == 0 ? 8 : 4;
  const size_t per_obs = precision >= 2 ? 22 * T : 17 * T;
  return (size_t)chunk_obs_cap(precision) * per_obs + (size_t)chunk_pts_cap(precision) * 6 * T +
         (size_t)chunk_cam_cap(precision) * (9 * T + 4);
}

// Dense co-visibility Schur form: cameras in tiles of kDnCams (kDnRows rows of S);
// one workgroup per (tile pair, point range) accumulates Z_a Z_b^T over its points,
// where the 6x3 block Z_aj = W_aj L_j^-T (V*_j = L_j L_j^T) exists for each
// observation, so that sum_j Z_aj Z_bj^T = sum_j W_aj V*_j^-1 W_bj^T.
constexpr int kDnCams = 16;
constexpr int kDnRows = 6 * kDnCams;
constexpr int kDnMaxCams = 1024;     // free cameras beyond which the dense form is not used
constexpr int kDnTargetWgs = 256;   // workgroups per problem the point ranges aim at
constexpr int kDnRangePts = 2048;   // points per range at most

constexpr double kLambdaMin = 1e-12;
constexpr double kLambdaMax = 1e16;
constexpr double kDMin = 1e-6;
constexpr double kDMax = 1e32;
constexpr double kAcceptRho = 1e-3;
constexpr double kZMin = 1e-6;

struct Tile {
  int32_t prob;
  int32_t idx;
};

// Per-problem Levenberg-Marquardt scalars, resident on the device.
struct LMState {
  double lambda, nu;
  double cost;        // cost of the accepted state
  double cost0;
  double trial_cost, dL, rho;
  double lambda0, pcg_tol, huber_delta;
  double pcg_bb, pcg_rz0;  // ||b||^2 and r0.z0 of the current linear solve
  double cg_alpha[2], cg_gamma[2];  // alpha_i, gamma_i of the one-reduction form, by parity
  double sq_sum;           // sum ||r||^2 at the final state (evaluation kernel)
  int32_t iter, max_iters, relin, status;
  int32_t accepted, cur, pcg_done, pcg_iters;
  int32_t pcg_max, init_done, n_masked;
  int32_t pcg_fault;       // 1: the resident PCG's grid barrier timed out (the solve stops)
  int32_t halted;          // 1: the solve ended before max_iters (after a barrier time-out)
  int32_t bar_polls;       // polls after which the resident PCG's grid barrier gives up
};
// Default of LMState::bar_polls: about a second of polling.
constexpr int32_t kBarPollsDefault = 1 << 20;

// Device view of one problem.  Arrays typed T hold the compute type of the
// precision mode (double or float); S is the Jacobian storage type.
struct ProbDev {
  int32_t C, Cf, P, N;
  int32_t Nf;            // observations in free cameras
  int32_t n_up;          // upper off-diagonal blocks of S
  int32_t nnzb;          // blocks of S stored (both triangles + diagonal)
  int32_t n_pt_tiles, n_pcg_tiles, n_cam_tiles;
  int32_t max_tcols;     // longest tile column list
  int32_t pcg_rows;      // rows per PCG tile: kPcgRows, kPcgRowsSparse or kPcgRowsMax
  int32_t pcg_resident;  // 1: the whole PCG runs in one launch with grid barriers (k_cg_run); 2: launched cooperatively
  int32_t chunked;       // 1: point-chunk Schur form, 0: pair-list form
  int32_t n_ch;          // point chunks (chunk form)
  int32_t n_red_tiles;   // reduction tiles (chunk form): four upper blocks each
  int32_t n_fin_tiles;   // camera-row tiles (chunk form): one camera each
  int32_t n_fsh_tiles;   // camera-finish tiles (chunk and dense forms): 64 cameras each
  int32_t pt_tile;       // points per point tile: kPtTile, or kPtTileLong for long tracks
  int32_t dense;         // 1: dense co-visibility Schur form
  int32_t dn_tiles;      // camera tiles (kDnCams free cameras each)
  int32_t dn_pairs;      // tile pairs (a <= b)
  int32_t dn_split;      // point ranges per tile pair
  const int32_t *dn_ts;  // [P][dn_tiles + 1] first record of each point in each camera tile
  const int32_t *dn_rcam;  // [Nf] free camera of each record
  const int2 *dn_crec;     // [Nf] (record, point) of each camera-major observation
  const uint16_t *dn_mask; // [P][dn_tiles] bit c: camera c of the tile observes the point
  void *dn_pfac;         // [P][9] T: L^-T (upper: 00 01 02 11 12 22) and h = L^-1 g_p of V*_j = L L^T
  void *dn_part;         // [dn_pairs][dn_split][kDnRows^2] T: Z Z^T over one point range
  // static structure
  const void *K;                  // [C][4] T: fx, fy, cx, cy
  const int32_t *free_idx;        // [C] free-camera index or -1
  const int32_t *free_cam;        // [Cf] camera of each free index
  const int32_t *obs_cam;         // [N] observations in (point, camera) order
  const int32_t *obs_pt;          // [N]
  const void *obs_uv;             // [N][2] T
  const int32_t *pt_start;        // [P + 1]
  const int32_t *obs_rpos;        // [N] record of each observation, -1 if its camera is fixed
  uint8_t *obs_act;               // [N] 1: in the problem; 0: removed by culling (contributes
                                  // nothing and is not counted as masked)
  // pair-list form: records are camera-major
  const int32_t *cam_obs;         // [Nf] observation of each camera-major record
  const int32_t *cam_obs_start;   // [Cf + 1] records of each free camera
  const int32_t *up_pair_start;   // [n_up + 1]
  const int2 *pairs;              // (c_a, c_b): records of one point in cameras a < b
  // point-chunk form: records are point-major; a chunk's entries are runs of at
  // most kChSubItems items of one S block (diagonal: local observation; upper:
  // local observation pair p | q << 16), diagonal entries first
  const int32_t *ch_pt;           // [n_ch + 1] point range of each chunk
  const int32_t *ch_f0;           // [n_ch + 1] record range of each chunk
  const int32_t *ch_ent;          // [n_ch + 1] entry range of each chunk
  const int32_t *ch_cam_start;    // [n_ch + 1] range in ch_cam
  const int32_t *ch_cam;          // cameras (caller's index) of each chunk's entries
  const int32_t *ent_tgt;         // target block: a < Cf diagonal of camera a, Cf + u upper block u
  const int32_t *ent_cam;         // chunk-local camera whose rotation the entry needs
  const int32_t *ent_slot;        // position of the entry's partial in part_d / part_o (its
                                  // position in its block's list, upper blocks counted from 0)
  const int32_t *ent_start;       // [n_ent] first item; item h of the entry at ent_start + h * kEntSlice
  const uint8_t *ent_len;         // [n_ent] items
  const uint32_t *ent_items;      // per chunk, slices of kEntSlice entries: [slice][h][entry of the slice]
  const int32_t *blk_start;       // [Cf + n_up + 1] entries of each block, in chunk order
  int32_t n_dent;                 // diagonal entries (part_d rows)
  const int32_t *up_pos;          // [n_up] block (a, b) in S
  const int32_t *up_tpos;         // [n_up] block (b, a) in S
  const int32_t *diag_pos;        // [Cf]
  const int32_t *S_rowptr;        // [Cf + 1]
  const int32_t *S_col;           // [nnzb]
  const int32_t *tcol;            // [n_pcg_tiles][max_tcols] distinct columns read by each PCG tile, -1 padded
  const int32_t *S_lcol;          // [nnzb] position of each block's column in its tile's list
  // state, double-buffered (LMState::cur selects the accepted copy)
  double *pose[2];                // [C][12]: R row-major, then t
  double *X[2];                   // [P][3]
  // linearisation and Schur complement
  void *lin;                      // [Nf] LinRec<T, S>
  void *part_d;                   // [diagonal entries][54] T: U, Y W^T (upper 21 each), g_c, Y g_p
  void *part_o;                   // [upper entries][36] T: sum Y W^T of the entry
  double *row_tot;                // [Cf][54] camera-row sums of the diagonal partials
  // relative-pose terms (FP64): the absolute prior's weight, the pairs (i, j) with
  // their measured A_ij = T_i T_j^-1 and rotation / translation weights (sequential
  // priors or pose-graph edges), per-camera U (21) and g (6) contributions, per-pair
  // off-diagonal blocks J_i^T W J_j oriented as the upper block of S
  double prior_abs;
  int32_t prior_on, n_pp, n_pri_tiles, pad1;
  double *part_prior;             // [2][n_pri_tiles] prior cost at the current and trial poses
  const double *pose0;            // [C][12] the initial poses (prior anchors)
  const int2 *pp_cam;             // [n_pp] (i, j), caller's camera indices, i != j
  const double *pp_meas;          // [n_pp][12] measured A_ij, R row-major then t
  const double *pp_w;             // [n_pp][2] weights of the 9 rotation and 3 translation entries
  const int32_t *pp_up;           // [n_pp] upper block of (free i, free j), or -1
  const int32_t *cam_pp_start;    // [Cf + 1]
  const int32_t *cam_pp;          // pairs of each free camera, ascending
  double *prior_diag;             // [Cf][27]
  double *prior_off;              // [n_pp][36]
  int32_t prior_abs_from;         // the absolute prior covers nodes [prior_abs_from, prior_nodes)
  int32_t prior_nodes;
  // vehicle-rig problems: rig_mode 1 is the view over composed cameras (f, c), camera
  // f * n_rigcam + c, whose S blocks are formed undamped; rig_mode 2 is the view over the
  // rig unknowns (vehicle poses, then extrinsics), whose reduced system the PCG solves
  int32_t rig_mode, n_frames, n_rigcam, pad2;
  double *Ucam;                   // (1) [C][21] undamped U of each composed camera
  double *rig_pose[2];            // (1) [n_frames + n_rigcam][12] rig poses (the rig view's pose)
  const void *rig_x, *rig_gc, *rig_Dc;  // (1) the rig view's x, g and D
  const int32_t *rig_free_idx;    // (1) rig node -> free rig block
  const int32_t *rb_start;        // (2) [nnzb + 1] contributions of camera S blocks to each rig block
  const int32_t *rb_pos;          // (2) camera S block of each contribution
  const int32_t *rb_lr;           // (2) (left rig camera + 1) | (right rig camera + 1) << 16; 0: identity
  const int32_t *rb_diag;         // (2) [nnzb] row of a diagonal rig block, -1 for the others
  const int32_t *rs_blk;          // (2) [nnzb + 1] segments of each rig block's contribution list
  const int32_t *rs_c0;           // (2) [n_seg + 1] first contribution of each segment (<= kRigSeg each)
  double *rpart;                  // (2) [n_seg][36] segment sums
  int32_t n_rig_seg, pad3;
  double *rdiag;                  // (2) [Cf][36] undamped diagonal rig blocks
  const int32_t *rr_start;        // (2) [Cf + 1] composed cameras of each rig row
  const int32_t *rr_cam;
  const void *cam_S, *cam_gc, *cam_brhs;  // (2) the camera view's S, g and b
  const double *cam_U;            // (2) the camera view's Ucam
  void *Q;                        // [Nf][6] T: J_p,k V*_j^-1 (2x3), camera-major
  void *V, *gp, *Dp, *Vinv;       // [P][6], [P][3], [P][3], [P][6] T
  void *gc, *Dc, *brhs;           // [Cf][6] T
  void *S;                        // [nnzb][36] T
  double *Minv;                   // [Cf][36]
  void *x, *r, *z, *p0, *p1, *q;  // [6 Cf] T
  // one-reduction PCG form: u = M^-1 r, w = S u, s = S p; two buffers each (parity)
  void *cg_r[2], *cg_u[2], *cg_w[2], *cg_s[2];
  // reductions (one partial per tile, summed in a fixed order)
  double *part_lin_cost;          // [n_pt_tiles]
  int32_t *part_masked;           // [n_pt_tiles]
  double *part_sq;                // [n_pt_tiles]
  double *part_trial_cost;        // [n_pt_tiles]
  int32_t *part_trial_masked;     // [n_pt_tiles]
  double *part_dl_pt;             // [n_pt_tiles]
  double *part_dl_cam;            // [n_cam_tiles]
  double *part_rz0;               // [Cf]
  double *part_bb;                // [Cf]
  double *part_rz[2];             // [n_pcg_tiles]
  double *part_pq;                // [n_pcg_tiles]
  double *part_cg[2];             // [3][n_pcg_tiles] r.u, w.u, r.r partials by parity
  uint32_t *cg_flag;              // [n_pcg_tiles] resident PCG: iterations each tile has finished
  double *part_rr;                // [n_pcg_tiles]
  int32_t *part_cull;             // [n_pt_tiles][2] active observations, points with one, after culling
  LMState *st;
  double *iter_cost;              // [max_iters + 1]
  int32_t *iter_pcg;              // [max_iters]
};

// Tile lists of one batch (device pointers) and their lengths.
struct BatchPlan {
  const ProbDev *probs;
  const Tile *pt, *diag, *off, *pcg, *cam, *ctl, *pp, *ch, *red, *fin, *fsh, *pri;
  int32_t n_pt, n_diag, n_off, n_pcg, n_cam, n_ctl, n_pp, n_ch, n_red, n_fin, n_fsh, n_pri;
  // dense form: point tiles (prep), free cameras (camera sums), (tile pair, range)
  // workgroups (Z Z^T) and tile pairs (reduction)
  const Tile *dpt, *dcm, *dsy, *dre;
  int32_t n_dpt, n_dcm, n_dsy, n_dre;
  int32_t n_probs;
  int32_t pcg_rows;  // rows per PCG tile shared by every problem of the batch, 0 if mixed
  ProbDev single;  // host copy of the descriptor when n_probs == 1 (passed by value to short kernels)
};

// One localization request on the device.
struct PoseDev {
  double K[4];
  double pose[12];     // in: initial pose; out: refined pose
  int64_t off;         // first correspondence
  int32_t n;
  int32_t status;
  double cost;
  double delta;        // the request's Huber threshold (<= 0: none)
  int32_t iters;       // the request's Gauss-Newton iterations
  int32_t reserved;
};

// Kernel timing hook: the host records events around launches when set.
// begin/end bracket `launches` consecutive launches of one kernel.
struct KernelTimer {
  virtual void begin(int kernel_id, hipStream_t s, int launches) = 0;
  virtual void end(int kernel_id, hipStream_t s) = 0;
  virtual ~KernelTimer() {}
};

enum KernelId {
  K_LINEARIZE = 0, K_POINT_PREP, K_SCHUR_DIAG, K_SCHUR_OFF, K_PCG_SPMV, K_PCG_UPDATE,
  K_CAM_UPDATE, K_POINT_TRIAL, K_LM_CONTROL, K_EVAL, K_POSE_GN, K_PCG_CG, K_SCHUR_CHUNK,
  K_SCHUR_REDUCE, K_SCHUR_ROWS, K_SCHUR_FINISH, K_PRIOR_LIN, K_PRIOR_APPLY, K_CULL, K_RIG_BLOCKS,
  K_RIG_ROWS, K_RIG_UPDATE, K_PRIOR_COST, K_DENSE_PREP, K_DENSE_CAMS, K_DENSE_SCHUR, K_DENSE_REDUCE,
  K_NUM_KERNELS
};
extern const char *const kKernelNames[K_NUM_KERNELS];

// Size in bytes of one stored linearisation record for a precision mode.
size_t lin_record_bytes(int precision);
// Size of the compute type (8 or 4).
size_t compute_bytes(int precision);

// Query device limits that select kernel forms; call before any graph capture.
int prepare_kernels();
// Dynamic LDS a workgroup may use on the current device (bytes); a gfx950's when no
// device is present.
size_t device_lds_limit();
// Whether the dense co-visibility form can run on the current device (on a gfx950 when
// no device is present).
bool dense_form_available();
// Whether the PCG runs in its one-reduction form (one launch per iteration) for
// a plan whose longest tile column list is max_tcols.
bool one_reduction_pcg(int precision, int max_tcols);
// True when the resident PCG (one launch, grid barriers) can run a problem: every
// tile's columns fit one sweep and all n_tiles workgroups can be resident at once.
bool resident_pcg_fits(int precision, int rows, int n_tiles, int max_tcols);
// Parts of one LM iteration: everything, or the launches before the PCG run, the
// PCG run itself, and the launches after it (so the run can be timed between graphs).
enum LmPart { LM_ALL = 0, LM_BEFORE_PCG, LM_PCG, LM_AFTER_PCG };
// Launch one Levenberg-Marquardt iteration (or a part of it) for every problem of
// the plan.  max_tcols: the longest PCG-tile column list of the plan (selects the PCG form).
hipError_t launch_lm_iteration(int precision, const BatchPlan &bp, int pcg_max, int max_tcols,
                               hipStream_t s, KernelTimer *timer, int part = LM_ALL);
// One LM iteration of a vehicle-rig problem: the camera plan holds the composed-camera
// view, the rig plan the rig view (its PCG tiles, prior tiles, rig-block tiles in .red,
// rig-row tiles in .fin, finish tiles in .fsh).
hipError_t launch_rig_iteration(int precision, const BatchPlan &cam, const BatchPlan &rig, int pcg_max,
                                int max_tcols, hipStream_t s, KernelTimer *timer);
// Evaluate sum ||r||^2 and the masked count at the accepted state.
hipError_t launch_eval(int precision, const BatchPlan &bp, hipStream_t s, KernelTimer *timer);
// Restores pose[0], X[0] from their initial copies and sets every observation active
// (act: a 256-byte-aligned device array of n_act bytes).
hipError_t launch_reset(double *pose, const double *pose_init, size_t n_pose, double *X, const double *X_init,
                        size_t n_X, uint8_t *act, size_t n_act, hipStream_t s);
// Culling and re-triangulation at the accepted state: observations with
// ||r||^2 > tau2 (or depth <= the threshold) leave the problem; points that lost
// one are re-triangulated (midpoint) from the rest, or leave if that fails.
hipError_t launch_cull(int precision, const BatchPlan &bp, double tau2, int method, hipStream_t s,
                       KernelTimer *timer);
// Triangulation from scratch (method 0 midpoint, 1 DLT), one thread per point.
hipError_t launch_triangulate(int n_pts, const int32_t *pt_start, const int32_t *cam, const double *xy,
                              const double *poses, int method, double *X, uint8_t *ok, hipStream_t s);
// RANSAC triangulation per track: pair hypotheses, inliers by reprojection threshold.
hipError_t launch_triangulate_ransac(int n_pts, const int32_t *pt_start, const int32_t *cam, const double *xy,
                                     const double *poses, const double *Kc, double tau2, int n_hyp, int method,
                                     double *X, uint8_t *ok, uint8_t *inl, hipStream_t s);
// Test export: sqrt(w) r (2), sqrt(w) J_c (12) and sqrt(w) J_p (6) of every observation
// in internal order, in FP64, from the stored records formed at state `cur`.
hipError_t launch_export_records(int precision, const ProbDev &pd, int cur, double *r, double *Jc, double *Jp,
                                 hipStream_t s);
// Pose-only Gauss-Newton, one workgroup per request.
// Each request carries its own iteration count and Huber threshold.
hipError_t launch_pose_gn(int n_req, PoseDev *reqs, const double *X, const float *uv, hipStream_t s,
                          KernelTimer *timer);

}  // namespace bax
