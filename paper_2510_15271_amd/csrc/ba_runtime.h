// Host-side runtime structures of the bundle-adjustment library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"

namespace bax {

extern thread_local std::string g_last_error;
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_pose(const ba_pose &p, const char *what, int64_t i);
int check_options(const ba_options *o, bool pose_only);
void quat_to_pose12(const ba_pose &p, double out[12]);
void relative_pose12(const double Ti[12], const double Tj[12], double A[12]);
ba_pose pose12_to_quat(const double M[12]);

// Result of the symbolic analysis of one problem (host arrays).
struct Symbolic {
  int32_t C = 0, Cf = 0, P = 0, N = 0;
  int32_t n_up = 0, nnzb = 0;
  std::vector<int32_t> free_idx, free_cam;
  std::vector<int32_t> obs_cam, obs_pt;
  std::vector<double> obs_uv;
  std::vector<int32_t> pt_start;
  std::vector<int32_t> pt_order;  // internal point -> caller's point index
  std::vector<int32_t> obs_rpos;  // record of each observation (-1: fixed camera)
  std::vector<int32_t> obs_order; // internal observation -> caller's observation index
  int32_t Nf = 0;                 // observations in free cameras (records)
  int64_t n_pairs = 0;            // observation pairs of one point in two free cameras
  bool chunked = false;           // point-chunk Schur form (else pair lists or dense)
  bool dense = false;             // dense co-visibility Schur form
  int32_t pt_tile = kPtTile;      // points per point tile (kPtTileLong for long tracks)
  int32_t dn_tiles = 0, dn_split = 0;
  std::vector<int32_t> dn_ts;     // [P][dn_tiles + 1] (dense form)
  std::vector<int32_t> dn_rcam;   // [Nf] (dense form)
  std::vector<int2> dn_crec;      // [Nf] (dense form) record and point of each camera-major observation
  std::vector<uint16_t> dn_mask;  // [P][dn_tiles] (dense form)
  // pair-list form
  std::vector<int32_t> cam_obs, cam_obs_start;
  std::vector<int32_t> up_pair_start;
  std::vector<int2> pairs;
  // point-chunk form (see ProbDev)
  std::vector<int32_t> ch_pt, ch_f0, ch_ent, ch_cam_start, ch_cam;
  std::vector<int32_t> ent_tgt, ent_cam, ent_slot, ent_start;
  std::vector<uint32_t> ent_items;
  std::vector<uint8_t> ent_len;
  std::vector<int32_t> blk_start;
  int32_t n_dent = 0, n_oent = 0;
  // relative-pose pairs (caller's camera indices): sequential prior pairs or pose-graph
  // edges, their measured A_ij (12 each) and weights (rotation, translation), their upper
  // block (both cameras free) or -1, and the pairs of each free camera
  double prior_abs = 0.0;
  std::vector<int2> pp_cam;
  std::vector<double> pp_meas, pp_w;
  std::vector<int32_t> pp_up, cam_pp_start, cam_pp;
  std::vector<int32_t> up_pos, up_tpos, diag_pos, S_rowptr, S_col;
  // distinct columns read by each PCG tile (kPcgRows rows) and, per block, the
  // position of its column in its tile's list
  std::vector<int32_t> tcol, S_lcol;
  int32_t max_tcols = 0;
  int32_t pcg_rows = kPcgRows;    // rows per PCG tile
  bool pcg_resident = false;      // the whole PCG in one launch (BA_FLAG_PCG_RESIDENT, when it fits)
  bool pcg_coop = false;          // ... started as a cooperative launch (BA_FLAG_PCG_COOPERATIVE)
};
// Edges of a pose graph: node pairs (i, j), measured A_ij (12 values each, R row-major
// then t) and weights (rotation, translation).
struct GraphEdges {
  std::vector<int2> pairs;
  std::vector<double> meas, w;
  std::vector<int2> pattern;  // node pairs whose block of S exists without a term of their own
};
// Symbolic analysis of a problem.  With edges, the description holds the nodes only
// (no points or observations) and the edges replace the sequential prior pairs.
// allow_dense: the dense co-visibility form may be chosen (not for the cameras of a rig).
int analyse(const ba_problem_desc *d, const ba_options *opt, Symbolic &sy, const GraphEdges *edges = nullptr,
            bool allow_dense = true);

struct Offsets {
  size_t st, K, free_idx, free_cam, obs_cam, obs_pt, obs_uv, pt_start, cam_obs, cam_obs_start, obs_rpos, obs_act;
  size_t up_pair_start, pairs, up_pos, up_tpos, diag_pos, S_rowptr, S_col, tcol, S_lcol;
  size_t ch_pt, ch_f0, ch_ent, ch_cam_start, ch_cam, ent_tgt, ent_cam, ent_slot, ent_start, ent_len, ent_items, blk_start;
  size_t part_d, part_o, row_tot, dn_ts, dn_rcam, dn_crec, dn_mask, dn_pfac, dn_part;
  size_t pp_cam, pp_meas, pp_w, pp_up, cam_pp_start, cam_pp, prior_diag, prior_off;
  size_t pose[2], X[2], pose_init, X_init, lin, Q, V, gp, Dp, Vinv, gc, Dc, brhs, S, Minv, vec[14];
  size_t part_lin_cost, part_masked, part_sq, part_trial_cost, part_trial_masked, part_dl_pt, part_dl_cam;
  size_t part_rz0, part_bb, part_rz[2], part_pq, part_rr, part_cg[2], cg_flag, part_prior, part_cull, iter_cost, iter_pcg;
  size_t total;
};

// One problem placed in a device block: its descriptor and host-side scalars.
struct DevProblem {
  int precision = BA_PREC_F32, max_iters = 0, pcg_max = 0;
  int32_t bar_polls = kBarPollsDefault;  // grid-barrier poll bound of the resident PCG
  double lambda0 = 1e-4, pcg_tol = 1e-6, huber = 0.0;
  int32_t C = 0, Cf = 0, P = 0, N = 0;
  int32_t max_tcols = 0;
  std::vector<int32_t> pt_order;  // internal point -> caller's point index
  std::vector<int32_t> obs_order; // internal observation -> caller's observation index
  int64_t n_active = 0;           // observations in the problem (after the last culling)
  Offsets off{};
  char *dev = nullptr;
  ProbDev view{};
  LMState host_state{};     // state read back after the last solve
  LMState pending_state{};  // state uploaded for the solve in flight
  std::vector<std::vector<float>> staging_f;
  std::vector<std::vector<double>> staging_d;

  static size_t plan(const Symbolic &sy, int precision, int max_iters, Offsets &o);
  static size_t bytes_for(const Symbolic &sy, int precision, int max_iters);
  int init(const Symbolic &sy, const ba_problem_desc *d, const ba_options *opt, char *base,
           hipStream_t s);
  LMState fresh_state() const;
  // rep_pin: the solve's report block staged by enqueue_report (already landed), or
  // nullptr to read the report from the device
  int read_result(hipStream_t s, ba_pose *poses_out, double *points_out, ba_report *rep,
                  bool solved, double solve_ms, double setup_ms, const char *rep_pin = nullptr);
  // The report of a solve without host round trips: enqueue_report queues on stream s
  // the copies of the state, the evaluation partials and the per-iteration arrays into
  // `pinned`, a page-locked buffer of report_bytes() (its first LMState is the upload
  // slot of the next solve's fresh state, see report_upload).
  size_t report_bytes() const;
  hipError_t enqueue_report(hipStream_t s, char *pinned) const;
  static size_t report_state_offset();
  // The same result without a host wait: enqueue_result queues on stream s the copies
  // of everything the report needs (the state, both pose and point buffers, the
  // evaluation partials and the per-iteration arrays) into `pinned`, a page-locked
  // buffer of result_bytes(); once they have landed, finish_result builds the outputs
  // from it alone.
  size_t result_bytes() const;
  hipError_t enqueue_result(hipStream_t s, char *pinned) const;
  void finish_result(const char *pinned, ba_pose *poses_out, double *points_out, ba_report *rep) const;
};

// Tile lists of a set of problems, mirrored on the device.
struct Batch {
  std::vector<ProbDev> probs;
  std::vector<int> tags;
  std::vector<Tile> tiles[16];  // pt, diag, off, pcg, cam, ctl, pp, ch, red, fin, fsh, pri, dpt, dcm, dsy, dre
  std::vector<char> host;
  void *dev = nullptr;
  size_t cap = 0;
  BatchPlan plan{};
  void clear();
  void add(const ProbDev &pd, int slot_tag);
  int upload(hipStream_t s);
  ~Batch();
};

// Per-kernel device time from pairs of HIP events around each launch.
struct EventTimer : KernelTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> ids, counts;
  size_t used = 0;
  uint32_t mask = 0xffffffffu;  // kernels to time (bit = KernelId)
  int32_t stride = 1;            // time every stride-th launch of each selected kernel
  int32_t seen[K_NUM_KERNELS] = {};
  bool active = false;
  void begin(int id, hipStream_t s, int launches) override;
  void end(int id, hipStream_t s) override;
  void reset();
  void reserve(size_t pairs);
  void collect(double ms[K_NUM_KERNELS], int32_t launches[K_NUM_KERNELS]);
  ~EventTimer() override;
};

// Pose-only requests packed for one launch.
struct PoseBatch {
  int n = 0;
  int64_t n_corr = 0;
  std::vector<PoseDev> hdr;
  std::vector<double> X;
  std::vector<float> uv;
  // opts[i]: the options of request i (its max_iters and huber_delta)
  int pack(const std::vector<const ba_pose_request *> &reqs, const std::vector<const ba_options *> &opts);
  size_t bytes() const;
  // Upload, launch and queue the download of the headers into hdr (caller syncs).
  int run(char *base, hipStream_t s, KernelTimer *tm);
};
int check_pose_request(const ba_pose_request &r, int64_t i);

}  // namespace bax
