// Host runtime of the bundle-adjustment library: validation, symbolic
// analysis, device layout, the Levenberg-Marquardt driver and the C-ABI.
//
// The symbolic analysis (done once per problem) orders observations by
// (point, camera), groups the observations of every free camera, and builds
// the block sparsity of the reduced camera system S together with, for every
// upper off-diagonal block (a, b), the list of observation pairs (k_a, k_b) of
// the points seen by both cameras.  The device then forms S block by block
// from those lists without atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_runtime.h"

namespace bax {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? BA_ENOMEM : BA_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

// ------------------------------------------------------------------ pose conversions
void quat_to_pose12(const ba_pose &p, double out[12]) {
  const double n = std::sqrt(p.qw * p.qw + p.qx * p.qx + p.qy * p.qy + p.qz * p.qz);
  const double w = p.qw / n, x = p.qx / n, y = p.qy / n, z = p.qz / n;
  out[0] = 1 - 2 * (y * y + z * z);
  out[1] = 2 * (x * y - w * z);
  out[2] = 2 * (x * z + w * y);
  out[3] = 2 * (x * y + w * z);
  out[4] = 1 - 2 * (x * x + z * z);
  out[5] = 2 * (y * z - w * x);
  out[6] = 2 * (x * z - w * y);
  out[7] = 2 * (y * z + w * x);
  out[8] = 1 - 2 * (x * x + y * y);
  out[9] = p.tx;
  out[10] = p.ty;
  out[11] = p.tz;
}

// A = T_i T_j^-1 = [R_i R_j^T | t_i - R_i R_j^T t_j] for poses held as 12 values.
void relative_pose12(const double Ti[12], const double Tj[12], double A[12]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      A[3 * a + b] = Ti[3 * a] * Tj[3 * b] + Ti[3 * a + 1] * Tj[3 * b + 1] + Ti[3 * a + 2] * Tj[3 * b + 2];
  for (int r = 0; r < 3; ++r)
    A[9 + r] = Ti[9 + r] - (A[3 * r] * Tj[9] + A[3 * r + 1] * Tj[10] + A[3 * r + 2] * Tj[11]);
}

// Rotation matrix -> unit quaternion with qw >= 0 (Shepperd's method: branch on
// the largest of the trace and the diagonal entries).
ba_pose pose12_to_quat(const double M[12]) {
  const double m00 = M[0], m01 = M[1], m02 = M[2], m10 = M[3], m11 = M[4], m12 = M[5];
  const double m20 = M[6], m21 = M[7], m22 = M[8];
  const double tr = m00 + m11 + m22;
  double q[4];
  if (tr >= m00 && tr >= m11 && tr >= m22) {
    const double s = std::sqrt(1.0 + tr) * 2;
    q[0] = 0.25 * s; q[1] = (m21 - m12) / s; q[2] = (m02 - m20) / s; q[3] = (m10 - m01) / s;
  } else if (m00 >= m11 && m00 >= m22) {
    const double s = std::sqrt(1.0 + m00 - m11 - m22) * 2;
    q[0] = (m21 - m12) / s; q[1] = 0.25 * s; q[2] = (m01 + m10) / s; q[3] = (m02 + m20) / s;
  } else if (m11 >= m22) {
    const double s = std::sqrt(1.0 + m11 - m00 - m22) * 2;
    q[0] = (m02 - m20) / s; q[1] = (m01 + m10) / s; q[2] = 0.25 * s; q[3] = (m12 + m21) / s;
  } else {
    const double s = std::sqrt(1.0 + m22 - m00 - m11) * 2;
    q[0] = (m10 - m01) / s; q[1] = (m02 + m20) / s; q[2] = (m12 + m21) / s; q[3] = 0.25 * s;
  }
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double sg = q[0] < 0 ? -1.0 : 1.0;
  ba_pose p;
  p.qw = sg * q[0] / n; p.qx = sg * q[1] / n; p.qy = sg * q[2] / n; p.qz = sg * q[3] / n;
  p.tx = M[9]; p.ty = M[10]; p.tz = M[11];
  return p;
}

static bool finite_pose(const ba_pose &p) {
  return std::isfinite(p.qw) && std::isfinite(p.qx) && std::isfinite(p.qy) && std::isfinite(p.qz) &&
         std::isfinite(p.tx) && std::isfinite(p.ty) && std::isfinite(p.tz);
}

int check_pose(const ba_pose &p, const char *what, int64_t i) {
  if (!finite_pose(p)) return fail(BA_EINVAL, "%s %lld: non-finite pose", what, (long long)i);
  const double n = std::sqrt(p.qw * p.qw + p.qx * p.qx + p.qy * p.qy + p.qz * p.qz);
  if (std::fabs(n - 1.0) > 1e-6)
    return fail(BA_EINVAL, "%s %lld: quaternion norm %.9g differs from 1 by more than 1e-6", what,
                (long long)i, n);
  return BA_OK;
}

int check_options(const ba_options *o, bool pose_only) {
  if (!o) return fail(BA_EINVAL, "options is NULL");
  if (o->max_iters < 1 || o->max_iters > 100000) return fail(BA_EINVAL, "max_iters out of range");
  if (!pose_only) {
    if (o->pcg_max_iters < 1 || o->pcg_max_iters > 100000)
      return fail(BA_EINVAL, "pcg_max_iters out of range");
    if (!(o->pcg_rel_tol >= 0.0) || !std::isfinite(o->pcg_rel_tol))
      return fail(BA_EINVAL, "pcg_rel_tol must be finite and >= 0");
    if (!(o->lambda0 > 0.0) || !std::isfinite(o->lambda0)) return fail(BA_EINVAL, "lambda0 must be > 0");
  }
  if (!std::isfinite(o->huber_delta)) return fail(BA_EINVAL, "huber_delta must be finite");
  if (o->precision < BA_PREC_F64 || o->precision > BA_PREC_BF16J)
    return fail(BA_EINVAL, "unknown precision %d", o->precision);
  if (o->flags & ~(BA_FLAG_NO_GRAPH | BA_FLAG_PAIR_LISTS | BA_FLAG_PCG_WIDE | BA_FLAG_PCG_RESIDENT |
                   BA_FLAG_DENSE_SCHUR | BA_FLAG_PCG_COOPERATIVE))
    return fail(BA_EINVAL, "unknown option flags 0x%x", o->flags);
  if (!pose_only) {
    if (!(o->prior_abs >= 0.0) || !std::isfinite(o->prior_abs))
      return fail(BA_EINVAL, "prior_abs must be finite and >= 0");
    if (!(o->prior_seq >= 0.0) || !std::isfinite(o->prior_seq))
      return fail(BA_EINVAL, "prior_seq must be finite and >= 0");
    if (o->prior_seq > 0.0 && (o->prior_seq_k < 1 || o->prior_seq_k > 64))
      return fail(BA_EINVAL, "prior_seq_k must be in [1, 64]");
  }
  return BA_OK;
}

// ------------------------------------------------------------------ symbolic analysis
// Point chunks and their entries (chunk form of the Schur complement).  A chunk
// is a run of internal points with at most pcap points, ocap records and ccap
// cameras.  For every S block it touches, the chunk's items of that block are
// listed in point order (diagonal block of camera a: the chunk's observations in
// a; upper block (a, b): the pairs (p in a, q in b) of one point) and cut into
// entries of at most kChSubItems items; each entry is summed by one thread into
// its own partial.  Entries are ordered diagonal first, then by decreasing
// length, so the threads of a wavefront have similar work.
static int build_chunks(Symbolic &sy, const std::vector<int32_t> &up_rowptr,
                        const std::vector<int32_t> &up_col, int pcap, int ocap, int ccap) {
  const int P = sy.P, Cf = sy.Cf;
  std::vector<int32_t> nf(P, 0);
  for (int j = 0; j < P; ++j)
    for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k) nf[j] += sy.obs_rpos[k] >= 0;
  // a chunk closes before it would exceed pcap points, ocap records or ccap cameras
  sy.ch_pt.assign(1, 0);
  sy.ch_f0.assign(1, 0);
  sy.ch_cam_start.assign(1, 0);
  sy.ch_cam.clear();
  std::vector<int32_t> lcam(Cf, -1), cams;
  int32_t rec = 0;
  for (int j = 0; j < P;) {
    const int j0 = j;
    int c = 0;
    cams.clear();
    while (j < P && j - j0 < pcap && c + nf[j] <= ocap) {
      int fresh = 0;
      for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k)
        if (sy.obs_rpos[k] >= 0 && lcam[sy.free_idx[sy.obs_cam[k]]] < 0) ++fresh;
      if ((int)cams.size() + fresh > ccap) break;
      for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k)
        if (sy.obs_rpos[k] >= 0) {
          const int a = sy.free_idx[sy.obs_cam[k]];
          if (lcam[a] < 0) {
            lcam[a] = 0;
            cams.push_back(a);
          }
        }
      c += nf[j++];
    }
    if (j == j0) return fail(BA_EDEVICE, "internal: point %d does not fit a chunk", j0);
    std::sort(cams.begin(), cams.end());
    for (int a : cams) {
      lcam[a] = -1;
      sy.ch_cam.push_back(sy.free_cam[a]);
    }
    rec += c;
    sy.ch_pt.push_back(j);
    sy.ch_f0.push_back(rec);
    sy.ch_cam_start.push_back((int32_t)sy.ch_cam.size());
  }
  const int n_ch = (int)sy.ch_pt.size() - 1;
  sy.ch_ent.assign(1, 0);
  sy.ent_tgt.clear();
  sy.ent_cam.clear();
  sy.ent_slot.clear();
  sy.ent_start.clear();
  sy.ent_len.clear();
  sy.ent_items.clear();
  sy.n_dent = sy.n_oent = 0;
  std::vector<int32_t> la, ll;  // local camera and local record of one point's observations
  std::vector<int32_t> kcnt;     // items per (local camera a, local camera b) key
  std::vector<uint32_t> items, sorted;
  std::vector<int32_t> keys;
  struct Ent {
    int32_t a, b;
    size_t i0, i1;
  };
  std::vector<Ent> wave, thread, ordered;  // diagonal and upper entries of one chunk; both in launch order
  for (int c = 0; c < n_ch; ++c) {
    const int f0 = sy.ch_f0[c];
    const int q0 = sy.ch_cam_start[c], nq = sy.ch_cam_start[c + 1] - q0;
    // chunk-local camera index of each free camera of the chunk (cameras sorted)
    for (int x = 0; x < nq; ++x) lcam[sy.free_idx[sy.ch_cam[q0 + x]]] = x;
    // items keyed by (a, b) in local camera indices, stably counting-sorted by key
    keys.clear();
    items.clear();
    for (int j = sy.ch_pt[c]; j < sy.ch_pt[c + 1]; ++j) {
      la.clear();
      ll.clear();
      for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k)
        if (sy.obs_rpos[k] >= 0) {
          la.push_back(lcam[sy.free_idx[sy.obs_cam[k]]]);
          ll.push_back(sy.obs_rpos[k] - f0);
        }
      for (size_t x = 0; x < la.size(); ++x) {
        keys.push_back(la[x] * nq + la[x]);
        items.push_back((uint32_t)ll[x]);
        for (size_t y = x + 1; y < la.size(); ++y) {
          keys.push_back(la[x] * nq + la[y]);
          items.push_back((uint32_t)ll[x] | ((uint32_t)ll[y] << 16));
        }
      }
    }
    kcnt.assign((size_t)nq * nq + 1, 0);
    for (int32_t kk : keys) kcnt[kk + 1]++;
    for (size_t x = 0; x < (size_t)nq * nq; ++x) kcnt[x + 1] += kcnt[x];
    sorted.resize(items.size());
    {
      std::vector<int32_t> fillk(kcnt.begin(), kcnt.end() - 1);
      for (size_t x = 0; x < items.size(); ++x) sorted[fillk[keys[x]]++] = items[x];
    }
    wave.clear();
    thread.clear();
    for (int key = 0; key < nq * nq; ++key) {
      const size_t i = kcnt[key], e = kcnt[key + 1];
      if (i == e) continue;
      // one observation (pair) per point and block: the kernel relies on this bound
      if (e - i > (size_t)pcap) return fail(BA_EDEVICE, "internal: entry with %zu items", e - i);
      const int32_t a = sy.free_idx[sy.ch_cam[q0 + key / nq]], b = sy.free_idx[sy.ch_cam[q0 + key % nq]];
      for (size_t x = i; x < e; x += kChSubItems) {
        const Ent en{a, b, x, std::min(e, x + kChSubItems)};
        (a == b ? wave : thread).push_back(en);
      }
    }
    // threads of a wavefront run their entries side by side: group equal lengths
    const auto longer = [](const Ent &p, const Ent &q) { return p.i1 - p.i0 > q.i1 - q.i0; };
    std::stable_sort(wave.begin(), wave.end(), longer);
    std::stable_sort(thread.begin(), thread.end(), longer);
    ordered.clear();
    for (const std::vector<Ent> *lst : {&wave, &thread}) ordered.insert(ordered.end(), lst->begin(), lst->end());
    for (const Ent &en : ordered) {
      if (en.a == en.b) {
        sy.ent_tgt.push_back(en.a);
        sy.ent_cam.push_back(lcam[en.a]);
        sy.ent_slot.push_back(sy.n_dent++);
      } else {
        const auto beg = up_col.begin() + up_rowptr[en.a], end = up_col.begin() + up_rowptr[en.a + 1];
        const auto pos = std::lower_bound(beg, end, en.b);
        if (pos == end || *pos != en.b) return fail(BA_EDEVICE, "internal: block (%d, %d) missing", en.a, en.b);
        sy.ent_tgt.push_back(Cf + (int32_t)(pos - up_col.begin()));
        sy.ent_cam.push_back(lcam[en.b]);
        sy.ent_slot.push_back(sy.n_oent++);
      }
    }
    // items in slices of kEntSlice entries (a wavefront's, in launch order): item h of the
    // slice's entry l at h * kEntSlice + l, so that the threads of a wavefront read item h
    // of their entries from one contiguous run; shorter entries leave zeros
    for (size_t s0 = 0; s0 < ordered.size(); s0 += kEntSlice) {
      const size_t sn = std::min(ordered.size() - s0, (size_t)kEntSlice);
      size_t H = 0;
      for (size_t l = 0; l < sn; ++l) H = std::max(H, ordered[s0 + l].i1 - ordered[s0 + l].i0);
      const size_t base = sy.ent_items.size();
      if (base + H * kEntSlice > (size_t)INT32_MAX) return fail(BA_EINVAL, "more than 2^31 chunk items");
      sy.ent_items.resize(base + H * kEntSlice, 0u);
      for (size_t l = 0; l < sn; ++l) {
        const Ent &en = ordered[s0 + l];
        for (size_t h = 0; h < en.i1 - en.i0; ++h) sy.ent_items[base + h * kEntSlice + l] = sorted[en.i0 + h];
        sy.ent_start.push_back((int32_t)(base + l));
        sy.ent_len.push_back((uint8_t)(en.i1 - en.i0));
      }
    }
    sy.ch_ent.push_back((int32_t)sy.ent_tgt.size());
    for (int x = sy.ch_cam_start[c]; x < sy.ch_cam_start[c + 1]; ++x) lcam[sy.free_idx[sy.ch_cam[x]]] = -1;
  }
  // entries of each block in chunk order; an entry's partial is stored at its
  // position in that list (diagonal blocks first), so a block's partials are contiguous
  const int nblk = Cf + sy.n_up;
  sy.blk_start.assign(nblk + 1, 0);
  for (int32_t t : sy.ent_tgt) sy.blk_start[t + 1]++;
  for (int b = 0; b < nblk; ++b) sy.blk_start[b + 1] += sy.blk_start[b];
  std::vector<int32_t> bf(sy.blk_start.begin(), sy.blk_start.end() - 1);
  for (size_t e = 0; e < sy.ent_tgt.size(); ++e) {
    const int32_t pos = bf[sy.ent_tgt[e]]++;
    sy.ent_slot[e] = sy.ent_tgt[e] < Cf ? pos : pos - sy.n_dent;
  }
  return BA_OK;
}

// Whether the free cameras' co-visibility is dense: at least half of the free-camera
// pairs (a <= b) share a point.  One bitset of free cameras per camera, or-ed with
// the camera set of every point it sees.
static bool dense_covisibility(const Symbolic &sy) {
  const int Cf = sy.Cf, P = sy.P;
  const int W = (Cf + 63) / 64;
  std::vector<uint64_t> cov((size_t)Cf * W, 0), pb(W);
  std::vector<int32_t> cams;
  for (int j = 0; j < P; ++j) {
    cams.clear();
    std::fill(pb.begin(), pb.end(), 0);
    for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k) {
      const int a = sy.free_idx[sy.obs_cam[k]];
      if (a < 0) continue;
      pb[a >> 6] |= uint64_t(1) << (a & 63);
      cams.push_back(a);
    }
    for (int a : cams) {
      uint64_t *row = &cov[(size_t)a * W];
      for (int w = 0; w < W; ++w) row[w] |= pb[w];
    }
  }
  int64_t shared = 0;
  for (int a = 0; a < Cf; ++a)
    for (int b = a; b < Cf; ++b) shared += (cov[(size_t)a * W + (b >> 6)] >> (b & 63)) & 1;
  return 2 * shared >= (int64_t)Cf * (Cf + 1) / 2;
}

int analyse(const ba_problem_desc *d, const ba_options *opt, Symbolic &sy, const GraphEdges *edges,
            bool allow_dense) {
  if (!d) return fail(BA_EINVAL, "problem description is NULL");
  if (int e = check_options(opt, false)) return e;
  if (d->n_cams < 1) return fail(BA_EINVAL, "n_cams must be >= 1");
  if (!edges) {
    if (d->n_pts < 1) return fail(BA_EINVAL, "n_pts must be >= 1");
    if (d->n_obs < 1) return fail(BA_EINVAL, "n_obs must be >= 1");
    if (!d->points_xyz || !d->obs) return fail(BA_EINVAL, "NULL array in problem");
  } else if (d->n_pts != 0 || d->n_obs != 0) {
    return fail(BA_EDEVICE, "internal: a pose graph has no points or observations");
  }
  if (d->n_obs > (int64_t)INT32_MAX - 1) return fail(BA_EINVAL, "n_obs exceeds 2^31 - 2");
  if (!d->K || !d->poses) return fail(BA_EINVAL, "NULL array in problem");
  const int C = d->n_cams, P = d->n_pts;
  const int64_t N = d->n_obs;
  const int nK = d->K_per_cam ? C : 1;
  for (int i = 0; i < nK; ++i) {
    const ba_intrinsics &k = d->K[i];
    if (!(std::isfinite(k.fx) && std::isfinite(k.fy) && std::isfinite(k.cx) && std::isfinite(k.cy)) ||
        k.fx == 0.0 || k.fy == 0.0)
      return fail(BA_EINVAL, "intrinsics %d invalid", i);
  }
  for (int i = 0; i < C; ++i)
    if (int e = check_pose(d->poses[i], "camera", i)) return e;
  for (int64_t i = 0; i < 3 * (int64_t)P; ++i)
    if (!std::isfinite(d->points_xyz[i])) return fail(BA_EINVAL, "point %lld non-finite", (long long)(i / 3));
  for (int64_t k = 0; k < N; ++k) {
    const ba_obs &o = d->obs[k];
    if (o.cam < 0 || o.cam >= C) return fail(BA_EINVAL, "observation %lld: camera %d out of range", (long long)k, o.cam);
    if (o.pt < 0 || o.pt >= P) return fail(BA_EINVAL, "observation %lld: point %d out of range", (long long)k, o.pt);
    if (!std::isfinite(o.u) || !std::isfinite(o.v)) return fail(BA_EINVAL, "observation %lld non-finite", (long long)k);
  }
  sy.C = C;
  sy.P = P;
  sy.N = (int32_t)N;
  sy.free_idx.assign(C, -1);
  sy.free_cam.clear();
  for (int i = 0; i < C; ++i)
    if (!(d->cam_fixed && d->cam_fixed[i])) {
      sy.free_idx[i] = (int32_t)sy.free_cam.size();
      sy.free_cam.push_back(i);
    }
  sy.Cf = (int32_t)sy.free_cam.size();
  if (sy.Cf == 0) return fail(BA_EINVAL, "every camera is fixed");

  const int Cf = sy.Cf;
  // Internal point order: by first free camera, then the caller's index, so that
  // consecutive points share a narrow window of cameras (the chunk form's
  // locality).  Results are returned in the caller's order.
  std::vector<int32_t> first(P, Cf);
  for (int64_t k = 0; k < N; ++k) {
    const int a = sy.free_idx[d->obs[k].cam];
    if (a >= 0 && a < first[d->obs[k].pt]) first[d->obs[k].pt] = a;
  }
  std::vector<int32_t> rank(P);
  {
    std::vector<int32_t> c(Cf + 2, 0);
    for (int j = 0; j < P; ++j) c[first[j] + 1]++;
    for (int a = 0; a <= Cf; ++a) c[a + 1] += c[a];
    sy.pt_order.resize(P);
    for (int j = 0; j < P; ++j) {
      rank[j] = c[first[j]]++;
      sy.pt_order[rank[j]] = j;
    }
  }

  // order by (internal point, camera): stable counting sort by camera, then by point
  std::vector<int32_t> cnt(std::max(C, P) + 1);
  std::vector<int32_t> by_cam(N);
  std::vector<int32_t> &order = sy.obs_order;
  order.assign(N, 0);
  std::fill(cnt.begin(), cnt.begin() + C + 1, 0);
  for (int64_t k = 0; k < N; ++k) cnt[d->obs[k].cam + 1]++;
  for (int i = 0; i < C; ++i) cnt[i + 1] += cnt[i];
  for (int64_t k = 0; k < N; ++k) by_cam[cnt[d->obs[k].cam]++] = (int32_t)k;
  sy.pt_start.assign(P + 1, 0);
  for (int64_t k = 0; k < N; ++k) sy.pt_start[rank[d->obs[k].pt] + 1]++;
  for (int j = 0; j < P; ++j) sy.pt_start[j + 1] += sy.pt_start[j];
  std::vector<int32_t> fill(sy.pt_start.begin(), sy.pt_start.end() - 1);
  for (int64_t t = 0; t < N; ++t) {
    const int32_t k = by_cam[t];
    order[fill[rank[d->obs[k].pt]]++] = k;
  }
  sy.obs_cam.resize(N);
  sy.obs_pt.resize(N);
  sy.obs_uv.resize(2 * N);
  for (int64_t k = 0; k < N; ++k) {
    const ba_obs &o = d->obs[order[k]];
    sy.obs_cam[k] = o.cam;
    sy.obs_pt[k] = rank[o.pt];
    sy.obs_uv[2 * k] = o.u;
    sy.obs_uv[2 * k + 1] = o.v;
  }
  for (int j = 0; j < P; ++j)
    for (int k = sy.pt_start[j] + 1; k < sy.pt_start[j + 1]; ++k)
      if (sy.obs_cam[k] == sy.obs_cam[k - 1])
        return fail(BA_EINVAL, "point %d observed twice by camera %d", sy.pt_order[j], sy.obs_cam[k]);

  // records: one per observation in a free camera
  int max_free = 0;
  sy.Nf = 0;
  int64_t free_pairs = 0;
  for (int j = 0; j < P; ++j) {
    int nfj = 0;
    for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k) nfj += sy.free_idx[sy.obs_cam[k]] >= 0;
    max_free = std::max(max_free, nfj);
    sy.Nf += nfj;
    free_pairs += (int64_t)nfj * (nfj - 1) / 2;
  }
  const int prec = opt->precision;
  // points with long tracks (16 or more observations on average) take tiles of fewer
  // points, so that a problem spreads over more workgroups.  Otherwise a tile walks its
  // observations in passes of one per thread, one after another, so a problem whose
  // full tiles would not give every CU 8 of them takes tiles of half the points: twice
  // the workgroups, still all resident at once, each with half the passes (the 2M-
  // observation drive: 977 -> 1954 tiles, point_trial 62 -> 50 us)
  sy.pt_tile = N >= 16 * (int64_t)std::max(P, 1)                ? kPtTileLong
               : (P + kPtTile - 1) / kPtTile < (int64_t)kPtTileFill ? kPtTile / 2
                                                                    : kPtTile;
  // the dense co-visibility form: forced by its flag, or chosen when tracks span at
  // least a quarter of the free cameras on average, the pairs are many per block of S
  // and most camera pairs share points (never with pair lists asked for)
  sy.dense = allow_dense && !edges && Cf <= kDnMaxCams && !(opt->flags & BA_FLAG_PAIR_LISTS) &&
             dense_form_available() &&
             ((opt->flags & BA_FLAG_DENSE_SCHUR) ||
              (4 * (int64_t)sy.Nf >= (int64_t)Cf * P && free_pairs >= 32 * ((int64_t)Cf * (Cf + 1) / 2) &&
               dense_covisibility(sy)));
  sy.chunked = !sy.dense && !(opt->flags & BA_FLAG_PAIR_LISTS) && max_free <= chunk_obs_cap(prec) &&
               max_free <= chunk_cam_cap(prec) &&
               chunk_lds_bytes(prec) <= device_lds_limit();

  // observations of each free camera (camera-major slots)
  sy.cam_obs_start.assign(Cf + 1, 0);
  for (int64_t k = 0; k < N; ++k) {
    const int a = sy.free_idx[sy.obs_cam[k]];
    if (a >= 0) sy.cam_obs_start[a + 1]++;
  }
  for (int a = 0; a < Cf; ++a) sy.cam_obs_start[a + 1] += sy.cam_obs_start[a];
  sy.cam_obs.resize(sy.cam_obs_start[Cf]);
  std::vector<int32_t> cpos(N, -1);
  {
    std::vector<int32_t> f(sy.cam_obs_start.begin(), sy.cam_obs_start.end() - 1);
    for (int64_t k = 0; k < N; ++k) {
      const int a = sy.free_idx[sy.obs_cam[k]];
      if (a >= 0) {
        cpos[k] = f[a];
        sy.cam_obs[f[a]++] = (int32_t)k;
      }
    }
  }
  // record of each observation: point-major in the chunk and dense forms, camera-major otherwise
  if (sy.chunked || sy.dense) {
    sy.obs_rpos.assign(N, -1);
    int32_t r = 0;
    for (int64_t k = 0; k < N; ++k)
      if (sy.free_idx[sy.obs_cam[k]] >= 0) sy.obs_rpos[k] = r++;
  } else {
    sy.obs_rpos = cpos;
  }

  // relative-pose pairs with at least one free camera (pairs of two fixed cameras are
  // constant): the pose-graph edges, or the sequential prior pairs (i, i + k) in the
  // caller's camera order, measured from the initial poses with weight lambda_c
  sy.prior_abs = opt->prior_abs;
  sy.pp_cam.clear();
  sy.pp_meas.clear();
  sy.pp_w.clear();
  if (edges) {
    for (size_t e = 0; e < edges->pairs.size(); ++e) {
      const int2 ij = edges->pairs[e];
      if (sy.free_idx[ij.x] < 0 && sy.free_idx[ij.y] < 0) continue;
      sy.pp_cam.push_back(ij);
      sy.pp_meas.insert(sy.pp_meas.end(), edges->meas.begin() + 12 * e, edges->meas.begin() + 12 * e + 12);
      sy.pp_w.insert(sy.pp_w.end(), edges->w.begin() + 2 * e, edges->w.begin() + 2 * e + 2);
    }
  } else if (opt->prior_seq > 0.0) {
    for (int i = 0; i < C; ++i)
      for (int k = 1; k <= opt->prior_seq_k && i + k < C; ++k)
        if (sy.free_idx[i] >= 0 || sy.free_idx[i + k] >= 0) {
          double Ti[12], Tj[12], A[12];
          quat_to_pose12(d->poses[i], Ti);
          quat_to_pose12(d->poses[i + k], Tj);
          relative_pose12(Ti, Tj, A);
          sy.pp_cam.push_back(int2{i, i + k});
          sy.pp_meas.insert(sy.pp_meas.end(), A, A + 12);
          sy.pp_w.push_back(opt->prior_seq);
          sy.pp_w.push_back(opt->prior_seq);
        }
  }
  // later free partners of each free camera through a pair: their blocks of S exist even
  // where no point is seen by both
  std::vector<int32_t> padj_start(Cf + 1, 0), padj;
  const std::vector<int2> no_pattern;
  const std::vector<int2> &pattern = edges ? edges->pattern : no_pattern;
  for (const std::vector<int2> *lst : {(const std::vector<int2> *)&sy.pp_cam, &pattern})
    for (const int2 &ij : *lst) {
      const int a = sy.free_idx[ij.x], b = sy.free_idx[ij.y];
      if (a >= 0 && b >= 0 && a != b) padj_start[std::min(a, b) + 1]++;
    }
  for (int a = 0; a < Cf; ++a) padj_start[a + 1] += padj_start[a];
  padj.resize(padj_start[Cf]);
  {
    std::vector<int32_t> f(padj_start.begin(), padj_start.end() - 1);
    for (const std::vector<int2> *lst : {(const std::vector<int2> *)&sy.pp_cam, &pattern})
      for (const int2 &ij : *lst) {
        const int a = sy.free_idx[ij.x], b = sy.free_idx[ij.y];
        if (a >= 0 && b >= 0 && a != b) padj[f[std::min(a, b)]++] = std::max(a, b);
      }
  }
  std::vector<uint8_t> pmark(Cf, 0);

  // upper blocks of S row by row (and their observation-pair lists in the pair-list form)
  std::vector<int32_t> up_rowptr(Cf + 1, 0), up_col;
  std::vector<int32_t> rowcnt(Cf, 0), slot(Cf, -1);
  std::vector<int32_t> touched;
  sy.pairs.clear();
  sy.up_pair_start.assign(1, 0);
  sy.n_pairs = 0;
  if (sy.dense) {  // every block of S is held: no pair enumeration
    for (int a = 0; a < Cf; ++a) {
      for (int b = a + 1; b < Cf; ++b) up_col.push_back(b);
      up_rowptr[a + 1] = (int32_t)up_col.size();
    }
    sy.n_pairs = free_pairs;
  }
  for (int a = 0; a < Cf && !sy.dense; ++a) {
    touched.clear();
    for (int o = sy.cam_obs_start[a]; o < sy.cam_obs_start[a + 1]; ++o) {
      const int k = sy.cam_obs[o];
      const int j = sy.obs_pt[k];
      for (int kb = k + 1; kb < sy.pt_start[j + 1]; ++kb) {
        const int b = sy.free_idx[sy.obs_cam[kb]];
        if (b < 0) continue;
        if (rowcnt[b]++ == 0) touched.push_back(b);
      }
    }
    for (int x = padj_start[a]; x < padj_start[a + 1]; ++x) {
      const int b = padj[x];
      if (rowcnt[b] == 0 && !pmark[b]) {
        pmark[b] = 1;
        touched.push_back(b);
      }
    }
    std::sort(touched.begin(), touched.end());
    const int base_blk = (int)up_col.size();
    int64_t pbase = sy.n_pairs;
    std::vector<int64_t> pfill(touched.size());
    for (size_t t = 0; t < touched.size(); ++t) {
      const int b = touched[t];
      slot[b] = base_blk + (int)t;
      up_col.push_back(b);
      pfill[t] = pbase;
      pbase += rowcnt[b];
      if (pbase > (int64_t)INT32_MAX) return fail(BA_EINVAL, "more than 2^31 observation pairs");
      if (!sy.chunked) sy.up_pair_start.push_back((int32_t)pbase);
    }
    sy.n_pairs = pbase;
    if (!sy.chunked) {
      sy.pairs.resize(pbase);
      for (int o = sy.cam_obs_start[a]; o < sy.cam_obs_start[a + 1]; ++o) {
        const int k = sy.cam_obs[o];
        const int j = sy.obs_pt[k];
        for (int kb = k + 1; kb < sy.pt_start[j + 1]; ++kb) {
          const int b = sy.free_idx[sy.obs_cam[kb]];
          if (b < 0) continue;
          const int t = slot[b] - base_blk;
          sy.pairs[pfill[t]++] = int2{o, cpos[kb]};  // camera-major slots
        }
      }
    }
    for (int b : touched) {
      rowcnt[b] = 0;
      slot[b] = -1;
      pmark[b] = 0;
    }
    up_rowptr[a + 1] = (int32_t)up_col.size();
  }
  sy.n_up = (int32_t)up_col.size();
  // prior pairs: upper block of each pair of free cameras, pairs of each free camera
  sy.pp_up.assign(sy.pp_cam.size(), -1);
  sy.cam_pp_start.assign(Cf + 1, 0);
  for (size_t p = 0; p < sy.pp_cam.size(); ++p) {
    const int fa = sy.free_idx[sy.pp_cam[p].x], fb = sy.free_idx[sy.pp_cam[p].y];
    if (fa >= 0) sy.cam_pp_start[fa + 1]++;
    if (fb >= 0) sy.cam_pp_start[fb + 1]++;
    if (fa >= 0 && fb >= 0) {
      const int a = std::min(fa, fb), b = std::max(fa, fb);
      const auto beg = up_col.begin() + up_rowptr[a], end = up_col.begin() + up_rowptr[a + 1];
      const auto pos = std::lower_bound(beg, end, b);
      if (pos == end || *pos != b) return fail(BA_EDEVICE, "internal: prior block (%d, %d) missing", a, b);
      sy.pp_up[p] = (int32_t)(pos - up_col.begin());
    }
  }
  for (int a = 0; a < Cf; ++a) sy.cam_pp_start[a + 1] += sy.cam_pp_start[a];
  sy.cam_pp.resize(sy.cam_pp_start[Cf]);
  {
    std::vector<int32_t> f(sy.cam_pp_start.begin(), sy.cam_pp_start.end() - 1);
    for (size_t p = 0; p < sy.pp_cam.size(); ++p) {
      const int a = sy.free_idx[sy.pp_cam[p].x], b = sy.free_idx[sy.pp_cam[p].y];
      if (a >= 0) sy.cam_pp[f[a]++] = (int32_t)p;
      if (b >= 0) sy.cam_pp[f[b]++] = (int32_t)p;
    }
  }
  if (sy.chunked) {
    sy.cam_obs.clear();
    sy.cam_obs.shrink_to_fit();
    sy.cam_obs_start.clear();
  }

  // full block rows of S: lower blocks (transposes), the diagonal, upper blocks
  std::vector<int32_t> n_low(Cf, 0);
  for (int u = 0; u < sy.n_up; ++u) n_low[up_col[u]]++;
  sy.S_rowptr.assign(Cf + 1, 0);
  for (int a = 0; a < Cf; ++a)
    sy.S_rowptr[a + 1] = sy.S_rowptr[a] + n_low[a] + 1 + (up_rowptr[a + 1] - up_rowptr[a]);
  sy.nnzb = sy.S_rowptr[Cf];
  sy.S_col.assign(sy.nnzb, -1);
  sy.diag_pos.resize(Cf);
  sy.up_pos.resize(sy.n_up);
  sy.up_tpos.resize(sy.n_up);
  std::vector<int32_t> low_fill(Cf);
  for (int a = 0; a < Cf; ++a) {
    low_fill[a] = sy.S_rowptr[a];
    sy.diag_pos[a] = sy.S_rowptr[a] + n_low[a];
    sy.S_col[sy.diag_pos[a]] = a;
  }
  for (int a = 0; a < Cf; ++a)
    for (int u = up_rowptr[a]; u < up_rowptr[a + 1]; ++u) {
      const int b = up_col[u];
      const int pos = sy.diag_pos[a] + 1 + (u - up_rowptr[a]);
      sy.S_col[pos] = b;
      sy.up_pos[u] = pos;
      const int tpos = low_fill[b]++;  // rows a are visited in increasing order
      sy.S_col[tpos] = a;
      sy.up_tpos[u] = tpos;
    }
  // distinct columns of each PCG tile and each block's position in its tile's list;
  // the lists are stored at a fixed stride (the longest list), padded with -1.
  // A tile holds kPcgRows rows, or kPcgRowsSparse when there are many rows: each launch
  // sums every tile's partials in every tile, so the tile count must stay modest.
  auto tile_lists = [&](int R) {
    const int ntile = (Cf + R - 1) / R;
    sy.pcg_rows = R;
    sy.S_lcol.assign(sy.nnzb, 0);
    sy.max_tcols = 0;
    std::vector<std::vector<int32_t>> lists(ntile);
    std::vector<int32_t> where(Cf, -1);
    for (int t = 0; t < ntile; ++t) {
      std::vector<int32_t> &cols = lists[t];
      const int r0 = t * R, r1 = std::min(Cf, r0 + R);
      for (int pos = sy.S_rowptr[r0]; pos < sy.S_rowptr[r1]; ++pos) cols.push_back(sy.S_col[pos]);
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      for (size_t i = 0; i < cols.size(); ++i) where[cols[i]] = (int32_t)i;
      for (int pos = sy.S_rowptr[r0]; pos < sy.S_rowptr[r1]; ++pos) sy.S_lcol[pos] = where[sy.S_col[pos]];
      sy.max_tcols = std::max(sy.max_tcols, (int32_t)cols.size());
    }
    sy.tcol.assign((size_t)ntile * sy.max_tcols, -1);
    for (int t = 0; t < ntile; ++t)
      std::copy(lists[t].begin(), lists[t].end(), sy.tcol.begin() + (size_t)t * sy.max_tcols);
  };
  // At least 1024 rows take 16 rows per tile, or 32 (half a wave each) once 16-row
  // tiles would outnumber what the device runs at once (two 1024-thread workgroups per
  // CU): 4-row tiles would outnumber the CUs, so that a step would run in several
  // rounds of workgroups (the 3000-camera loop scene, 148 blocks per row: 19.8 us per
  // step with 750 tiles, 9.6 us with 188), and on sparse rows they would leave most
  // lanes idle.  A tile whose columns do not fit in LDS falls back to fewer rows.
  const bool sparse_rows = Cf >= 1024;
  const bool wide = (opt->flags & BA_FLAG_PCG_WIDE) || (Cf + kPcgRowsSparse - 1) / kPcgRowsSparse > 512;
  tile_lists(!(sparse_rows || (opt->flags & BA_FLAG_PCG_WIDE)) ? kPcgRows : wide ? kPcgRowsMax : kPcgRowsSparse);
  if (sy.pcg_rows == kPcgRowsMax && !one_reduction_pcg(prec, sy.max_tcols)) tile_lists(kPcgRowsSparse);
  if (sy.pcg_rows == kPcgRowsSparse && !one_reduction_pcg(prec, sy.max_tcols)) tile_lists(kPcgRows);
  sy.pcg_resident = (opt->flags & BA_FLAG_PCG_RESIDENT) &&
                    resident_pcg_fits(prec, sy.pcg_rows, (Cf + sy.pcg_rows - 1) / sy.pcg_rows, sy.max_tcols);
  sy.pcg_coop = sy.pcg_resident && (opt->flags & BA_FLAG_PCG_COOPERATIVE);
  if (sy.dense) {
    // first record of each point in each camera tile: the point's records in the tile
    // are the range [ts[t], ts[t + 1]) (records are point-major, in camera order), and
    // each record's free camera
    const int nt = (Cf + kDnCams - 1) / kDnCams;
    sy.dn_tiles = nt;
    const int64_t pairs_t = (int64_t)nt * (nt + 1) / 2;
    // point ranges: enough workgroups for the problem, each at most kDnRangePts points
    // so that no range outlasts the others by much
    sy.dn_split = (int32_t)std::max<int64_t>(
        {1, std::min<int64_t>((kDnTargetWgs + pairs_t - 1) / pairs_t, (int64_t)P / 256),
         ((int64_t)P + kDnRangePts - 1) / kDnRangePts});
    sy.dn_ts.assign((size_t)P * (nt + 1), 0);
    sy.dn_rcam.assign(sy.Nf, 0);
    sy.dn_mask.assign((size_t)P * nt, 0);
    int32_t r = 0;
    for (int j = 0; j < P; ++j) {
      int32_t *ts = &sy.dn_ts[(size_t)j * (nt + 1)];
      uint16_t *mk = &sy.dn_mask[(size_t)j * nt];
      int t = 0;
      for (int k = sy.pt_start[j]; k < sy.pt_start[j + 1]; ++k) {
        const int a = sy.free_idx[sy.obs_cam[k]];
        if (a < 0) continue;
        while (t <= a / kDnCams) ts[t++] = r;
        mk[a / kDnCams] |= (uint16_t)(1u << (a % kDnCams));
        sy.dn_rcam[r++] = a;
      }
      while (t <= nt) ts[t++] = r;
    }
    // the camera-major walk of dense_cams reads each observation's record position and
    // point from here, in order, instead of gathering them by observation index
    sy.dn_crec.resize(sy.cam_obs.size());
    for (size_t o = 0; o < sy.cam_obs.size(); ++o) {
      const int k = sy.cam_obs[o];
      sy.dn_crec[o] = make_int2(sy.obs_rpos[k], sy.obs_pt[k]);
    }
  }
  if (sy.chunked)
    return build_chunks(sy, up_rowptr, up_col, chunk_pts_cap(prec), chunk_obs_cap(prec), chunk_cam_cap(prec));
  return BA_OK;
}

// ------------------------------------------------------------------ device layout
namespace {
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};
}  // namespace

namespace {
// Byte offsets of the report block (each part 8-byte aligned): the upload slot of the
// fresh state, then the state after the solve, the evaluation partials and the
// per-iteration arrays.
struct ReportLayout {
  size_t up, st, sq, nm, ic, pi, total;
  ReportLayout(int npt, int max_iters) {
    size_t o = 0;
    auto take = [&](size_t b) {
      const size_t r = o;
      o += (b + 7) & ~size_t(7);
      return r;
    };
    up = take(sizeof(LMState));
    st = take(sizeof(LMState));
    sq = take((size_t)npt * 8);
    nm = take((size_t)npt * 4);
    ic = take(((size_t)max_iters + 1) * 8);
    pi = take((size_t)max_iters * 4);
    total = o;
  }
};
}  // namespace

size_t DevProblem::plan(const Symbolic &sy, int precision, int max_iters, Offsets &o) {
  const size_t T = compute_bytes(precision);
  const size_t C = sy.C, Cf = sy.Cf, P = sy.P, N = sy.N;
  const size_t npt = (P + sy.pt_tile - 1) / sy.pt_tile;
  const size_t npcg = (Cf + sy.pcg_rows - 1) / sy.pcg_rows;
  const size_t ncam = (C + kCamTile - 1) / kCamTile;
  Layout L;
  // the report block: the state, the evaluation partials and the per-iteration arrays,
  // placed as in the page-locked report, so that one copy brings a solve's report up
  const ReportLayout RL((int)npt, max_iters);
  const size_t rep = L.take(RL.total);
  o.st = rep + RL.st;
  o.K = L.take(C * 4 * T);
  o.free_idx = L.take(C * 4);
  o.free_cam = L.take(Cf * 4);
  o.obs_cam = L.take(N * 4);
  o.obs_pt = L.take(N * 4);
  o.obs_uv = L.take(N * 2 * T);
  o.pt_start = L.take((P + 1) * 4);
  o.obs_rpos = L.take(N * 4);
  o.obs_act = L.take(N);
  o.cam_obs = L.take(sy.cam_obs.size() * 4 + 4);
  o.cam_obs_start = L.take(sy.cam_obs_start.size() * 4 + 4);
  o.up_pair_start = L.take(sy.up_pair_start.size() * 4 + 4);
  o.pairs = L.take(sy.pairs.size() * sizeof(int2) + 8);
  o.ch_pt = L.take(sy.ch_pt.size() * 4 + 4);
  o.ch_f0 = L.take(sy.ch_f0.size() * 4 + 4);
  o.ch_ent = L.take(sy.ch_ent.size() * 4 + 4);
  o.ch_cam_start = L.take(sy.ch_cam_start.size() * 4 + 4);
  o.ch_cam = L.take(sy.ch_cam.size() * 4 + 4);
  o.ent_tgt = L.take(sy.ent_tgt.size() * 4 + 4);
  o.ent_cam = L.take(sy.ent_cam.size() * 4 + 4);
  o.ent_slot = L.take(sy.ent_slot.size() * 4 + 4);
  o.ent_start = L.take(sy.ent_start.size() * 4 + 4);
  o.ent_len = L.take(sy.ent_len.size() + 4);
  o.ent_items = L.take(sy.ent_items.size() * 4 + 4);
  o.blk_start = L.take(sy.blk_start.size() * 4 + 4);
  o.part_d = L.take((size_t)sy.n_dent * 54 * T + 16);
  o.part_o = L.take((size_t)sy.n_oent * 36 * T + 16);
  o.row_tot = L.take(sy.chunked || sy.dense ? Cf * 54 * 8 : 16);
  o.dn_ts = L.take(sy.dn_ts.size() * 4 + 4);
  o.dn_rcam = L.take(sy.dn_rcam.size() * 4 + 4);
  o.dn_crec = L.take(sy.dn_crec.size() * 8 + 8);
  o.dn_mask = L.take(sy.dn_mask.size() * 2 + 4);
  o.dn_pfac = L.take(sy.dense ? P * 9 * T : 16);
  o.dn_part = L.take(sy.dense ? (size_t)sy.dn_tiles * (sy.dn_tiles + 1) / 2 * sy.dn_split * kDnRows * kDnRows * T
                              : 16);
  o.pp_cam = L.take(sy.pp_cam.size() * sizeof(int2) + 8);
  o.pp_meas = L.take(sy.pp_meas.size() * 8 + 8);
  o.pp_w = L.take(sy.pp_w.size() * 8 + 8);
  o.pp_up = L.take(sy.pp_up.size() * 4 + 4);
  o.cam_pp_start = L.take(sy.cam_pp_start.size() * 4 + 4);
  o.cam_pp = L.take(sy.cam_pp.size() * 4 + 4);
  const bool prior_on = sy.prior_abs > 0.0 || !sy.pp_cam.empty();
  o.prior_diag = L.take(prior_on ? Cf * 27 * 8 : 16);
  o.part_prior = L.take(prior_on ? 2 * ((std::max(Cf, sy.pp_cam.size()) + 255) / 256) * 8 : 16);
  o.prior_off = L.take(sy.pp_cam.size() * 36 * 8 + 16);
  o.up_pos = L.take(sy.n_up * 4 + 4);
  o.up_tpos = L.take(sy.n_up * 4 + 4);
  o.diag_pos = L.take(Cf * 4);
  o.S_rowptr = L.take((Cf + 1) * 4);
  o.S_col = L.take(sy.nnzb * 4);
  o.tcol = L.take(sy.tcol.size() * 4 + 4);
  o.S_lcol = L.take(sy.nnzb * 4);
  for (int b = 0; b < 2; ++b) o.pose[b] = L.take(C * 12 * 8);
  for (int b = 0; b < 2; ++b) o.X[b] = L.take(P * 3 * 8);
  o.pose_init = L.take(C * 12 * 8);
  o.X_init = L.take(P * 3 * 8);
  const size_t Nf = sy.Nf;
  o.lin = L.take(Nf * lin_record_bytes(precision) + 16);
  o.Q = L.take((sy.chunked ? 0 : Nf * 6 * T) + 16);
  o.V = L.take(P * 6 * T);
  o.gp = L.take(P * 3 * T);
  o.Dp = L.take(P * 3 * T);
  o.Vinv = L.take(P * 6 * T);
  o.gc = L.take(Cf * 6 * T);
  o.Dc = L.take(Cf * 6 * T);
  o.brhs = L.take(Cf * 6 * T);
  o.S = L.take((size_t)sy.nnzb * 36 * T);
  o.Minv = L.take(Cf * 36 * 8);
  for (int i = 0; i < 14; ++i) o.vec[i] = L.take(Cf * 6 * T);
  o.part_lin_cost = L.take(npt * 8);
  o.part_masked = rep + RL.nm;
  o.part_sq = rep + RL.sq;
  o.part_trial_cost = L.take(npt * 8);
  o.part_trial_masked = L.take(npt * 4);
  o.part_dl_pt = L.take(npt * 8);
  o.part_dl_cam = L.take(ncam * 8);
  o.part_rz0 = L.take(Cf * 8);
  o.part_bb = L.take(Cf * 8);
  o.part_rz[0] = L.take(npcg * 8);
  o.part_rz[1] = L.take(npcg * 8);
  o.part_pq = L.take(npcg * 8);
  o.part_cg[0] = L.take(3 * npcg * 8);
  o.part_cg[1] = L.take(3 * npcg * 8);
  o.cg_flag = L.take(npcg * 4);
  o.part_rr = L.take(npcg * 8);
  o.part_cull = L.take(npt * 8);
  o.iter_cost = rep + RL.ic;
  o.iter_pcg = rep + RL.pi;
  o.total = L.off;
  return L.off;
}

size_t DevProblem::bytes_for(const Symbolic &sy, int precision, int max_iters) {
  Offsets o;
  return plan(sy, precision, max_iters, o);
}

template <class T>
static std::vector<T> cast_vec(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

int DevProblem::init(const Symbolic &sy, const ba_problem_desc *d, const ba_options *opt,
                     char *base, hipStream_t s) {
  precision = opt->precision;
  max_iters = opt->max_iters;
  pcg_max = opt->pcg_max_iters;
  lambda0 = opt->lambda0;
  pcg_tol = opt->pcg_rel_tol;
  huber = opt->huber_delta;
  C = sy.C;
  Cf = sy.Cf;
  P = sy.P;
  N = sy.N;
  max_tcols = sy.max_tcols;
  pt_order = sy.pt_order;
  obs_order = sy.obs_order;
  n_active = N;
  plan(sy, precision, max_iters, off);
  dev = base;
  auto ptr = [&](size_t o) { return (void *)(base + o); };
  ProbDev &pd = view;
  std::memset(&pd, 0, sizeof(pd));
  pd.C = C;
  pd.Cf = Cf;
  pd.P = P;
  pd.N = N;
  pd.Nf = sy.Nf;
  pd.chunked = sy.chunked ? 1 : 0;
  pd.n_ch = sy.chunked ? (int32_t)sy.ch_pt.size() - 1 : 0;
  pd.n_red_tiles = sy.chunked ? (sy.n_up + 3) / 4 : 0;  // four upper blocks (one wave each) per tile
  pd.n_fin_tiles = sy.chunked && sy.Nf > 0 ? Cf : 0;
  pd.n_fsh_tiles = sy.chunked || sy.dense ? (Cf + 63) / 64 : 0;
  pd.dense = sy.dense ? 1 : 0;
  pd.dn_tiles = sy.dense ? sy.dn_tiles : 0;
  pd.dn_pairs = sy.dense ? sy.dn_tiles * (sy.dn_tiles + 1) / 2 : 0;
  pd.dn_split = sy.dense ? sy.dn_split : 0;
  pd.n_up = sy.n_up;
  pd.nnzb = sy.nnzb;
  pd.n_pt_tiles = (P + sy.pt_tile - 1) / sy.pt_tile;
  pd.pt_tile = sy.pt_tile;
  pd.n_pcg_tiles = (Cf + sy.pcg_rows - 1) / sy.pcg_rows;
  pd.pcg_rows = sy.pcg_rows;
  pd.pcg_resident = sy.pcg_resident ? (sy.pcg_coop ? 2 : 1) : 0;
  pd.n_cam_tiles = (C + kCamTile - 1) / kCamTile;
  pd.K = ptr(off.K);
  pd.free_idx = (const int32_t *)ptr(off.free_idx);
  pd.free_cam = (const int32_t *)ptr(off.free_cam);
  pd.obs_cam = (const int32_t *)ptr(off.obs_cam);
  pd.obs_pt = (const int32_t *)ptr(off.obs_pt);
  pd.obs_uv = ptr(off.obs_uv);
  pd.pt_start = (const int32_t *)ptr(off.pt_start);
  pd.obs_rpos = (const int32_t *)ptr(off.obs_rpos);
  pd.obs_act = (uint8_t *)ptr(off.obs_act);
  pd.cam_obs = (const int32_t *)ptr(off.cam_obs);
  pd.cam_obs_start = (const int32_t *)ptr(off.cam_obs_start);
  pd.up_pair_start = (const int32_t *)ptr(off.up_pair_start);
  pd.pairs = (const int2 *)ptr(off.pairs);
  pd.ch_pt = (const int32_t *)ptr(off.ch_pt);
  pd.ch_f0 = (const int32_t *)ptr(off.ch_f0);
  pd.ch_ent = (const int32_t *)ptr(off.ch_ent);
  pd.ch_cam_start = (const int32_t *)ptr(off.ch_cam_start);
  pd.ch_cam = (const int32_t *)ptr(off.ch_cam);
  pd.ent_tgt = (const int32_t *)ptr(off.ent_tgt);
  pd.ent_cam = (const int32_t *)ptr(off.ent_cam);
  pd.ent_slot = (const int32_t *)ptr(off.ent_slot);
  pd.ent_start = (const int32_t *)ptr(off.ent_start);
  pd.ent_len = (const uint8_t *)ptr(off.ent_len);
  pd.ent_items = (const uint32_t *)ptr(off.ent_items);
  pd.blk_start = (const int32_t *)ptr(off.blk_start);
  pd.n_dent = sy.n_dent;
  pd.part_d = ptr(off.part_d);
  pd.part_o = ptr(off.part_o);
  pd.row_tot = (double *)ptr(off.row_tot);
  pd.dn_ts = (const int32_t *)ptr(off.dn_ts);
  pd.dn_rcam = (const int32_t *)ptr(off.dn_rcam);
  pd.dn_crec = (const int2 *)ptr(off.dn_crec);
  pd.dn_mask = (const uint16_t *)ptr(off.dn_mask);
  pd.dn_pfac = ptr(off.dn_pfac);
  pd.dn_part = ptr(off.dn_part);
  pd.prior_abs = sy.prior_abs;
  pd.n_pp = (int32_t)sy.pp_cam.size();
  pd.prior_on = (sy.prior_abs > 0.0 || pd.n_pp > 0) ? 1 : 0;
  pd.prior_abs_from = 0;
  pd.prior_nodes = C;
  pd.n_pri_tiles = pd.prior_on ? (std::max(Cf, pd.n_pp) + 255) / 256 : 0;
  pd.part_prior = (double *)ptr(off.part_prior);
  pd.pose0 = (const double *)ptr(off.pose_init);
  pd.pp_cam = (const int2 *)ptr(off.pp_cam);
  pd.pp_meas = (const double *)ptr(off.pp_meas);
  pd.pp_w = (const double *)ptr(off.pp_w);
  pd.pp_up = (const int32_t *)ptr(off.pp_up);
  pd.cam_pp_start = (const int32_t *)ptr(off.cam_pp_start);
  pd.cam_pp = (const int32_t *)ptr(off.cam_pp);
  pd.prior_diag = (double *)ptr(off.prior_diag);
  pd.prior_off = (double *)ptr(off.prior_off);
  pd.up_pos = (const int32_t *)ptr(off.up_pos);
  pd.up_tpos = (const int32_t *)ptr(off.up_tpos);
  pd.diag_pos = (const int32_t *)ptr(off.diag_pos);
  pd.S_rowptr = (const int32_t *)ptr(off.S_rowptr);
  pd.S_col = (const int32_t *)ptr(off.S_col);
  pd.tcol = (const int32_t *)ptr(off.tcol);
  pd.S_lcol = (const int32_t *)ptr(off.S_lcol);
  pd.max_tcols = sy.max_tcols;
  for (int b = 0; b < 2; ++b) {
    pd.pose[b] = (double *)ptr(off.pose[b]);
    pd.X[b] = (double *)ptr(off.X[b]);
  }
  pd.lin = ptr(off.lin);
  pd.Q = ptr(off.Q);
  pd.V = ptr(off.V);
  pd.gp = ptr(off.gp);
  pd.Dp = ptr(off.Dp);
  pd.Vinv = ptr(off.Vinv);
  pd.gc = ptr(off.gc);
  pd.Dc = ptr(off.Dc);
  pd.brhs = ptr(off.brhs);
  pd.S = ptr(off.S);
  pd.Minv = (double *)ptr(off.Minv);
  pd.x = ptr(off.vec[0]);
  pd.r = ptr(off.vec[1]);
  pd.z = ptr(off.vec[2]);
  pd.p0 = ptr(off.vec[3]);
  pd.p1 = ptr(off.vec[4]);
  pd.q = ptr(off.vec[5]);
  // one-reduction form: r and u of parity 0 alias r and z (written by the diagonal kernel)
  pd.cg_r[0] = pd.r;
  pd.cg_u[0] = pd.z;
  pd.cg_r[1] = ptr(off.vec[6]);
  pd.cg_u[1] = ptr(off.vec[7]);
  pd.cg_w[0] = ptr(off.vec[8]);
  pd.cg_w[1] = ptr(off.vec[9]);
  pd.cg_s[0] = ptr(off.vec[10]);
  pd.cg_s[1] = ptr(off.vec[11]);
  pd.part_lin_cost = (double *)ptr(off.part_lin_cost);
  pd.part_masked = (int32_t *)ptr(off.part_masked);
  pd.part_sq = (double *)ptr(off.part_sq);
  pd.part_trial_cost = (double *)ptr(off.part_trial_cost);
  pd.part_trial_masked = (int32_t *)ptr(off.part_trial_masked);
  pd.part_dl_pt = (double *)ptr(off.part_dl_pt);
  pd.part_dl_cam = (double *)ptr(off.part_dl_cam);
  pd.part_rz0 = (double *)ptr(off.part_rz0);
  pd.part_bb = (double *)ptr(off.part_bb);
  pd.part_rz[0] = (double *)ptr(off.part_rz[0]);
  pd.part_rz[1] = (double *)ptr(off.part_rz[1]);
  pd.part_pq = (double *)ptr(off.part_pq);
  pd.part_cg[0] = (double *)ptr(off.part_cg[0]);
  pd.part_cg[1] = (double *)ptr(off.part_cg[1]);
  pd.cg_flag = (uint32_t *)ptr(off.cg_flag);
  pd.part_rr = (double *)ptr(off.part_rr);
  pd.part_cull = (int32_t *)ptr(off.part_cull);
  pd.st = (LMState *)ptr(off.st);
  pd.iter_cost = (double *)ptr(off.iter_cost);
  pd.iter_pcg = (int32_t *)ptr(off.iter_pcg);

  // host staging of every input in its device form
  std::vector<double> Kd(4 * (size_t)C);
  for (int i = 0; i < C; ++i) {
    const ba_intrinsics &k = d->K[d->K_per_cam ? i : 0];
    Kd[4 * i] = k.fx;
    Kd[4 * i + 1] = k.fy;
    Kd[4 * i + 2] = k.cx;
    Kd[4 * i + 3] = k.cy;
  }
  std::vector<double> poses(12 * (size_t)C);
  for (int i = 0; i < C; ++i) quat_to_pose12(d->poses[i], &poses[12 * (size_t)i]);
  auto up = [&](size_t o, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  if (precision == BA_PREC_F64) {
    chk(up(off.K, Kd.data(), Kd.size() * 8));
    chk(up(off.obs_uv, sy.obs_uv.data(), sy.obs_uv.size() * 8));
  } else {
    staging_f.push_back(cast_vec<float>(Kd));
    chk(up(off.K, staging_f.back().data(), Kd.size() * 4));
    staging_f.push_back(cast_vec<float>(sy.obs_uv));
    chk(up(off.obs_uv, staging_f.back().data(), sy.obs_uv.size() * 4));
  }
  chk(up(off.free_idx, sy.free_idx.data(), sy.free_idx.size() * 4));
  chk(up(off.free_cam, sy.free_cam.data(), sy.free_cam.size() * 4));
  chk(up(off.obs_cam, sy.obs_cam.data(), sy.obs_cam.size() * 4));
  chk(up(off.obs_pt, sy.obs_pt.data(), sy.obs_pt.size() * 4));
  chk(up(off.pt_start, sy.pt_start.data(), sy.pt_start.size() * 4));
  chk(up(off.obs_rpos, sy.obs_rpos.data(), sy.obs_rpos.size() * 4));
  if (N > 0) chk(hipMemsetAsync(base + off.obs_act, 1, (size_t)N, s));
  chk(up(off.cam_obs, sy.cam_obs.data(), sy.cam_obs.size() * 4));
  chk(up(off.cam_obs_start, sy.cam_obs_start.data(), sy.cam_obs_start.size() * 4));
  chk(up(off.up_pair_start, sy.up_pair_start.data(), sy.up_pair_start.size() * 4));
  chk(up(off.pairs, sy.pairs.data(), sy.pairs.size() * sizeof(int2)));
  chk(up(off.pp_cam, sy.pp_cam.data(), sy.pp_cam.size() * sizeof(int2)));
  chk(up(off.pp_meas, sy.pp_meas.data(), sy.pp_meas.size() * 8));
  chk(up(off.pp_w, sy.pp_w.data(), sy.pp_w.size() * 8));
  chk(up(off.pp_up, sy.pp_up.data(), sy.pp_up.size() * 4));
  chk(up(off.cam_pp_start, sy.cam_pp_start.data(), sy.cam_pp_start.size() * 4));
  chk(up(off.cam_pp, sy.cam_pp.data(), sy.cam_pp.size() * 4));
  chk(up(off.ch_pt, sy.ch_pt.data(), sy.ch_pt.size() * 4));
  chk(up(off.ch_f0, sy.ch_f0.data(), sy.ch_f0.size() * 4));
  chk(up(off.ch_ent, sy.ch_ent.data(), sy.ch_ent.size() * 4));
  chk(up(off.ch_cam_start, sy.ch_cam_start.data(), sy.ch_cam_start.size() * 4));
  chk(up(off.ch_cam, sy.ch_cam.data(), sy.ch_cam.size() * 4));
  chk(up(off.ent_tgt, sy.ent_tgt.data(), sy.ent_tgt.size() * 4));
  chk(up(off.ent_cam, sy.ent_cam.data(), sy.ent_cam.size() * 4));
  chk(up(off.ent_slot, sy.ent_slot.data(), sy.ent_slot.size() * 4));
  chk(up(off.ent_start, sy.ent_start.data(), sy.ent_start.size() * 4));
  chk(up(off.ent_len, sy.ent_len.data(), sy.ent_len.size()));
  chk(up(off.ent_items, sy.ent_items.data(), sy.ent_items.size() * 4));
  chk(up(off.blk_start, sy.blk_start.data(), sy.blk_start.size() * 4));
  chk(up(off.dn_ts, sy.dn_ts.data(), sy.dn_ts.size() * 4));
  chk(up(off.dn_rcam, sy.dn_rcam.data(), sy.dn_rcam.size() * 4));
  chk(up(off.dn_crec, sy.dn_crec.data(), sy.dn_crec.size() * 8));
  chk(up(off.dn_mask, sy.dn_mask.data(), sy.dn_mask.size() * 2));
  chk(up(off.up_pos, sy.up_pos.data(), sy.up_pos.size() * 4));
  chk(up(off.up_tpos, sy.up_tpos.data(), sy.up_tpos.size() * 4));
  chk(up(off.diag_pos, sy.diag_pos.data(), sy.diag_pos.size() * 4));
  chk(up(off.S_rowptr, sy.S_rowptr.data(), sy.S_rowptr.size() * 4));
  chk(up(off.S_col, sy.S_col.data(), sy.S_col.size() * 4));
  chk(up(off.tcol, sy.tcol.data(), sy.tcol.size() * 4));
  chk(up(off.S_lcol, sy.S_lcol.data(), sy.S_lcol.size() * 4));
  staging_d.push_back(std::move(poses));
  chk(up(off.pose[0], staging_d.back().data(), 12 * (size_t)C * 8));
  chk(up(off.pose_init, staging_d.back().data(), 12 * (size_t)C * 8));
  std::vector<double> Xi(3 * (size_t)P);  // points in the internal order
  for (int j = 0; j < P; ++j)
    for (int m = 0; m < 3; ++m) Xi[3 * (size_t)j + m] = d->points_xyz[3 * (size_t)pt_order[j] + m];
  staging_d.push_back(std::move(Xi));
  chk(up(off.X[0], staging_d.back().data(), 3 * (size_t)P * 8));
  chk(up(off.X_init, staging_d.back().data(), 3 * (size_t)P * 8));
  host_state = LMState{};
  host_state.cur = 0;
  if (e != hipSuccess) return hip_fail(e, "upload");
  return BA_OK;
}

LMState DevProblem::fresh_state() const {
  LMState st{};
  st.lambda = lambda0;
  st.lambda0 = lambda0;
  st.nu = 2.0;
  st.pcg_tol = pcg_tol;
  st.huber_delta = huber;
  st.iter = 0;
  st.max_iters = max_iters;
  st.relin = 1;
  st.status = 0;
  st.accepted = 0;
  st.cur = host_state.cur;
  st.pcg_max = pcg_max;
  st.init_done = 0;
  st.bar_polls = bar_polls;
  return st;
}

// ------------------------------------------------------------------ batches
void Batch::clear() {
  probs.clear();
  tags.clear();
  for (auto &v : tiles) v.clear();
}

void Batch::add(const ProbDev &pd, int slot_tag) {
  const int pi = (int)probs.size();
  probs.push_back(pd);
  tags.push_back(slot_tag);
  for (int t = 0; t < pd.n_pt_tiles; ++t) tiles[0].push_back(Tile{pi, t});
  if (pd.dense) {
    for (int t = 0; t < pd.n_pt_tiles; ++t) tiles[12].push_back(Tile{pi, t});
    for (int a = 0; a < pd.Cf; ++a) tiles[13].push_back(Tile{pi, a});
    for (int t = 0; t < pd.dn_pairs * pd.dn_split; ++t) tiles[14].push_back(Tile{pi, t});
    for (int t = 0; t < pd.dn_pairs * kDnCams; ++t) tiles[15].push_back(Tile{pi, t});
    for (int t = 0; t < pd.n_fsh_tiles; ++t) tiles[10].push_back(Tile{pi, t});
  } else if (pd.chunked) {
    for (int c = 0; c < pd.n_ch; ++c) tiles[7].push_back(Tile{pi, c});
    for (int t = 0; t < pd.n_red_tiles; ++t) tiles[8].push_back(Tile{pi, t});
    for (int t = 0; t < pd.n_fin_tiles; ++t) tiles[9].push_back(Tile{pi, t});
    for (int t = 0; t < pd.n_fsh_tiles; ++t) tiles[10].push_back(Tile{pi, t});
  } else {
    for (int t = 0; t < pd.n_pt_tiles; ++t) tiles[6].push_back(Tile{pi, t});
    for (int a = 0; a < pd.Cf; ++a) tiles[1].push_back(Tile{pi, a});
    for (int t = 0; t < (pd.n_up + kOffWaves - 1) / kOffWaves; ++t) tiles[2].push_back(Tile{pi, t});
  }
  for (int t = 0; t < pd.n_pcg_tiles; ++t) tiles[3].push_back(Tile{pi, t});
  for (int t = 0; t < pd.n_cam_tiles; ++t) tiles[4].push_back(Tile{pi, t});
  tiles[5].push_back(Tile{pi, 0});
  for (int t = 0; t < pd.n_pri_tiles; ++t) tiles[11].push_back(Tile{pi, t});
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup j to XCD j mod 8),
// and each XCD has its own L2.  Reordering a tile list so that XCD x receives a
// contiguous run of tiles keeps the blocks that share a camera's records on one
// L2.  The map is a bijection and changes no result.
static void xcd_contiguous(std::vector<Tile> &v) {
  constexpr int kXcd = 8;
  const size_t n = v.size();
  if (n < 2 * kXcd) return;
  size_t start[kXcd + 1];
  start[0] = 0;
  for (int x = 0; x < kXcd; ++x) start[x + 1] = start[x] + n / kXcd + ((size_t)x < n % kXcd ? 1 : 0);
  std::vector<Tile> out(n);
  for (size_t j = 0; j < n; ++j) out[j] = v[start[j % kXcd] + j / kXcd];
  v.swap(out);
}

int Batch::upload(hipStream_t s) {
  xcd_contiguous(tiles[2]);
  xcd_contiguous(tiles[7]);
  size_t need = probs.size() * sizeof(ProbDev);
  constexpr int NL = 16;
  size_t offs[NL];
  for (int i = 0; i < NL; ++i) {
    need = (need + 255) & ~size_t(255);
    offs[i] = need;
    need += tiles[i].size() * sizeof(Tile);
  }
  if (need > cap) {
    if (dev) (void)hipFree(dev);
    dev = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&dev, need * 2);
    if (e != hipSuccess) return hip_fail(e, "batch table allocation");
    cap = need * 2;
  }
  host.assign(need, 0);
  std::memcpy(host.data(), probs.data(), probs.size() * sizeof(ProbDev));
  for (int i = 0; i < NL; ++i)
    std::memcpy(host.data() + offs[i], tiles[i].data(), tiles[i].size() * sizeof(Tile));
  hipError_t e = hipMemcpyAsync(dev, host.data(), need, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "batch table upload");
  char *b = (char *)dev;
  plan.probs = (const ProbDev *)b;
  const Tile **dst[NL] = {&plan.pt, &plan.diag, &plan.off, &plan.pcg, &plan.cam, &plan.ctl,
                          &plan.pp, &plan.ch, &plan.red, &plan.fin, &plan.fsh, &plan.pri,
                          &plan.dpt, &plan.dcm, &plan.dsy, &plan.dre};
  int32_t *cnt[NL] = {&plan.n_pt, &plan.n_diag, &plan.n_off, &plan.n_pcg, &plan.n_cam, &plan.n_ctl,
                      &plan.n_pp, &plan.n_ch, &plan.n_red, &plan.n_fin, &plan.n_fsh, &plan.n_pri,
                      &plan.n_dpt, &plan.n_dcm, &plan.n_dsy, &plan.n_dre};
  for (int i = 0; i < NL; ++i) {
    *dst[i] = (const Tile *)(b + offs[i]);
    *cnt[i] = (int32_t)tiles[i].size();
  }
  plan.n_probs = (int32_t)probs.size();
  plan.pcg_rows = probs.empty() ? kPcgRows : probs[0].pcg_rows;
  for (const ProbDev &pd : probs)
    if (pd.pcg_rows != plan.pcg_rows) plan.pcg_rows = 0;
  if (probs.size() == 1) plan.single = probs[0];
  return BA_OK;
}

Batch::~Batch() {
  if (dev) (void)hipFree(dev);
}

// ------------------------------------------------------------------ timing
void EventTimer::begin(int id, hipStream_t s, int launches) {
  active = ((mask >> id) & 1u) != 0 && (seen[id]++ % stride) == 0;
  if (!active) return;
  if (used == pool.size()) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    pool.push_back({a, b});
  }
  (void)hipEventRecord(pool[used].first, s);
  ids.push_back(id);
  counts.push_back(launches);
}
void EventTimer::end(int, hipStream_t s) {
  if (!active) return;
  (void)hipEventRecord(pool[used].second, s);
  ++used;
  active = false;
}
void EventTimer::reset() {
  used = 0;
  ids.clear();
  counts.clear();
  for (int i = 0; i < K_NUM_KERNELS; ++i) seen[i] = 0;
}
void EventTimer::reserve(size_t pairs) {
  while (pool.size() < pairs) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    pool.push_back({a, b});
  }
}
void EventTimer::collect(double ms[K_NUM_KERNELS], int32_t launches[K_NUM_KERNELS]) {
  for (int i = 0; i < K_NUM_KERNELS; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (size_t i = 0; i < used; ++i) {
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, pool[i].first, pool[i].second);
    ms[ids[i]] += t;
    launches[ids[i]] += counts[i];
  }
}
EventTimer::~EventTimer() {
  for (auto &p : pool) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
}

}  // namespace bax

// ====================================================================== C-ABI
using namespace bax;

// The rig unknowns of a vehicle-rig problem: their view (vehicle poses, then
// extrinsics, as nodes), its batch, and the lists that project the composed cameras'
// reduced system onto them.
struct RigPart {
  int F = 0, nr = 0;
  Symbolic sy;
  DevProblem dp;
  Batch batch;
  void *mem = nullptr;    // the rig view's arrays
  void *extra = nullptr;  // Ucam, rdiag, contribution and row lists
  size_t bytes = 0;
  ~RigPart() {
    if (mem) (void)hipFree(mem);
    if (extra) (void)hipFree(extra);
  }
};

struct ba_problem {
  Symbolic sy;
  DevProblem dp;
  Batch batch;
  std::unique_ptr<RigPart> rig;  // vehicle-rig problems only
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void *mem = nullptr;
  size_t bytes = 0;
  double setup_ms = 0.0;
  int64_t n_pairs = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool pending = false;
  bool solved = false;
  bool profiling = false;
  bool use_graph = true;
  hipGraph_t graph = nullptr;       // the launch sequence of one solve, captured once
  hipGraphExec_t graph_exec = nullptr;
  // the LM iterations around their PCG runs: before the first run, the run, after a run and
  // before the next one, after the last run
  hipGraph_t seg_graph[4] = {};
  hipGraphExec_t seg_exec[4] = {};
  EventTimer timer;  // times the kernels selected by timer.mask
  double kernel_ms[K_NUM_KERNELS] = {};
  int32_t kernel_launches[K_NUM_KERNELS] = {};
  double solve_ms = 0.0;
  char *rep_pin = nullptr;  // page-locked: the fresh state's upload slot and the report block
  bool rep_ok = false;      // rep_pin holds the last solve's report
};

extern "C" {

const char *ba_version(void) { return "ba_mi355x 0.1 (gfx950)"; }
const char *ba_last_error(void) { return g_last_error.c_str(); }

void ba_default_options(ba_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iters = 10;
  o->pcg_max_iters = 50;
  o->pcg_rel_tol = 1e-6;
  o->lambda0 = 1e-4;
  o->huber_delta = 0.0;
  o->precision = BA_PREC_F32;
  o->prior_seq_k = 1;
}

static int create_problem(const ba_problem_desc *d, const ba_options *opt, void *hip_stream,
                          const GraphEdges *edges, ba_problem **out,
                          const std::function<int(ba_problem *)> &before_upload = nullptr) {
  if (!out) return fail(BA_EINVAL, "out is NULL");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<ba_problem> p(new ba_problem());
  // before_upload builds a vehicle rig's second view, whose camera view keeps the
  // chunk or pair-list form (the rig kernels read its per-block layout)
  if (int e = analyse(d, opt, p->sy, edges, !before_upload)) return e;
  if (prepare_kernels() != 0) return fail(BA_EDEVICE, "no HIP device");
  p->bytes = DevProblem::bytes_for(p->sy, opt->precision, opt->max_iters);
  p->use_graph = (opt->flags & BA_FLAG_NO_GRAPH) == 0;
  if (hip_stream) {
    p->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreate(&p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    p->own_stream = true;
  }
  hipError_t e = hipMalloc(&p->mem, p->bytes);
  if (e != hipSuccess) {
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    return hip_fail(e, "problem allocation");
  }
  int rc = p->dp.init(p->sy, d, opt, (char *)p->mem, p->stream);
  if (rc == BA_OK && before_upload) rc = before_upload(p.get());
  if (rc == BA_OK) {
    p->batch.add(p->dp.view, 0);
    rc = p->batch.upload(p->stream);
  }
  if (rc == BA_OK) {
    hipError_t e2 = hipEventCreate(&p->ev0);
    if (e2 == hipSuccess) e2 = hipEventCreate(&p->ev1);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(p->stream);
    if (e2 != hipSuccess) rc = hip_fail(e2, "setup");
  }
  if (rc != BA_OK) {
    (void)hipFree(p->mem);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    return rc;
  }
  // the host copies needed later are the sizes only; drop the big arrays
  p->n_pairs = p->sy.n_pairs;
  p->sy.pairs.clear();
  p->sy.pairs.shrink_to_fit();
  p->sy.ent_items.clear();
  p->sy.ent_items.shrink_to_fit();
  p->sy.ent_len.clear();
  p->sy.ent_len.shrink_to_fit();
  p->sy.obs_order.clear();
  p->sy.obs_order.shrink_to_fit();
  p->dp.staging_f.clear();
  p->dp.staging_d.clear();
  p->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p.release();
  return BA_OK;
}

int ba_create(const ba_problem_desc *d, const ba_options *opt, void *hip_stream, ba_problem **out) {
  return create_problem(d, opt, hip_stream, nullptr, out);
}

// Builds the rig view over the composed-camera problem p (analysed and initialised,
// not yet uploaded) and ties the two views together.
static int build_rig(ba_problem *p, const ba_rig_desc *r, const ba_options *opt) {
  RigPart &rg = *p->rig;
  const int F = rg.F, nr = rg.nr, nodes = F + nr;
  const Symbolic &sc = p->sy;
  // rig nodes: vehicles 0..F-1, then extrinsics
  std::vector<ba_pose> npose(nodes);
  std::vector<uint8_t> nfixed(nodes, 0);
  for (int f = 0; f < F; ++f) {
    npose[f] = r->vehicle_poses[f];
    nfixed[f] = r->vehicle_fixed ? r->vehicle_fixed[f] : 0;
  }
  for (int c = 0; c < nr; ++c) {
    npose[F + c] = r->extrinsics[c];
    nfixed[F + c] = r->extrinsic_fixed ? r->extrinsic_fixed[c] : 0;
  }
  std::vector<int32_t> nfree(nodes, -1);
  {
    int k = 0;
    for (int n = 0; n < nodes; ++n)
      if (!nfixed[n]) nfree[n] = k++;
    if (k == 0) return fail(BA_EINVAL, "every vehicle pose and extrinsic is fixed");
  }
  // rigidity pairs, measured from the initial extrinsics; couplings of the composed
  // cameras' reduced system carried over to the rig unknowns
  GraphEdges ge;
  for (int k = 0; k < r->n_rig_pairs; ++k) {
    const int c = r->rig_pairs[2 * k], d = r->rig_pairs[2 * k + 1];
    double Ec[12], Ed[12], A[12];
    quat_to_pose12(r->extrinsics[c], Ec);
    quat_to_pose12(r->extrinsics[d], Ed);
    relative_pose12(Ec, Ed, A);
    ge.pairs.push_back(int2{F + c, F + d});
    ge.meas.insert(ge.meas.end(), A, A + 12);
    ge.w.push_back(r->prior_rig);
    ge.w.push_back(r->prior_rig);
  }
  auto nodes_of = [&](int cam, int out[2]) {
    out[0] = cam / nr;           // vehicle of its frame
    out[1] = F + cam % nr;       // its extrinsic
  };
  for (int a = 0; a < sc.Cf; ++a)
    for (int pos = sc.S_rowptr[a]; pos < sc.S_rowptr[a + 1]; ++pos) {
      const int b = sc.S_col[pos];
      if (b < a) continue;  // the upper triangle carries every coupling
      int na[2], nb[2];
      nodes_of(sc.free_cam[a], na);
      nodes_of(sc.free_cam[b], nb);
      for (int x : na)
        for (int y : nb)
          if (x != y) ge.pattern.push_back(int2{std::min(x, y), std::max(x, y)});
    }
  std::sort(ge.pattern.begin(), ge.pattern.end(),
            [](const int2 &u, const int2 &v) { return u.x < v.x || (u.x == v.x && u.y < v.y); });
  ge.pattern.erase(std::unique(ge.pattern.begin(), ge.pattern.end(),
                               [](const int2 &u, const int2 &v) { return u.x == v.x && u.y == v.y; }),
                   ge.pattern.end());
  const ba_intrinsics K1{1.0, 1.0, 0.0, 0.0};
  ba_problem_desc dn{};
  dn.n_cams = nodes;
  dn.K = &K1;
  dn.poses = npose.data();
  dn.cam_fixed = nfixed.data();
  ba_options on = *opt;
  on.prior_abs = r->prior_ext;
  on.prior_seq = 0.0;
  on.huber_delta = 0.0;
  on.flags &= ~BA_FLAG_PAIR_LISTS;
  if (int e = analyse(&dn, &on, rg.sy, &ge)) return e;
  if (!rg.sy.chunked) return fail(BA_EDEVICE, "internal: the rig view needs the chunk layout");
  const Symbolic &sr = rg.sy;
  rg.bytes = DevProblem::bytes_for(sr, opt->precision, opt->max_iters);
  hipError_t e = hipMalloc(&rg.mem, rg.bytes);
  if (e != hipSuccess) return hip_fail(e, "rig allocation");
  if (int rc = rg.dp.init(sr, &dn, &on, (char *)rg.mem, p->stream)) return rc;
  // contributions of camera blocks to rig blocks (rig BSR position order, camera order)
  auto rig_pos = [&](int x, int y) -> int {
    const auto beg = sr.S_col.begin() + sr.S_rowptr[x], end = sr.S_col.begin() + sr.S_rowptr[x + 1];
    const auto it = std::lower_bound(beg, end, y);
    return (it != end && *it == y) ? (int)(it - sr.S_col.begin()) : -1;
  };
  const int nnzb = sr.nnzb, Cfr = sr.Cf;
  std::vector<int32_t> rb_start(nnzb + 1, 0), rb_pos, rb_lr, rb_diag(nnzb, -1);
  std::vector<std::array<int32_t, 3>> contrib;  // rig position, camera position, transforms
  for (int a = 0; a < sc.Cf; ++a)
    for (int pos = sc.S_rowptr[a]; pos < sc.S_rowptr[a + 1]; ++pos) {
      const int b = sc.S_col[pos];
      const int ca = sc.free_cam[a], cb = sc.free_cam[b];
      int na[2], nb[2];
      nodes_of(ca, na);
      nodes_of(cb, nb);
      for (int s1 = 0; s1 < 2; ++s1)
        for (int s2 = 0; s2 < 2; ++s2) {
          const int x = nfree[na[s1]], y = nfree[nb[s2]];
          if (x < 0 || y < 0) continue;
          const int rp = rig_pos(x, y);
          if (rp < 0) return fail(BA_EDEVICE, "internal: rig block (%d, %d) missing", x, y);
          const int lc = s1 == 0 ? ca % nr : -1, rc2 = s2 == 0 ? cb % nr : -1;
          contrib.push_back({rp, pos, (lc + 1) | ((rc2 + 1) << 16)});
        }
    }
  for (const auto &c : contrib) rb_start[c[0] + 1]++;
  for (int i = 0; i < nnzb; ++i) rb_start[i + 1] += rb_start[i];
  rb_pos.resize(contrib.size());
  rb_lr.resize(contrib.size());
  {
    std::vector<int32_t> f(rb_start.begin(), rb_start.end() - 1);
    for (const auto &c : contrib) {
      rb_pos[f[c[0]]] = c[1];
      rb_lr[f[c[0]]++] = c[2];
    }
  }
  for (int x = 0; x < Cfr; ++x) rb_diag[sr.diag_pos[x]] = x;
  // segments of at most kRigSeg contributions, never across two rig blocks
  std::vector<int32_t> rs_blk(nnzb + 1, 0), rs_c0;
  for (int bk = 0; bk < nnzb; ++bk) {
    for (int c = rb_start[bk]; c < rb_start[bk + 1]; c += kRigSeg) rs_c0.push_back(c);
    rs_blk[bk + 1] = (int32_t)rs_c0.size();
  }
  const int n_seg = (int)rs_c0.size();
  rs_c0.push_back((int32_t)contrib.size());
  // rs_c0[s + 1] must end segment s inside its block: close each block's last segment
  {
    std::vector<int32_t> ends(n_seg);
    for (int bk = 0; bk < nnzb; ++bk)
      for (int sg = rs_blk[bk]; sg < rs_blk[bk + 1]; ++sg)
        ends[sg] = std::min(rs_c0[sg] + kRigSeg, rb_start[bk + 1]);
    for (int sg = 0; sg + 1 < n_seg; ++sg)
      if (ends[sg] != rs_c0[sg + 1]) return fail(BA_EDEVICE, "internal: rig segments");
  }
  // composed cameras of each free rig unknown
  std::vector<int32_t> rr_start(Cfr + 1, 0), rr_cam;
  for (int x = 0; x < Cfr; ++x) {
    const int node = sr.free_cam[x];
    if (node < F)
      for (int c = 0; c < nr; ++c) rr_cam.push_back(node * nr + c);
    else
      for (int f = 0; f < F; ++f) rr_cam.push_back(f * nr + (node - F));
    rr_start[x + 1] = (int32_t)rr_cam.size();
  }
  // one more allocation: Ucam, rdiag and the lists
  const size_t C = (size_t)sc.C;
  constexpr int NA = 11;
  size_t off[NA], tot = 0;
  const size_t sizes[NA] = {C * 21 * 8, (size_t)Cfr * 36 * 8, rb_start.size() * 4, rb_pos.size() * 4 + 4,
                            rb_lr.size() * 4 + 4, rb_diag.size() * 4 + 4, rr_start.size() * 4, rr_cam.size() * 4 + 4,
                            rs_blk.size() * 4, rs_c0.size() * 4, (size_t)n_seg * 36 * 8 + 8};
  for (int i = 0; i < NA; ++i) {
    off[i] = tot;
    tot += (sizes[i] + 255) & ~size_t(255);
  }
  e = hipMalloc(&rg.extra, tot);
  if (e != hipSuccess) return hip_fail(e, "rig allocation");
  char *xb = (char *)rg.extra;
  const void *src[NA] = {nullptr, nullptr, rb_start.data(), rb_pos.data(), rb_lr.data(), rb_diag.data(),
                         rr_start.data(), rr_cam.data(), rs_blk.data(), rs_c0.data(), nullptr};
  const size_t nbytes[NA] = {0, 0, rb_start.size() * 4, rb_pos.size() * 4, rb_lr.size() * 4, rb_diag.size() * 4,
                             rr_start.size() * 4, rr_cam.size() * 4, rs_blk.size() * 4, rs_c0.size() * 4, 0};
  for (int i = 2; i < NA && e == hipSuccess; ++i)
    if (nbytes[i]) e = hipMemcpy(xb + off[i], src[i], nbytes[i], hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "rig upload");
  // the rig view: its LM state is the composed-camera problem's
  ProbDev &rv = rg.dp.view;
  ProbDev &cv = p->dp.view;
  rv.st = cv.st;
  rv.rig_mode = 2;
  rv.n_frames = F;
  rv.n_rigcam = nr;
  rv.prior_abs_from = F;
  rv.prior_nodes = nodes;
  rv.Nf = 1;  // its row sums come from k_rig_rows
  rv.chunked = 1;
  rv.n_ch = (n_seg + 3) / 4;        // rig-segment tiles (4 segments each)
  rv.n_rig_seg = n_seg;
  rv.rs_blk = (const int32_t *)(xb + off[8]);
  rv.rs_c0 = (const int32_t *)(xb + off[9]);
  rv.rpart = (double *)(xb + off[10]);
  rv.n_red_tiles = (nnzb + 3) / 4;  // rig-block tiles (4 blocks each)
  rv.n_fin_tiles = Cfr;             // rig-row tiles
  rv.n_fsh_tiles = (Cfr + 63) / 64;
  rv.n_pt_tiles = 0;
  rv.n_cam_tiles = 0;
  rv.rdiag = (double *)(xb + off[1]);
  rv.rb_start = (const int32_t *)(xb + off[2]);
  rv.rb_pos = (const int32_t *)(xb + off[3]);
  rv.rb_lr = (const int32_t *)(xb + off[4]);
  rv.rb_diag = (const int32_t *)(xb + off[5]);
  rv.rr_start = (const int32_t *)(xb + off[6]);
  rv.rr_cam = (const int32_t *)(xb + off[7]);
  rv.cam_S = cv.S;
  rv.cam_gc = cv.gc;
  rv.cam_brhs = cv.brhs;
  rv.cam_U = (const double *)(xb + off[0]);
  rg.batch.add(rv, 0);
  if (int rc = rg.batch.upload(p->stream)) return rc;
  // the composed-camera view: undamped blocks, the rig's priors for the cost, the rig update
  cv.rig_mode = 1;
  cv.n_frames = F;
  cv.n_rigcam = nr;
  cv.Ucam = (double *)(xb + off[0]);
  cv.rig_pose[0] = rv.pose[0];
  cv.rig_pose[1] = rv.pose[1];
  cv.rig_x = rv.x;
  cv.rig_gc = rv.gc;
  cv.rig_Dc = rv.Dc;
  cv.rig_free_idx = rv.free_idx;
  cv.prior_on = 0;
  cv.prior_abs = rv.prior_abs;
  cv.prior_abs_from = F;
  cv.prior_nodes = nodes;
  cv.pose0 = rv.pose0;
  cv.n_pp = rv.n_pp;
  cv.pp_cam = rv.pp_cam;
  cv.pp_meas = rv.pp_meas;
  cv.pp_w = rv.pp_w;
  cv.n_pri_tiles = 0;
  cv.n_cam_tiles = (std::max(cv.C, nodes) + kCamTile - 1) / kCamTile;
  // the update's per-tile partials go to part_dl_cam, sized for the camera tiles (256-byte padded)
  const size_t dl_slots = ((((size_t)cv.C + kCamTile - 1) / kCamTile * 8 + 255) & ~size_t(255)) / 8;
  if ((size_t)cv.n_cam_tiles > dl_slots) return fail(BA_EINVAL, "rig too large for one camera per frame");
  return BA_OK;
}

int ba_rig_create(const ba_rig_desc *r, const ba_options *opt, void *hip_stream, ba_problem **out) {
  if (out) *out = nullptr;
  if (!r) return fail(BA_EINVAL, "rig description is NULL");
  if (!opt) return fail(BA_EINVAL, "options are NULL");
  if (r->n_frames < 1) return fail(BA_EINVAL, "n_frames must be >= 1");
  if (r->n_rig < 1 || r->n_rig > BA_RIG_MAX_CAMS) return fail(BA_EINVAL, "n_rig must be in 1..%d", BA_RIG_MAX_CAMS);
  if ((int64_t)r->n_frames * r->n_rig > INT32_MAX / 2) return fail(BA_EINVAL, "n_frames * n_rig too large");
  if (r->n_pts < 1 || r->n_obs < 1) return fail(BA_EINVAL, "n_pts and n_obs must be >= 1");
  if (!r->K || !r->vehicle_poses || !r->extrinsics || !r->points_xyz || !r->obs)
    return fail(BA_EINVAL, "NULL array in rig description");
  if (opt->prior_abs != 0.0 || opt->prior_seq != 0.0)
    return fail(BA_EINVAL, "a rig problem takes its priors from the rig description (prior_abs, prior_seq must be 0)");
  if (!(std::isfinite(r->prior_ext) && r->prior_ext >= 0.0) || !(std::isfinite(r->prior_rig) && r->prior_rig >= 0.0))
    return fail(BA_EINVAL, "prior_ext and prior_rig must be finite and >= 0");
  if (r->n_rig_pairs < 0 || (r->n_rig_pairs > 0 && !r->rig_pairs)) return fail(BA_EINVAL, "bad rig pairs");
  const int F = r->n_frames, nr = r->n_rig;
  for (int f = 0; f < F; ++f)
    if (int e = check_pose(r->vehicle_poses[f], "vehicle", f)) return e;
  for (int c = 0; c < nr; ++c)
    if (int e = check_pose(r->extrinsics[c], "extrinsic", c)) return e;
  {
    std::vector<int32_t> keys;
    for (int k = 0; k < r->n_rig_pairs; ++k) {
      const int c = r->rig_pairs[2 * k], d = r->rig_pairs[2 * k + 1];
      if (c < 0 || c >= nr || d < 0 || d >= nr || c == d) return fail(BA_EINVAL, "rig pair %d invalid", k);
      keys.push_back(std::min(c, d) * nr + std::max(c, d));
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return fail(BA_EINVAL, "a rig pair is given twice");
  }
  // the composed cameras, camera f * nr + c
  std::vector<ba_intrinsics> K((size_t)F * nr);
  std::vector<ba_pose> poses((size_t)F * nr);
  for (int f = 0; f < F; ++f) {
    double Tv[12];
    quat_to_pose12(r->vehicle_poses[f], Tv);
    for (int c = 0; c < nr; ++c) {
      double Te[12], Tc[12];
      quat_to_pose12(r->extrinsics[c], Te);
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          Tc[3 * i + j] = Te[3 * i] * Tv[j] + Te[3 * i + 1] * Tv[3 + j] + Te[3 * i + 2] * Tv[6 + j];
        Tc[9 + i] = Te[3 * i] * Tv[9] + Te[3 * i + 1] * Tv[10] + Te[3 * i + 2] * Tv[11] + Te[9 + i];
      }
      poses[(size_t)f * nr + c] = pose12_to_quat(Tc);
      K[(size_t)f * nr + c] = r->K[c];
    }
  }
  std::vector<ba_obs> obs(r->n_obs);
  for (int64_t k = 0; k < r->n_obs; ++k) {
    const ba_rig_obs &o = r->obs[k];
    if (o.frame < 0 || o.frame >= F || o.cam < 0 || o.cam >= nr)
      return fail(BA_EINVAL, "observation %lld: frame or rig camera out of range", (long long)k);
    obs[k] = ba_obs{o.frame * nr + o.cam, o.pt, o.u, o.v};
  }
  ba_problem_desc d{};
  d.n_cams = F * nr;
  d.K = K.data();
  d.K_per_cam = 1;
  d.poses = poses.data();
  d.cam_fixed = nullptr;
  d.n_pts = r->n_pts;
  d.points_xyz = r->points_xyz;
  d.n_obs = r->n_obs;
  d.obs = obs.data();
  return create_problem(&d, opt, hip_stream, nullptr, out, [&](ba_problem *p) {
    p->rig.reset(new RigPart());
    p->rig->F = F;
    p->rig->nr = nr;
    return build_rig(p, r, opt);
  });
}

int ba_rig_get_result(const ba_problem *pc, ba_pose *vehicles_out, ba_pose *extrinsics_out, double *points_out,
                      ba_report *rep) {
  ba_problem *p = const_cast<ba_problem *>(pc);
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (!p->rig) return fail(BA_EINVAL, "not a rig problem");
  if (p->pending)
    if (int e = ba_wait(p)) return e;
  if (vehicles_out || extrinsics_out) {
    const RigPart &rg = *p->rig;
    std::vector<double> buf(12 * (size_t)(rg.F + rg.nr));
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
      e = hipMemcpy(buf.data(), rg.dp.view.pose[p->dp.host_state.cur], buf.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rig pose download");
    if (vehicles_out)
      for (int f = 0; f < rg.F; ++f) vehicles_out[f] = pose12_to_quat(&buf[12 * (size_t)f]);
    if (extrinsics_out)
      for (int c = 0; c < rg.nr; ++c) extrinsics_out[c] = pose12_to_quat(&buf[12 * (size_t)(rg.F + c)]);
  }
  return p->dp.read_result(p->stream, nullptr, points_out, rep, p->solved, p->solve_ms, p->setup_ms);
}

int ba_pose_graph_create(const ba_pose_graph_desc *g, const ba_options *opt, void *hip_stream,
                         ba_problem **out) {
  if (out) *out = nullptr;
  if (!g) return fail(BA_EINVAL, "pose graph description is NULL");
  if (!opt) return fail(BA_EINVAL, "options are NULL");
  if (g->n_nodes < 2) return fail(BA_EINVAL, "n_nodes must be >= 2");
  if (g->n_edges < 1) return fail(BA_EINVAL, "n_edges must be >= 1");
  if (g->n_edges > (int64_t)INT32_MAX / 2) return fail(BA_EINVAL, "n_edges exceeds 2^30");
  if (!g->poses || !g->edges) return fail(BA_EINVAL, "NULL array in pose graph");
  if (opt->huber_delta > 0.0) return fail(BA_EINVAL, "a pose graph takes no robust loss (huber_delta must be <= 0)");
  if (opt->prior_seq != 0.0) return fail(BA_EINVAL, "a pose graph takes its relative terms as edges (prior_seq must be 0)");
  const int n = g->n_nodes;
  GraphEdges ge;
  ge.pairs.reserve(g->n_edges);
  ge.meas.resize(12 * (size_t)g->n_edges);
  ge.w.resize(2 * (size_t)g->n_edges);
  std::vector<int64_t> keys(g->n_edges);
  for (int64_t e = 0; e < g->n_edges; ++e) {
    const ba_pose_edge &ed = g->edges[e];
    if (ed.i < 0 || ed.i >= n || ed.j < 0 || ed.j >= n)
      return fail(BA_EINVAL, "edge %lld: node out of range", (long long)e);
    if (ed.i == ed.j) return fail(BA_EINVAL, "edge %lld joins node %d to itself", (long long)e, ed.i);
    if (int rc = check_pose(ed.meas, "edge", e)) return rc;
    if (!(std::isfinite(ed.w_rot) && std::isfinite(ed.w_trans) && ed.w_rot >= 0.0 && ed.w_trans >= 0.0 &&
          ed.w_rot + ed.w_trans > 0.0))
      return fail(BA_EINVAL, "edge %lld: weights must be finite, >= 0 and not both 0", (long long)e);
    ge.pairs.push_back(int2{ed.i, ed.j});
    quat_to_pose12(ed.meas, &ge.meas[12 * (size_t)e]);
    ge.w[2 * e] = ed.w_rot;
    ge.w[2 * e + 1] = ed.w_trans;
    keys[e] = (int64_t)std::min(ed.i, ed.j) * n + std::max(ed.i, ed.j);
  }
  std::sort(keys.begin(), keys.end());
  for (size_t e = 1; e < keys.size(); ++e)
    if (keys[e] == keys[e - 1])
      return fail(BA_EINVAL, "two edges join nodes %lld and %lld", (long long)(keys[e] / n), (long long)(keys[e] % n));
  const ba_intrinsics K1{1.0, 1.0, 0.0, 0.0};  // unused: a pose graph has no observations
  ba_problem_desc d{};
  d.n_cams = n;
  d.K = &K1;
  d.K_per_cam = 0;
  d.poses = g->poses;
  d.cam_fixed = g->node_fixed;
  d.n_pts = 0;
  d.points_xyz = nullptr;
  d.n_obs = 0;
  d.obs = nullptr;
  return create_problem(&d, opt, hip_stream, &ge, out);
}

int ba_solve_async(ba_problem *p) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (p->pending) return fail(BA_ESTATE, "a solve is already in flight");
  p->rep_ok = false;
  if (!p->rep_pin) {
    hipError_t ea = hipHostMalloc((void **)&p->rep_pin, p->dp.report_bytes(), hipHostMallocDefault);
    if (ea != hipSuccess) {
      p->rep_pin = nullptr;
      return hip_fail(ea, "report buffer");
    }
  }
  // the fresh state goes up from page-locked memory (the slot is free: no solve is in flight)
  const LMState fresh = p->dp.fresh_state();
  std::memcpy(p->rep_pin, &fresh, sizeof(LMState));
  hipError_t e = hipMemcpyAsync(p->dp.view.st, p->rep_pin, sizeof(LMState), hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) return hip_fail(e, "state upload");
  KernelTimer *tm = p->profiling ? &p->timer : nullptr;
  if (p->use_graph && !p->profiling) {
    // The kernels of a solve read their scalars from the device state, so the
    // same launch sequence serves every solve: capture it once and replay it.
    // (Per-kernel timing needs events between launches: profiled solves are
    // enqueued kernel by kernel instead.)
    if (!p->graph_exec) {
      e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture");
      hipError_t el = hipSuccess;
      for (int it = 0; it < p->dp.max_iters && el == hipSuccess; ++it)
        el = p->rig ? launch_rig_iteration(p->dp.precision, p->batch.plan, p->rig->batch.plan, p->dp.pcg_max,
                                           p->rig->sy.max_tcols, p->stream, nullptr)
                    : launch_lm_iteration(p->dp.precision, p->batch.plan, p->dp.pcg_max, p->dp.max_tcols,
                                          p->stream, nullptr);
      e = hipStreamEndCapture(p->stream, &p->graph);
      if (el != hipSuccess) return hip_fail(el, "kernel launch during capture");
      if (e != hipSuccess) return hip_fail(e, "graph capture");
      e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    }
    (void)hipEventRecord(p->ev0, p->stream);
    e = hipGraphLaunch(p->graph_exec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    (void)hipEventRecord(p->ev1, p->stream);
    // the final evaluation stays outside the graph and is not timed
    e = launch_eval(p->dp.precision, p->batch.plan, p->stream, nullptr);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    e = p->dp.enqueue_report(p->stream, p->rep_pin);
    if (e != hipSuccess) return hip_fail(e, "report copy");
    p->pending = true;
    return BA_OK;
  } else if (p->use_graph && !p->rig && p->timer.mask == (1u << K_PCG_CG) &&
             one_reduction_pcg(p->dp.precision, p->dp.max_tcols)) {
    // Only the PCG run is timed: the solve is replayed as graphs between the PCG runs
    // (their launches are the same in every iteration), with the timing events around
    // each run: two graph launches per LM iteration.
    if (!p->seg_exec[0]) {
      for (int part = 0; part < 4; ++part) {
        e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        // 0: before the first run; 1: a run; 2: after a run, then before the next; 3: after
        // the last run
        const int first = part == 0 ? LM_BEFORE_PCG : part == 1 ? LM_PCG : LM_AFTER_PCG;
        hipError_t el = launch_lm_iteration(p->dp.precision, p->batch.plan, p->dp.pcg_max, p->dp.max_tcols,
                                            p->stream, nullptr, first);
        if (part == 2 && el == hipSuccess)
          el = launch_lm_iteration(p->dp.precision, p->batch.plan, p->dp.pcg_max, p->dp.max_tcols, p->stream,
                                   nullptr, LM_BEFORE_PCG);
        e = hipStreamEndCapture(p->stream, &p->seg_graph[part]);
        if (el != hipSuccess) return hip_fail(el, "kernel launch during capture");
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        e = hipGraphInstantiate(&p->seg_exec[part], p->seg_graph[part], nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
      }
    }
    p->timer.reset();
    (void)hipEventRecord(p->ev0, p->stream);
    if (p->dp.max_iters > 0) e = hipGraphLaunch(p->seg_exec[0], p->stream);
    for (int it = 0; it < p->dp.max_iters && e == hipSuccess; ++it) {
      p->timer.begin(K_PCG_CG, p->stream, p->sy.pcg_resident ? 1 : p->dp.pcg_max);
      // the resident run is one kernel: launched directly, not as a one-node graph
      e = p->sy.pcg_resident ? launch_lm_iteration(p->dp.precision, p->batch.plan, p->dp.pcg_max, p->dp.max_tcols,
                                                   p->stream, nullptr, LM_PCG)
                             : hipGraphLaunch(p->seg_exec[1], p->stream);
      p->timer.end(K_PCG_CG, p->stream);
      if (e == hipSuccess) e = hipGraphLaunch(p->seg_exec[it + 1 < p->dp.max_iters ? 2 : 3], p->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "graph launch");
  } else {
    p->timer.reset();
    (void)hipEventRecord(p->ev0, p->stream);
    for (int it = 0; it < p->dp.max_iters; ++it) {
      e = p->rig ? launch_rig_iteration(p->dp.precision, p->batch.plan, p->rig->batch.plan, p->dp.pcg_max,
                                        p->rig->sy.max_tcols, p->stream, tm)
                 : launch_lm_iteration(p->dp.precision, p->batch.plan, p->dp.pcg_max, p->dp.max_tcols, p->stream, tm);
      if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
  }
  (void)hipEventRecord(p->ev1, p->stream);
  e = launch_eval(p->dp.precision, p->batch.plan, p->stream, tm);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  e = p->dp.enqueue_report(p->stream, p->rep_pin);
  if (e != hipSuccess) return hip_fail(e, "report copy");
  p->pending = true;
  return BA_OK;
}

int ba_wait(ba_problem *p) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (!p->pending) return BA_OK;
  hipError_t e = hipStreamSynchronize(p->stream);
  p->pending = false;
  if (e != hipSuccess) return hip_fail(e, "solve");
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, p->ev0, p->ev1);
  p->solve_ms = ms;
  std::memcpy(&p->dp.host_state, p->rep_pin + DevProblem::report_state_offset(), sizeof(LMState));
  p->rep_ok = true;
  if (p->profiling) p->timer.collect(p->kernel_ms, p->kernel_launches);
  p->solved = true;
  return BA_OK;
}

int ba_solve(ba_problem *p) {
  if (int e = ba_solve_async(p)) return e;
  return ba_wait(p);
}

int ba_get_result(const ba_problem *pc, ba_pose *poses_out, double *points_out, ba_report *rep) {
  ba_problem *p = const_cast<ba_problem *>(pc);
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (p->pending)
    if (int e = ba_wait(p)) return e;
  return p->dp.read_result(p->stream, poses_out, points_out, rep, p->solved, p->solve_ms, p->setup_ms,
                           p->rep_ok ? p->rep_pin : nullptr);
}

int ba_reset(ba_problem *p) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (p->pending) return fail(BA_ESTATE, "a solve is in flight");
  DevProblem &dp = p->dp;
  // one launch in place of two copies and a fill
  hipError_t e = launch_reset(dp.view.pose[0], (const double *)(dp.dev + dp.off.pose_init), 12 * (size_t)dp.C,
                              dp.view.X[0], (const double *)(dp.dev + dp.off.X_init), 3 * (size_t)dp.P,
                              dp.view.obs_act, (size_t)dp.N, p->stream);
  if (e == hipSuccess && p->rig) {
    DevProblem &rd = p->rig->dp;
    e = hipMemcpyAsync(rd.view.pose[0], rd.dev + rd.off.pose_init, 12 * (size_t)rd.C * 8, hipMemcpyDeviceToDevice,
                       p->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "reset");
  dp.n_active = dp.N;
  dp.host_state = LMState{};
  dp.host_state.cur = 0;
  p->solved = false;
  p->rep_ok = false;
  return BA_OK;
}

int ba_refine(ba_problem *p, int32_t n_stages, const ba_refine_stage *stages, int32_t rounds,
              ba_refine_round *hist) {
  if (n_stages < 1 || !stages) return fail(BA_EINVAL, "n_stages must be >= 1, with a stage array");
  if (rounds < 1) return fail(BA_EINVAL, "rounds must be >= 1");
  for (int i = 0; i < n_stages; ++i) {
    if (!std::isfinite(stages[i].huber_delta))
      return fail(BA_EINVAL, "stage %d: huber_delta must be finite", i);
    if (!std::isfinite(stages[i].cull_px) || !(stages[i].cull_px > 0.0))
      return fail(BA_EINVAL, "stage %d: cull_px must be positive and finite", i);
    if (stages[i].triangulation != BA_TRI_MIDPOINT && stages[i].triangulation != BA_TRI_DLT)
      return fail(BA_EINVAL, "stage %d: unknown triangulation method %d", i, stages[i].triangulation);
  }
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (p->pending) return fail(BA_ESTATE, "a solve is in flight");
  if (p->sy.N == 0) return fail(BA_EINVAL, "a pose graph has no observations to cull");
  if (p->rig) return fail(BA_EINVAL, "ba_refine does not take rig problems");
  DevProblem &dp = p->dp;
  const double huber0 = dp.huber;
  std::vector<int32_t> cnt(2 * (size_t)dp.view.n_pt_tiles);
  // the culling launches are timed with their own events when profiling selects them
  const bool time_cull = p->profiling && (p->timer.mask & (1u << K_CULL)) != 0;
  hipEvent_t c0 = nullptr, c1 = nullptr;
  if (time_cull) {
    hipError_t e = hipEventCreate(&c0);
    if (e == hipSuccess) e = hipEventCreate(&c1);
    if (e != hipSuccess) {
      if (c0) (void)hipEventDestroy(c0);
      return hip_fail(e, "event");
    }
  }
  double cull_ms = 0.0;
  int32_t n_cull = 0;
  int rc = BA_OK;
  for (int si = 0; si < n_stages && rc == BA_OK; ++si) {
    dp.huber = stages[si].huber_delta > 0.0 ? stages[si].huber_delta : 0.0;
    for (int r = 0; r < rounds; ++r) {
      rc = ba_solve(p);
      if (rc != BA_OK) break;
      const double tau = stages[si].cull_px;
      if (time_cull) (void)hipEventRecord(c0, p->stream);
      hipError_t e = launch_cull(dp.precision, p->batch.plan, tau * tau, stages[si].triangulation, p->stream, nullptr);
      if (time_cull) (void)hipEventRecord(c1, p->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(cnt.data(), dp.view.part_cull, cnt.size() * 4, hipMemcpyDeviceToHost, p->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
      if (e != hipSuccess) {
        rc = hip_fail(e, "culling");
        break;
      }
      if (time_cull) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, c0, c1);
        cull_ms += ms;
        ++n_cull;
      }
      int64_t na = 0, np = 0;
      for (size_t i = 0; i < cnt.size(); i += 2) {
        na += cnt[i];
        np += cnt[i + 1];
      }
      dp.n_active = na;
      if (hist) {
        ba_refine_round &h = hist[(size_t)si * rounds + r];
        std::memset(&h, 0, sizeof(h));
        h.stage = si;
        h.round = r;
        h.iters = dp.host_state.iter;
        h.status = dp.host_state.status;
        h.cost = dp.host_state.cost;
        h.n_active_obs = na;
        h.n_active_pts = (int32_t)np;
      }
    }
  }
  dp.huber = huber0;
  if (time_cull) {
    (void)hipEventDestroy(c0);
    (void)hipEventDestroy(c1);
    p->kernel_ms[K_CULL] = cull_ms;
    p->kernel_launches[K_CULL] = n_cull;
  }
  if (rc != BA_OK) return rc;
  // the report's rms and masked count describe the final state and mask
  hipError_t e = launch_eval(dp.precision, p->batch.plan, p->stream, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "evaluation");
  return BA_OK;
}

// Triangulation from scratch on the device (plain, or RANSAC when inlier_out is given).
static int triangulate_impl(const ba_problem_desc *d, int32_t method, bool ransac, double tau_px, int32_t n_hyp,
                            void *hip_stream, double *points_out, uint8_t *ok_out, uint8_t *inlier_out,
                            double *device_ms) {
  if (!d) return fail(BA_EINVAL, "problem description is NULL");
  if (method != BA_TRI_MIDPOINT && method != BA_TRI_DLT) return fail(BA_EINVAL, "unknown triangulation method %d", method);
  if (!points_out || !ok_out || (ransac && !inlier_out)) return fail(BA_EINVAL, "NULL output");
  if (ransac && !(std::isfinite(tau_px) && tau_px > 0.0)) return fail(BA_EINVAL, "tau_px must be positive and finite");
  if (ransac && (n_hyp < 1 || n_hyp > 4096)) return fail(BA_EINVAL, "n_hyp must be in 1..4096");
  if (d->n_cams < 1 || d->n_pts < 1 || d->n_obs < 1) return fail(BA_EINVAL, "n_cams, n_pts and n_obs must be >= 1");
  if (d->n_obs > (int64_t)INT32_MAX - 1) return fail(BA_EINVAL, "n_obs exceeds 2^31 - 2");
  if (!d->K || !d->poses || !d->obs) return fail(BA_EINVAL, "NULL array in problem");
  const int C = d->n_cams, P = d->n_pts;
  const int64_t N = d->n_obs;
  const int nK = d->K_per_cam ? C : 1;
  for (int i = 0; i < nK; ++i) {
    const ba_intrinsics &k = d->K[i];
    if (!(std::isfinite(k.fx) && std::isfinite(k.fy) && std::isfinite(k.cx) && std::isfinite(k.cy)) ||
        k.fx == 0.0 || k.fy == 0.0)
      return fail(BA_EINVAL, "intrinsics %d invalid", i);
  }
  for (int i = 0; i < C; ++i)
    if (int e = check_pose(d->poses[i], "camera", i)) return e;
  std::vector<int32_t> start(P + 1, 0);
  for (int64_t k = 0; k < N; ++k) {
    const ba_obs &o = d->obs[k];
    if (o.cam < 0 || o.cam >= C) return fail(BA_EINVAL, "observation %lld: camera %d out of range", (long long)k, o.cam);
    if (o.pt < 0 || o.pt >= P) return fail(BA_EINVAL, "observation %lld: point %d out of range", (long long)k, o.pt);
    if (!std::isfinite(o.u) || !std::isfinite(o.v)) return fail(BA_EINVAL, "observation %lld non-finite", (long long)k);
    start[o.pt + 1]++;
  }
  if (prepare_kernels() != 0) return fail(BA_EDEVICE, "no HIP device");
  for (int j = 0; j < P; ++j) start[j + 1] += start[j];
  // observations by point (stable), with normalized coordinates
  std::vector<int32_t> cam(N), fill(start.begin(), start.end() - 1), where(N);
  std::vector<double> xy(2 * N), poses(12 * (size_t)C), X(3 * (size_t)P), Kc(4 * (size_t)C);
  for (int i = 0; i < C; ++i) {
    const ba_intrinsics &K = d->K[d->K_per_cam ? i : 0];
    Kc[4 * i] = K.fx;
    Kc[4 * i + 1] = K.fy;
    Kc[4 * i + 2] = K.cx;
    Kc[4 * i + 3] = K.cy;
  }
  for (int64_t k = 0; k < N; ++k) {
    const ba_obs &o = d->obs[k];
    const ba_intrinsics &K = d->K[d->K_per_cam ? o.cam : 0];
    const int32_t at = fill[o.pt]++;
    where[k] = at;
    cam[at] = o.cam;
    xy[2 * (size_t)at] = (o.u - K.cx) / K.fx;
    xy[2 * (size_t)at + 1] = (o.v - K.cy) / K.fy;
  }
  for (int i = 0; i < C; ++i) quat_to_pose12(d->poses[i], &poses[12 * (size_t)i]);
  for (size_t i = 0; i < X.size(); ++i) X[i] = d->points_xyz ? d->points_xyz[i] : NAN;
  hipStream_t s = (hipStream_t)hip_stream;
  bool own = false;
  if (!s) {
    hipError_t e = hipStreamCreate(&s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    own = true;
  }
  const size_t b_start = ((size_t)(P + 1) * 4 + 255) & ~size_t(255), b_cam = ((size_t)N * 4 + 255) & ~size_t(255);
  const size_t b_xy = (size_t)N * 16, b_pose = (size_t)C * 96, b_X = (size_t)P * 24, b_ok = ((size_t)P + 255) & ~size_t(255);
  const size_t b_K = (size_t)C * 32, b_in = ((size_t)N + 255) & ~size_t(255);
  char *mem = nullptr;
  hipError_t e = hipMalloc((void **)&mem, b_start + b_cam + b_xy + b_pose + b_X + b_ok + b_K + b_in);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  char *q = mem;
  int32_t *d_start = (int32_t *)q;
  int32_t *d_cam = (int32_t *)(q += b_start);
  double *d_xy = (double *)(q += b_cam);
  double *d_pose = (double *)(q += b_xy);
  double *d_X = (double *)(q += b_pose);
  uint8_t *d_ok = (uint8_t *)(q += b_X);
  double *d_K = (double *)(q += b_ok);
  uint8_t *d_in = (uint8_t *)(q += b_K);
  if (e == hipSuccess) e = hipMemcpyAsync(d_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_cam, cam.data(), cam.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_xy, xy.data(), xy.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_pose, poses.data(), poses.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_X, X.data(), X.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_K, Kc.data(), Kc.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess)
    e = ransac ? launch_triangulate_ransac(P, d_start, d_cam, d_xy, d_pose, d_K, tau_px * tau_px, n_hyp, method, d_X,
                                           d_ok, d_in, s)
               : launch_triangulate(P, d_start, d_cam, d_xy, d_pose, method, d_X, d_ok, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipMemcpyAsync(points_out, d_X, X.size() * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ok_out, d_ok, (size_t)P, hipMemcpyDeviceToHost, s);
  std::vector<uint8_t> in_sorted(ransac ? N : 0);
  if (e == hipSuccess && ransac) e = hipMemcpyAsync(in_sorted.data(), d_in, (size_t)N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && ransac)
    for (int64_t k = 0; k < N; ++k) inlier_out[k] = in_sorted[where[k]];
  if (e == hipSuccess && device_ms) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *device_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (mem) (void)hipFree(mem);
  if (own) (void)hipStreamDestroy(s);
  if (e != hipSuccess) return hip_fail(e, "triangulation");
  return BA_OK;
}

int ba_triangulate(const ba_problem_desc *d, int32_t method, void *hip_stream, double *points_out,
                   uint8_t *ok_out, double *device_ms) {
  return triangulate_impl(d, method, false, 0.0, 0, hip_stream, points_out, ok_out, nullptr, device_ms);
}

int ba_triangulate_ransac(const ba_problem_desc *d, int32_t method, double tau_px, int32_t n_hyp, void *hip_stream,
                          double *points_out, uint8_t *ok_out, uint8_t *inlier_out, double *device_ms) {
  return triangulate_impl(d, method, true, tau_px, n_hyp, hip_stream, points_out, ok_out, inlier_out, device_ms);
}

int ba_get_active(const ba_problem *p, uint8_t *active_out) {
  if (!p || !active_out) return fail(BA_EINVAL, "NULL argument");
  if (p->pending) return fail(BA_ESTATE, "a solve is in flight");
  const DevProblem &dp = p->dp;
  if (dp.N == 0) return BA_OK;
  std::vector<uint8_t> buf((size_t)dp.N);
  hipError_t e = hipMemcpyAsync(buf.data(), dp.view.obs_act, buf.size(), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "mask download");
  for (size_t k = 0; k < buf.size(); ++k) active_out[dp.obs_order[k]] = buf[k];
  return BA_OK;
}

}  // extern "C"

static void fill_info(const Symbolic &sy, int64_t n_pairs, int precision, ba_problem_info *out) {
  out->n_cams = sy.C;
  out->n_free_cams = sy.Cf;
  out->n_pts = sy.P;
  out->n_obs = sy.N;
  out->n_pairs = n_pairs;
  out->n_up_blocks = sy.n_up;
  out->nnzb = sy.nnzb;
  out->n_free_obs = sy.Nf;
  out->precision = precision;
  out->schur_form = sy.dense ? 2 : sy.chunked ? 1 : 0;
  out->n_chunks = sy.chunked ? (int32_t)sy.ch_pt.size() - 1 : 0;
  out->n_entries = (int64_t)sy.ent_tgt.size();
  out->pcg_rows = sy.pcg_rows;
  out->pcg_resident = sy.pcg_resident ? (sy.pcg_coop ? 2 : 1) : 0;
}

extern "C" {

int ba_get_info(const ba_problem *p, ba_problem_info *out) {
  if (!p || !out) return fail(BA_EINVAL, "NULL argument");
  fill_info(p->sy, p->n_pairs, p->dp.precision, out);
  return BA_OK;
}

int ba_analyse(const ba_problem_desc *d, const ba_options *opt, ba_problem_info *info, int64_t *bytes) {
  if (!d || !opt) return fail(BA_EINVAL, "NULL argument");
  Symbolic sy;
  if (int e = analyse(d, opt, sy)) return e;
  if (info) fill_info(sy, sy.n_pairs, opt->precision, info);
  if (bytes) *bytes = (int64_t)DevProblem::bytes_for(sy, opt->precision, opt->max_iters);
  return BA_OK;
}

int64_t ba_problem_bytes(const ba_problem *p) { return p ? (int64_t)p->bytes : 0; }

void ba_destroy(ba_problem *p) {
  if (!p) return;
  if (p->pending) (void)hipStreamSynchronize(p->stream);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  for (int i = 0; i < 4; ++i) {
    if (p->seg_exec[i]) (void)hipGraphExecDestroy(p->seg_exec[i]);
    if (p->seg_graph[i]) (void)hipGraphDestroy(p->seg_graph[i]);
  }
  if (p->mem) (void)hipFree(p->mem);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->rep_pin) (void)hipHostFree(p->rep_pin);
  if (p->own_stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

int ba_set_profiling(ba_problem *p, int32_t mask, int32_t stride) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (stride < 1) return fail(BA_EINVAL, "stride must be >= 1");
  p->profiling = mask != 0;
  p->timer.mask = (uint32_t)mask;
  p->timer.stride = stride;
  return BA_OK;
}

int ba_set_barrier_polls(ba_problem *p, int32_t polls) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  if (polls < 0) return fail(BA_EINVAL, "polls must be >= 0");
  p->dp.bar_polls = polls;
  return BA_OK;
}

int ba_debug_iteration_export(ba_problem *p, ba_debug_iteration *out) {
  if (!p || !out) return fail(BA_EINVAL, "NULL argument");
  if (p->rig) return fail(BA_EINVAL, "the iteration export covers single-view problems, not vehicle rigs");
  if (p->pending) return fail(BA_ESTATE, "a solve is in flight");
  DevProblem &dp = p->dp;
  const ProbDev &v = dp.view;
  const int cur0 = dp.host_state.cur;
  dp.pending_state = dp.fresh_state();
  dp.pending_state.max_iters = 1;
  hipError_t e = hipMemcpyAsync(v.st, &dp.pending_state, sizeof(LMState), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = launch_lm_iteration(dp.precision, p->batch.plan, dp.pcg_max, dp.max_tcols, p->stream, nullptr);
  if (e == hipSuccess) e = launch_eval(dp.precision, p->batch.plan, p->stream, nullptr);
  double *dev = nullptr;  // records widened to FP64: r (2), J_c (12), J_p (6) per observation
  const size_t N = (size_t)v.N;
  if (e == hipSuccess && N && (out->r || out->Jc || out->Jp)) {
    e = hipMalloc(&dev, N * 20 * sizeof(double));
    if (e == hipSuccess) e = launch_export_records(dp.precision, v, cur0, dev, dev + 2 * N, dev + 14 * N, p->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e == hipSuccess) e = hipMemcpy(&dp.host_state, v.st, sizeof(LMState), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    if (dev) (void)hipFree(dev);
    return hip_fail(e, "iteration export");
  }
  p->solved = true;
  p->solve_ms = 0.0;
  const LMState &st = dp.host_state;
  out->lambda = dp.pending_state.lambda;
  out->accepted = st.accepted;
  int32_t pi = 0;
  e = hipMemcpy(&pi, v.iter_pcg, 4, hipMemcpyDeviceToHost);
  out->pcg_iters = pi;
  const size_t tb = compute_bytes(dp.precision);
  // a device array of the compute type, widened to FP64
  auto fetch = [&](const void *src, size_t n, std::vector<double> &dst) -> hipError_t {
    dst.resize(n);
    if (tb == 8) return hipMemcpy(dst.data(), src, n * 8, hipMemcpyDeviceToHost);
    std::vector<float> f(n);
    hipError_t r2 = hipMemcpy(f.data(), src, n * 4, hipMemcpyDeviceToHost);
    for (size_t i = 0; i < n; ++i) dst[i] = f[i];
    return r2;
  };
  const int Cf = v.Cf, P = v.P;
  std::vector<double> buf;
  if (e == hipSuccess && out->S_rowptr) std::copy(p->sy.S_rowptr.begin(), p->sy.S_rowptr.end(), out->S_rowptr);
  if (e == hipSuccess && out->S_col) std::copy(p->sy.S_col.begin(), p->sy.S_col.end(), out->S_col);
  if (e == hipSuccess && out->S && (e = fetch(v.S, 36 * (size_t)v.nnzb, buf)) == hipSuccess)
    std::copy(buf.begin(), buf.end(), out->S);
  const std::pair<const void *, double *> cams[3] = {{v.brhs, out->b}, {v.gc, out->gc}, {v.x, out->dc}};
  for (const auto &c : cams)
    if (e == hipSuccess && c.second && (e = fetch(c.first, 6 * (size_t)Cf, buf)) == hipSuccess)
      std::copy(buf.begin(), buf.end(), c.second);
  if (e == hipSuccess && out->gp && P > 0 && (e = fetch(v.gp, 3 * (size_t)P, buf)) == hipSuccess)
    for (int j = 0; j < P; ++j)
      for (int m = 0; m < 3; ++m) out->gp[3 * (size_t)dp.pt_order[j] + m] = buf[3 * (size_t)j + m];
  if (e == hipSuccess && out->dp && P > 0) {
    std::vector<double> X0(3 * (size_t)P), X1(3 * (size_t)P);
    e = hipMemcpy(X0.data(), v.X[cur0], X0.size() * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(X1.data(), v.X[1 - cur0], X1.size() * 8, hipMemcpyDeviceToHost);
    for (int j = 0; j < P && e == hipSuccess; ++j)
      for (int m = 0; m < 3; ++m)
        out->dp[3 * (size_t)dp.pt_order[j] + m] = X1[3 * (size_t)j + m] - X0[3 * (size_t)j + m];
  }
  if (e == hipSuccess && dev) {
    std::vector<double> rec(N * 20);
    e = hipMemcpy(rec.data(), dev, rec.size() * 8, hipMemcpyDeviceToHost);
    for (size_t k = 0; k < N && e == hipSuccess; ++k) {
      const size_t o = (size_t)dp.obs_order[k];
      if (out->r)
        for (int i = 0; i < 2; ++i) out->r[2 * o + i] = rec[2 * k + i];
      if (out->Jc)
        for (int i = 0; i < 12; ++i) out->Jc[12 * o + i] = rec[2 * N + 12 * k + i];
      if (out->Jp)
        for (int i = 0; i < 6; ++i) out->Jp[6 * o + i] = rec[14 * N + 6 * k + i];
    }
  }
  if (dev) (void)hipFree(dev);
  if (e != hipSuccess) return hip_fail(e, "iteration export");
  return BA_OK;
}

int ba_get_kernel_times(const ba_problem *p, int32_t max_kernels, const char **names, double *ms,
                        int32_t *launches, int32_t *n_out) {
  if (!p) return fail(BA_EINVAL, "problem is NULL");
  const int n = std::min<int>(max_kernels, K_NUM_KERNELS);
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = kKernelNames[i];
    if (ms) ms[i] = p->kernel_ms[i];
    if (launches) launches[i] = p->kernel_launches[i];
  }
  if (n_out) *n_out = n;
  return BA_OK;
}

}  // extern "C"

namespace bax {

namespace {
// Byte offsets of the result staging layout (each part 8-byte aligned).
struct ResultLayout {
  size_t st, pose[2], X[2], sq, nm, ic, pi, total;
  ResultLayout(int C, int P, int npt, int max_iters) {
    size_t o = 0;
    auto take = [&](size_t b) {
      const size_t r = o;
      o += (b + 7) & ~size_t(7);
      return r;
    };
    st = take(sizeof(LMState));
    for (int b = 0; b < 2; ++b) pose[b] = take(12 * (size_t)C * 8);
    for (int b = 0; b < 2; ++b) X[b] = take(3 * (size_t)P * 8);
    sq = take((size_t)npt * 8);
    nm = take((size_t)npt * 4);
    ic = take(((size_t)max_iters + 1) * 8);
    pi = take((size_t)max_iters * 4);
    total = o;
  }
};
}  // namespace

size_t DevProblem::result_bytes() const { return ResultLayout(C, P, view.n_pt_tiles, max_iters).total; }


size_t DevProblem::report_bytes() const { return ReportLayout(view.n_pt_tiles, max_iters).total; }
size_t DevProblem::report_state_offset() { return ReportLayout(0, 0).st; }

hipError_t DevProblem::enqueue_report(hipStream_t s, char *pinned) const {
  // the device block has the same layout (plan): one copy from the state to the end
  const ReportLayout L(view.n_pt_tiles, max_iters);
  return hipMemcpyAsync(pinned + L.st, view.st, L.total - L.st, hipMemcpyDeviceToHost, s);
}

hipError_t DevProblem::enqueue_result(hipStream_t s, char *pinned) const {
  const ResultLayout L(C, P, view.n_pt_tiles, max_iters);
  hipError_t e = hipMemcpyAsync(pinned + L.st, view.st, sizeof(LMState), hipMemcpyDeviceToHost, s);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipMemcpyAsync(pinned + L.pose[b], view.pose[b], 12 * (size_t)C * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && P > 0) e = hipMemcpyAsync(pinned + L.X[b], view.X[b], 3 * (size_t)P * 8, hipMemcpyDeviceToHost, s);
  }
  const size_t npt = (size_t)view.n_pt_tiles;
  if (e == hipSuccess && npt) e = hipMemcpyAsync(pinned + L.sq, view.part_sq, npt * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && npt) e = hipMemcpyAsync(pinned + L.nm, view.part_masked, npt * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pinned + L.ic, view.iter_cost, ((size_t)max_iters + 1) * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pinned + L.pi, view.iter_pcg, (size_t)max_iters * 4, hipMemcpyDeviceToHost, s);
  return e;
}

void DevProblem::finish_result(const char *pinned, ba_pose *poses_out, double *points_out, ba_report *rep) const {
  const ResultLayout L(C, P, view.n_pt_tiles, max_iters);
  LMState st;
  std::memcpy(&st, pinned + L.st, sizeof(LMState));
  const int cur = st.cur;
  const double *pose = (const double *)(pinned + L.pose[cur]);
  const double *X = (const double *)(pinned + L.X[cur]);
  if (poses_out)
    for (int i = 0; i < C; ++i) poses_out[i] = pose12_to_quat(pose + 12 * (size_t)i);
  if (points_out)
    for (int j = 0; j < P; ++j)
      for (int m = 0; m < 3; ++m) points_out[3 * (size_t)pt_order[j] + m] = X[3 * (size_t)j + m];
  if (!rep) return;
  double *ic = rep->iter_cost;
  int32_t *pi = rep->pcg_iters;
  std::memset(rep, 0, sizeof(*rep));
  rep->iter_cost = ic;
  rep->pcg_iters = pi;
  rep->iters = st.iter;
  rep->accepted = st.accepted;
  rep->status = st.status;
  rep->cost0 = st.cost0;
  rep->cost = st.cost;
  rep->lambda = st.lambda;
  const double *sq = (const double *)(pinned + L.sq);
  const int32_t *nm = (const int32_t *)(pinned + L.nm);
  double tot = 0.0;
  int64_t masked = 0;
  for (int i = 0; i < view.n_pt_tiles; ++i) {
    tot += sq[i];
    masked += nm[i];
  }
  rep->n_masked = (int32_t)masked;
  rep->rms_px = (n_active - masked) > 0 ? std::sqrt(tot / (double)(n_active - masked)) : 0.0;
  if (ic) std::memcpy(ic, pinned + L.ic, ((size_t)st.iter + 1) * 8);
  if (pi && st.iter > 0) std::memcpy(pi, pinned + L.pi, (size_t)st.iter * 4);
}

int DevProblem::read_result(hipStream_t s, ba_pose *poses_out, double *points_out, ba_report *rep,
                            bool solved, double solve_ms, double setup_ms, const char *rep_pin) {
  hipError_t e = hipSuccess;
  if (!rep_pin || poses_out || points_out) {  // a staged report has landed already
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "sync");
  }
  const int cur = host_state.cur;
  if (poses_out) {
    std::vector<double> buf(12 * (size_t)C);
    e = hipMemcpy(buf.data(), view.pose[cur], buf.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "pose download");
    for (int i = 0; i < C; ++i) poses_out[i] = pose12_to_quat(&buf[12 * (size_t)i]);
  }
  if (points_out && P > 0) {
    std::vector<double> buf(3 * (size_t)P);
    e = hipMemcpy(buf.data(), view.X[cur], buf.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "point download");
    for (int j = 0; j < P; ++j)
      for (int m = 0; m < 3; ++m) points_out[3 * (size_t)pt_order[j] + m] = buf[3 * (size_t)j + m];
  }
  if (rep) {
    double *ic = rep->iter_cost;
    int32_t *pi = rep->pcg_iters;
    std::memset(rep, 0, sizeof(*rep));
    rep->iter_cost = ic;
    rep->pcg_iters = pi;
    rep->setup_ms = setup_ms;
    if (solved) {
      const LMState &st = host_state;
      rep->iters = st.iter;
      rep->accepted = st.accepted;
      rep->status = st.status;
      rep->cost0 = st.cost0;
      rep->cost = st.cost;
      rep->lambda = st.lambda;
      rep->solve_ms = solve_ms;
      const int npt = view.n_pt_tiles;
      const ReportLayout RL(npt, max_iters);
      std::vector<double> sq(npt);
      std::vector<int32_t> nm(npt);
      if (rep_pin) {
        std::memcpy(sq.data(), rep_pin + RL.sq, npt * 8);
        std::memcpy(nm.data(), rep_pin + RL.nm, npt * 4);
      } else {
        e = hipMemcpy(sq.data(), view.part_sq, npt * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(nm.data(), view.part_masked, npt * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "report download");
      }
      double tot = 0.0;
      int64_t masked = 0;
      for (int i = 0; i < npt; ++i) {
        tot += sq[i];
        masked += nm[i];
      }
      rep->n_masked = (int32_t)masked;
      rep->rms_px = (n_active - masked) > 0 ? std::sqrt(tot / (double)(n_active - masked)) : 0.0;
      if (ic) {
        e = rep_pin ? (std::memcpy(ic, rep_pin + RL.ic, (st.iter + 1) * 8), hipSuccess)
                    : hipMemcpy(ic, view.iter_cost, (st.iter + 1) * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "report download");
      }
      if (pi && st.iter > 0) {
        e = rep_pin ? (std::memcpy(pi, rep_pin + RL.pi, st.iter * 4), hipSuccess)
                    : hipMemcpy(pi, view.iter_pcg, st.iter * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "report download");
      }
    }
  }
  return BA_OK;
}

}  // namespace bax
