// Serving loop: continuous batching of bundle-adjustment and pose-only
// requests under a device-memory budget.
//
// The server owns one device block of budget bytes, carved by a first-fit
// allocator.  A scheduler thread repeats: admit queued requests in arrival
// order while a slot is free and their bytes fit; launch one LM iteration for
// every admitted problem at once (one launch per kernel for the whole batch);
// run all admitted pose-only requests in one launch; read back which problems
// finished; evaluate and download those, free their bytes and slots.  A
// problem's kernels read only its own data and reduce in a fixed order, so its
// result does not depend on the batch it shares.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_runtime.h"

namespace bax {

hipError_t launch_gather_iters(const BatchPlan &bp, int32_t *out, hipStream_t s);

namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap) with coalescing of free ranges.
struct Arena {
  std::map<size_t, size_t> free_;  // offset -> size
  size_t cap = 0, used = 0;
  void reset(size_t c) {
    cap = c;
    used = 0;
    free_.clear();
    free_[0] = c;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
  bool alloc(size_t bytes, size_t &off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  int64_t ticket = 0;
  bool pose = false;
  bool holds_block = false;  // owns [off, off + bytes) of the arena
  ba_options opt{};
  size_t bytes = 0, off = 0;
  double t_submit = 0, t_done = 0;
  bool done = false;
  int rc = BA_OK;
  // bundle adjustment
  Symbolic sy;
  std::vector<ba_intrinsics> K;
  int32_t K_per_cam = 0;
  std::vector<ba_pose> poses;
  std::vector<double> pts;
  DevProblem dp;
  // pose-only
  ba_pose_request preq{};
  std::vector<double> pX, puv;
  // results
  std::vector<ba_pose> out_poses;
  std::vector<double> out_pts;
  std::vector<double> iter_cost;
  std::vector<int32_t> iter_pcg;
  ba_report rep{};
};
using ReqP = std::shared_ptr<Req>;

}  // namespace
}  // namespace bax

using namespace bax;

struct ba_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ReqP> queue;
  std::vector<ReqP> active;
  std::unordered_map<int64_t, ReqP> tickets;
  Arena arena;
  void *mem = nullptr;
  int32_t *d_iters = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_slots = 1;
  int precision = BA_PREC_F32;
  int64_t budget = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  Batch batch;
  // statistics
  std::vector<double> lat_ms;
  double first_submit = -1, last_done = -1;
  int64_t n_done = 0;
  size_t peak = 0;
  int fatal = BA_OK;
  void loop();
  void finish(const std::vector<ReqP> &done_now);
};

void ba_server::finish(const std::vector<ReqP> &done_now) {
  std::lock_guard<std::mutex> lk(mu);
  for (auto &r : done_now) {
    r->done = true;
    r->t_done = now_ms();
    if (r->holds_block) arena.release(r->off, r->bytes);
    r->holds_block = false;
    lat_ms.push_back(r->t_done - r->t_submit);
    last_done = r->t_done;
    ++n_done;
  }
  cv_done.notify_all();
}

void ba_server::loop() {
  std::vector<int32_t> iters;
  bool dirty = true;
  while (true) {
    std::vector<ReqP> admitted, pose_now;
    size_t pose_bytes = 0;
    size_t pb_off = 0;
    bool pb_ok = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop && queue.empty() && active.empty()) break;
      // admission in arrival order; a request that does not fit blocks the ones behind it
      while (!queue.empty() && fatal == BA_OK) {
        ReqP r = queue.front();
        if (r->pose) {
          // pose requests of one step share one block; 512 bytes cover its alignment
          if (pose_bytes + r->bytes + 512 > arena.largest_free()) break;
          pose_bytes += r->bytes;
          pose_now.push_back(r);
          queue.pop_front();
          continue;
        }
        if (!pose_now.empty()) break;  // keep arrival order across the two kinds
        if ((int)(active.size() + admitted.size()) >= max_slots) break;
        size_t off;
        if (!arena.alloc(r->bytes, off)) break;
        r->off = off;
        r->holds_block = true;
        admitted.push_back(r);
        queue.pop_front();
      }
      if (!pose_now.empty()) pb_ok = arena.alloc(pose_bytes + 512, pb_off);
      peak = std::max(peak, arena.used);
    }
    std::vector<ReqP> failed;
    for (auto &r : admitted) {
      ba_problem_desc d{};
      d.n_cams = r->sy.C;
      d.K = r->K.data();
      d.K_per_cam = r->K_per_cam;
      d.poses = r->poses.data();
      d.n_pts = r->sy.P;
      d.points_xyz = r->pts.data();
      d.n_obs = r->sy.N;
      int rc = r->dp.init(r->sy, &d, &r->opt, (char *)mem + r->off, stream);
      if (rc == BA_OK) {
        r->dp.pending_state = r->dp.fresh_state();
        hipError_t e = hipMemcpyAsync(r->dp.view.st, &r->dp.pending_state, sizeof(LMState),
                                      hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) rc = hip_fail(e, "server state upload");
      }
      if (rc != BA_OK) {
        r->rc = rc;
        failed.push_back(r);
      } else {
        std::lock_guard<std::mutex> lk(mu);
        active.push_back(r);
        dirty = true;
      }
    }
    if (!failed.empty()) finish(failed);
    int pcg_max = 1;
    if (!active.empty()) {
      if (dirty) {
        batch.clear();
        for (size_t i = 0; i < active.size(); ++i) batch.add(active[i]->dp.view, (int)i);
        if (batch.upload(stream) != BA_OK) {
          fatal = BA_EDEVICE;
        }
        dirty = false;
      }
      int max_cf = 1;
      for (auto &r : active) {
        pcg_max = std::max(pcg_max, r->dp.pcg_max);
        max_cf = std::max(max_cf, (int)r->dp.max_tcols);
      }
      if (fatal == BA_OK &&
          launch_lm_iteration(precision, batch.plan, pcg_max, max_cf, stream, nullptr) != hipSuccess)
        fatal = BA_EDEVICE;
      if (fatal == BA_OK && launch_gather_iters(batch.plan, d_iters, stream) != hipSuccess)
        fatal = BA_EDEVICE;
    }
    PoseBatch pb;
    if (!pose_now.empty() && fatal == BA_OK) {
      std::vector<const ba_pose_request *> rp;
      std::vector<const ba_options *> ro;
      for (auto &r : pose_now) {
        rp.push_back(&r->preq);
        ro.push_back(&r->opt);
      }
      pb.pack(rp, ro);
      if (pb_ok && pb.run((char *)mem + pb_off, stream, nullptr) != BA_OK)
        fatal = BA_EDEVICE;
    }
    iters.assign(active.size(), 0);
    if (!active.empty() && fatal == BA_OK)
      if (hipMemcpyAsync(iters.data(), d_iters, active.size() * 4, hipMemcpyDeviceToHost, stream) != hipSuccess)
        fatal = BA_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) fatal = BA_EDEVICE;
    for (auto &r : admitted) {
      r->dp.staging_f.clear();
      r->dp.staging_d.clear();
      r->sy.pairs = std::vector<int2>();
      r->sy.ent_items = std::vector<uint32_t>();
    }
    if (!pose_now.empty()) {
      if (pb_ok) {
        std::lock_guard<std::mutex> lk(mu);
        arena.release(pb_off, pose_bytes + 512);
      }
      for (size_t i = 0; i < pose_now.size(); ++i) {
        Req &r = *pose_now[i];
        if (!pb_ok || fatal != BA_OK) {
          r.rc = pb_ok ? fatal : BA_ENOMEM;
          continue;
        }
        r.out_poses.assign(1, pose12_to_quat(pb.hdr[i].pose));
        r.rep.iters = r.opt.max_iters;
        r.rep.status = pb.hdr[i].status;
        r.rep.cost = pb.hdr[i].cost;
      }
      finish(pose_now);
    }
    if (fatal != BA_OK) {
      // fail everything still pending; the device state is unknown
      std::vector<ReqP> all;
      {
        std::lock_guard<std::mutex> lk(mu);
        all.insert(all.end(), active.begin(), active.end());
        all.insert(all.end(), queue.begin(), queue.end());
        active.clear();
        queue.clear();
      }
      for (auto &r : all) r->rc = fatal;
      finish(all);
      continue;
    }
    // retire finished problems
    std::vector<ReqP> fin;
    std::vector<ReqP> keep;
    for (size_t i = 0; i < active.size(); ++i) {
      if (iters[i] >= active[i]->dp.max_iters) fin.push_back(active[i]);
      else keep.push_back(active[i]);
    }
    if (!fin.empty()) {
      Batch fb;
      for (auto &r : fin) fb.add(r->dp.view, 0);
      int rc = fb.upload(stream);
      if (rc == BA_OK && launch_eval(precision, fb.plan, stream, nullptr) != hipSuccess) rc = BA_EDEVICE;
      for (auto &r : fin) {
        if (hipMemcpyAsync(&r->dp.host_state, r->dp.view.st, sizeof(LMState), hipMemcpyDeviceToHost, stream) != hipSuccess)
          rc = BA_EDEVICE;
      }
      if (hipStreamSynchronize(stream) != hipSuccess) rc = BA_EDEVICE;
      for (auto &r : fin) {
        if (rc != BA_OK) {
          r->rc = rc;
          continue;
        }
        r->out_poses.resize(r->sy.C);
        r->out_pts.resize(3 * (size_t)r->sy.P);
        r->iter_cost.resize(r->dp.max_iters + 1);
        r->iter_pcg.resize(r->dp.max_iters);
        r->rep.iter_cost = r->iter_cost.data();
        r->rep.pcg_iters = r->iter_pcg.data();
        r->rc = r->dp.read_result(stream, r->out_poses.data(), r->out_pts.data(), &r->rep, true, 0.0, 0.0);
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        active = keep;
      }
      dirty = true;
      finish(fin);
    }
  }
}

extern "C" {

int ba_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int32_t precision, void *hip_stream,
                     ba_server **out) {
  if (!out) return fail(BA_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < (1 << 20)) return fail(BA_EINVAL, "budget below 1 MiB");
  if (max_slots < 1 || max_slots > 4096) return fail(BA_EINVAL, "max_slots outside [1, 4096]");
  if (precision < BA_PREC_F64 || precision > BA_PREC_BF16J) return fail(BA_EINVAL, "unknown precision");
  if (prepare_kernels() != 0) return fail(BA_EDEVICE, "no HIP device");
  std::unique_ptr<ba_server> s(new ba_server());
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->precision = precision;
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreate(&s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    s->own_stream = true;
  }
  hipError_t e = hipMalloc(&s->mem, (size_t)hbm_budget_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_iters, (size_t)max_slots * 4);
  if (e != hipSuccess) {
    if (s->mem) (void)hipFree(s->mem);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    return hip_fail(e, "server arena allocation");
  }
  s->arena.reset((size_t)hbm_budget_bytes);
  ba_server *raw = s.get();
  s->th = std::thread([raw] { raw->loop(); });
  *out = s.release();
  return BA_OK;
}

int ba_server_submit(ba_server *s, const ba_problem_desc *d, const ba_options *opt, int64_t *ticket) {
  if (!s || !ticket) return fail(BA_EINVAL, "NULL argument");
  if (opt && opt->precision != s->precision)
    return fail(BA_EINVAL, "request precision %d differs from the server's %d", opt->precision, s->precision);
  auto r = std::make_shared<Req>();
  r->t_submit = now_ms();
  if (int e = analyse(d, opt, r->sy)) return e;
  r->opt = *opt;
  r->bytes = DevProblem::bytes_for(r->sy, opt->precision, opt->max_iters);
  if ((int64_t)r->bytes > s->budget)
    return fail(BA_ENOMEM, "problem needs %lld bytes, budget is %lld", (long long)r->bytes, (long long)s->budget);
  r->K_per_cam = d->K_per_cam;
  r->K.assign(d->K, d->K + (d->K_per_cam ? d->n_cams : 1));
  r->poses.assign(d->poses, d->poses + d->n_cams);
  r->pts.assign(d->points_xyz, d->points_xyz + 3 * (size_t)d->n_pts);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BA_ESTATE, "server is shutting down");
  r->ticket = s->next_ticket++;
  if (s->first_submit < 0) s->first_submit = r->t_submit;
  s->tickets[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return BA_OK;
}

int ba_server_submit_pose(ba_server *s, const ba_pose_request *req, const ba_options *opt, int64_t *ticket) {
  if (!s || !req || !ticket) return fail(BA_EINVAL, "NULL argument");
  if (int e = check_options(opt, true)) return e;
  if (int e = check_pose_request(*req, 0)) return e;
  auto r = std::make_shared<Req>();
  r->t_submit = now_ms();
  r->pose = true;
  r->opt = *opt;
  r->pX.assign(req->X, req->X + 3 * (size_t)req->n);
  r->puv.assign(req->uv, req->uv + 2 * (size_t)req->n);
  r->preq = *req;
  r->preq.X = r->pX.data();
  r->preq.uv = r->puv.data();
  r->bytes = sizeof(PoseDev) + (size_t)req->n * (3 * 8 + 2 * 4);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BA_ESTATE, "server is shutting down");
  r->ticket = s->next_ticket++;
  if (s->first_submit < 0) s->first_submit = r->t_submit;
  s->tickets[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return BA_OK;
}

int ba_server_wait(ba_server *s, int64_t ticket, ba_pose *poses_out, double *points_out, ba_report *rep) {
  if (!s) return fail(BA_EINVAL, "server is NULL");
  ReqP r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(BA_EINVAL, "unknown or already collected ticket %lld", (long long)ticket);
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->tickets.erase(it);
  }
  if (r->rc != BA_OK) return fail(r->rc, "request %lld failed", (long long)ticket);
  if (poses_out) std::copy(r->out_poses.begin(), r->out_poses.end(), poses_out);
  if (points_out && !r->pose) std::copy(r->out_pts.begin(), r->out_pts.end(), points_out);
  if (rep) {
    double *ic = rep->iter_cost;
    int32_t *pi = rep->pcg_iters;
    *rep = r->rep;
    rep->iter_cost = ic;
    rep->pcg_iters = pi;
    rep->solve_ms = r->t_done - r->t_submit;
    if (ic && !r->pose) std::copy(r->iter_cost.begin(), r->iter_cost.begin() + r->rep.iters + 1, ic);
    if (pi && !r->pose) std::copy(r->iter_pcg.begin(), r->iter_pcg.begin() + r->rep.iters, pi);
  }
  return BA_OK;
}

int ba_server_stats(ba_server *s, ba_server_stats_t *out) {
  if (!s || !out) return fail(BA_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  std::vector<double> l = s->lat_ms;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const double pos = q * (l.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
  };
  out->p50_ms = pct(0.50);
  out->p99_ms = pct(0.99);
  out->done = s->n_done;
  out->queued = (int64_t)s->queue.size();
  out->active = (int64_t)s->active.size();
  out->bytes_in_use = (int64_t)s->arena.used;
  out->peak_bytes = (int64_t)s->peak;
  const double span = s->last_done - s->first_submit;
  out->solves_per_s = (span > 0 && s->n_done > 0) ? s->n_done / (span / 1000.0) : 0.0;
  return BA_OK;
}

void ba_server_destroy(ba_server *s) {
  if (!s) return;
  std::vector<ReqP> cancelled;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    cancelled.assign(s->queue.begin(), s->queue.end());
    s->queue.clear();
    for (auto &r : cancelled) {
      r->rc = BA_ESTATE;
      r->done = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(s->mem);
  (void)hipFree(s->d_iters);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
