// Serving loop: continuous batching of bundle-adjustment and pose-only
// requests under a device-memory budget.
//
// The server owns one device block of budget bytes, carved by a first-fit
// allocator.  A submitted problem is validated and copied in the caller's
// thread; its symbolic analysis runs on a pool of host threads.  A scheduler
// thread repeats: admit analysed problems in ticket order while a slot is free
// and their bytes fit (a later problem that fits may pass one that does not, a
// bounded number of times); launch one LM iteration for every admitted problem at
// once (one launch per kernel for the whole batch); run all queued pose-only
// requests in one launch.  Each launch sequence advances every problem it holds
// by exactly one iteration, so the host counts iterations itself and never waits
// on the device to learn which problems finished: it queues their evaluation
// and result copies into page-locked buffers behind an event, frees their bytes
// and slots, and hands the results over once the event has passed.  At most two
// launch sequences are in flight.  A problem's kernels read only its own data
// and reduce in a fixed order, so its result does not depend on the batch it shares.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_runtime.h"

namespace bax {


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
  std::string err;
  // bundle adjustment: the caller's arrays, copied at submission
  int32_t n_cams = 0, n_pts = 0, K_per_cam = 0;
  std::vector<ba_intrinsics> K;
  std::vector<ba_pose> poses;
  std::vector<uint8_t> fixed;
  std::vector<double> pts;
  std::vector<ba_obs> obs;
  Symbolic sy;
  DevProblem dp;
  int steps = 0;  // LM iterations launched for it
  int passed = 0; // later problems admitted while it waited for memory
  // pose-only
  ba_pose_request preq{};
  std::vector<double> pX, puv;
  // results
  std::vector<ba_pose> out_poses;
  std::vector<double> out_pts;
  std::vector<double> iter_cost;
  std::vector<int32_t> iter_pcg;
  ba_report rep{};

  ba_problem_desc desc() const {
    ba_problem_desc d{};
    d.n_cams = n_cams;
    d.K = K.data();
    d.K_per_cam = K_per_cam;
    d.poses = poses.data();
    d.cam_fixed = fixed.empty() ? nullptr : fixed.data();
    d.n_pts = n_pts;
    d.points_xyz = pts.data();
    d.n_obs = (int64_t)obs.size();
    d.obs = obs.data();
    return d;
  }
};
using ReqP = std::shared_ptr<Req>;

// Page-locked host memory for result copies, reused across requests.
struct Pinned {
  char *p = nullptr;
  size_t n = 0;
};

// Result copies of the problems that finished in one launch sequence, in flight.
struct Completion {
  std::vector<ReqP> reqs;
  std::vector<Pinned> bufs;
  hipEvent_t ev = nullptr;
};

constexpr int kLookahead = 2;  // launch sequences the scheduler may run ahead of the device
// Later problems that may be admitted ahead of one that waits for memory; past that,
// admission waits for it, so that a large request is not starved by small ones.
constexpr int kMaxPassed = 16;

// A lower bound of the device bytes a problem needs, from its sizes alone: its
// observation arrays and its point and camera state.
size_t min_problem_bytes(int64_t n_obs, int32_t n_pts, int32_t n_cams, int precision) {
  const size_t T = compute_bytes(precision);
  return (size_t)n_obs * (4 + 4 + 2 * T + 4 + 1) + (size_t)n_pts * (3 * 8 * 3 + 15 * T) +
         (size_t)n_cams * 12 * 8 * 3;
}

}  // namespace
}  // namespace bax

using namespace bax;

struct ba_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_ana;
  std::deque<ReqP> ana_q;            // submitted problems awaiting their analysis
  int analysing = 0;                 // problems being analysed now
  std::map<int64_t, ReqP> ready;     // analysed problems, admitted in ticket order
  std::deque<ReqP> pose_q;
  std::deque<ReqP> up_q;             // admitted problems awaiting their upload
  int uploading = 0;                 // problems being uploaded now
  std::vector<ReqP> uploaded;        // on the device, to join the batch at the next step
  std::vector<ReqP> active;
  std::deque<Completion> completing;  // scheduler thread only
  std::unordered_map<int64_t, ReqP> tickets;
  Arena arena;
  void *mem = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t up_stream = nullptr;   // uploads of admitted problems, beside the compute stream
  bool own_stream = false;
  int max_slots = 1;
  int precision = BA_PREC_F32;
  int64_t budget = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  std::thread th, up_th;
  std::vector<std::thread> ana_th;
  Batch batch, fin_batch;
  hipEvent_t ev_step[kLookahead] = {};
  int64_t n_steps = 0;
  std::vector<Pinned> pinned_free;
  // statistics
  std::vector<double> lat_ms;
  double first_submit = -1, last_done = -1;
  int64_t n_done = 0;
  size_t peak = 0;
  int fatal = BA_OK;
  void loop();
  void ana_loop();
  void up_loop();
  void finish(const std::vector<ReqP> &done_now);
  Pinned take_pinned(size_t n);
  int complete(bool block);
  bool idle_locked() const {
    return ana_q.empty() && analysing == 0 && ready.empty() && pose_q.empty() && up_q.empty() &&
           uploading == 0 && uploaded.empty() && active.empty() && completing.empty();
  }
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

Pinned ba_server::take_pinned(size_t n) {
  for (size_t i = 0; i < pinned_free.size(); ++i)
    if (pinned_free[i].n >= n) {
      Pinned b = pinned_free[i];
      pinned_free.erase(pinned_free.begin() + i);
      return b;
    }
  Pinned b;
  const size_t want = std::max<size_t>(n, 1 << 16);
  if (hipHostMalloc((void **)&b.p, want, hipHostMallocDefault) == hipSuccess) b.n = want;
  else b.p = nullptr;
  return b;
}

// Symbolic analysis of submitted problems, off the caller's thread and the scheduler's.
void ba_server::ana_loop() {
  while (true) {
    ReqP r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_ana.wait(lk, [&] { return stop || !ana_q.empty(); });
      if (ana_q.empty()) return;
      r = ana_q.front();
      ana_q.pop_front();
      ++analysing;
    }
    const ba_problem_desc d = r->desc();
    int rc = analyse(&d, &r->opt, r->sy);
    if (rc == BA_OK) {
      r->bytes = DevProblem::bytes_for(r->sy, r->opt.precision, r->opt.max_iters);
      if ((int64_t)r->bytes > budget)
        rc = fail(BA_ENOMEM, "problem needs %lld bytes, budget is %lld", (long long)r->bytes, (long long)budget);
    }
    if (rc != BA_OK) {
      r->rc = rc;
      r->err = g_last_error;
    }
    r->obs = std::vector<ba_obs>();  // the analysis holds everything the upload needs
    bool failed = rc != BA_OK;
    {
      std::lock_guard<std::mutex> lk(mu);
      --analysing;
      if (!failed && stop) {
        r->rc = BA_ESTATE;
        r->err = "server is shutting down";
        failed = true;
      }
      if (!failed) ready[r->ticket] = r;
    }
    if (failed) finish({r});
    cv_work.notify_one();
  }
}

// Uploads of admitted problems on their own stream and thread, so that the scheduler
// keeps launching iterations meanwhile; a problem joins the batch once its copies are done.
void ba_server::up_loop() {
  while (true) {
    ReqP r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_ana.wait(lk, [&] { return stop || !up_q.empty(); });
      if (up_q.empty()) {
        if (stop) return;
        continue;
      }
      r = up_q.front();
      up_q.pop_front();
      ++uploading;
    }
    const ba_problem_desc d = r->desc();
    int rc = r->dp.init(r->sy, &d, &r->opt, (char *)mem + r->off, up_stream);
    if (rc == BA_OK) {
      r->dp.pending_state = r->dp.fresh_state();
      hipError_t e = hipMemcpyAsync(r->dp.view.st, &r->dp.pending_state, sizeof(LMState),
                                    hipMemcpyHostToDevice, up_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(up_stream);
      if (e != hipSuccess) rc = hip_fail(e, "server upload");
    }
    // what the device copy and the report still need is in dp; drop the rest
    r->dp.staging_f.clear();
    r->dp.staging_d.clear();
    r->sy = Symbolic();
    r->sy.C = r->dp.C;
    r->sy.P = r->dp.P;
    r->pts = std::vector<double>();
    if (rc != BA_OK) {
      r->rc = rc;
      r->err = g_last_error;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      --uploading;
      if (rc == BA_OK) uploaded.push_back(r);
    }
    if (rc != BA_OK) finish({r});
    cv_work.notify_one();
  }
}

// Hand over the problems whose result copies have landed.  block: wait for the oldest.
int ba_server::complete(bool block) {
  while (!completing.empty()) {
    Completion &c = completing.front();
    hipError_t e = block ? hipEventSynchronize(c.ev) : hipEventQuery(c.ev);
    if (e == hipErrorNotReady) return BA_OK;
    block = false;
    if (e != hipSuccess) return hip_fail(e, "server result copies");
    for (size_t i = 0; i < c.reqs.size(); ++i) {
      Req &r = *c.reqs[i];
      r.out_poses.resize(r.sy.C);
      r.out_pts.resize(3 * (size_t)r.sy.P);
      r.iter_cost.resize(r.dp.max_iters + 1);
      r.iter_pcg.resize(r.dp.max_iters);
      r.rep.iter_cost = r.iter_cost.data();
      r.rep.pcg_iters = r.iter_pcg.data();
      r.dp.finish_result(c.bufs[i].p, r.out_poses.data(), r.out_pts.data(), &r.rep);
      pinned_free.push_back(c.bufs[i]);
    }
    (void)hipEventDestroy(c.ev);
    std::vector<ReqP> done_now = std::move(c.reqs);
    completing.pop_front();
    finish(done_now);
  }
  return BA_OK;
}

void ba_server::loop() {
  bool dirty = true;
  while (true) {
    std::vector<ReqP> admitted, pose_now;
    size_t pose_bytes = 0;
    size_t pb_off = 0;
    bool pb_ok = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return (stop && idle_locked()) || !ready.empty() || !pose_q.empty() || !active.empty() ||
               !completing.empty() || !uploaded.empty();
      });
      if (stop && idle_locked()) break;
      // pose requests of one step share one block; 512 bytes cover its alignment
      while (!pose_q.empty() && fatal == BA_OK) {
        ReqP r = pose_q.front();
        if (pose_bytes + r->bytes + 512 > arena.largest_free()) break;
        pose_bytes += r->bytes;
        pose_now.push_back(r);
        pose_q.pop_front();
      }
      if (!pose_now.empty()) pb_ok = arena.alloc(pose_bytes + 512, pb_off);
      // analysed problems in ticket order; a later one that fits may go ahead of one that
      // does not fit, until that one has been passed kMaxPassed times
      {
        std::vector<Req *> waiting;  // earlier problems that did not fit, in ticket order
        for (auto it = ready.begin(); it != ready.end() && fatal == BA_OK;) {
          if ((int)(active.size() + uploaded.size() + up_q.size() + uploading + admitted.size()) >= max_slots) break;
          if (!waiting.empty() && waiting.front()->passed >= kMaxPassed) break;
          ReqP r = it->second;
          size_t off;
          if (!arena.alloc(r->bytes, off)) {
            waiting.push_back(r.get());
            ++it;
            continue;
          }
          for (Req *w : waiting) ++w->passed;
          r->off = off;
          r->holds_block = true;
          admitted.push_back(r);
          it = ready.erase(it);
        }
      }
      peak = std::max(peak, arena.used);
      for (auto &r : admitted) up_q.push_back(r);
      if (!admitted.empty()) cv_ana.notify_all();
      // uploaded problems join the batch
      if (!uploaded.empty()) {
        active.insert(active.end(), uploaded.begin(), uploaded.end());
        uploaded.clear();
        dirty = true;
      }
    }
    if (!active.empty() && fatal == BA_OK) {
      if (dirty) {
        batch.clear();
        for (size_t i = 0; i < active.size(); ++i) batch.add(active[i]->dp.view, (int)i);
        if (batch.upload(stream) != BA_OK) fatal = BA_EDEVICE;
        dirty = false;
      }
      int pcg_max = 1, max_cf = 1;
      for (auto &r : active) {
        pcg_max = std::max(pcg_max, r->dp.pcg_max);
        max_cf = std::max(max_cf, (int)r->dp.max_tcols);
      }
      // at most kLookahead launch sequences in flight
      hipEvent_t &ev = ev_step[n_steps % kLookahead];
      if (fatal == BA_OK && n_steps >= kLookahead && hipEventSynchronize(ev) != hipSuccess) fatal = BA_EDEVICE;
      if (fatal == BA_OK &&
          launch_lm_iteration(precision, batch.plan, pcg_max, max_cf, stream, nullptr) != hipSuccess)
        fatal = BA_EDEVICE;
      if (fatal == BA_OK && hipEventRecord(ev, stream) != hipSuccess) fatal = BA_EDEVICE;
      ++n_steps;
      // every launch sequence advances each problem it holds by one iteration (batched
      // solves never stop early), so the host knows which ones are finished
      std::vector<ReqP> fin, keep;
      for (auto &r : active) (++r->steps >= r->dp.max_iters ? fin : keep).push_back(r);
      if (!fin.empty() && fatal == BA_OK) {
        fin_batch.clear();
        for (auto &r : fin) fin_batch.add(r->dp.view, 0);
        Completion c;
        int rc = fin_batch.upload(stream);
        if (rc == BA_OK && launch_eval(precision, fin_batch.plan, stream, nullptr) != hipSuccess) rc = BA_EDEVICE;
        for (auto &r : fin) {
          Pinned b = take_pinned(r->dp.result_bytes());
          if (!b.p) rc = BA_ENOMEM;
          if (rc == BA_OK && r->dp.enqueue_result(stream, b.p) != hipSuccess) rc = BA_EDEVICE;
          c.reqs.push_back(r);
          c.bufs.push_back(b);
        }
        if (rc == BA_OK && hipEventCreateWithFlags(&c.ev, hipEventDisableTiming) != hipSuccess) rc = BA_EDEVICE;
        if (rc == BA_OK && hipEventRecord(c.ev, stream) != hipSuccess) rc = BA_EDEVICE;
        if (rc != BA_OK) fatal = rc;
        {
          // the blocks stay held until the copies have landed (finish releases them):
          // uploads into a freed block run on another stream
          std::lock_guard<std::mutex> lk(mu);
          active = keep;
        }
        if (rc == BA_OK) completing.push_back(std::move(c));
        else for (auto &b : c.bufs) if (b.p) pinned_free.push_back(b);
        dirty = true;
      }
    }
    if (!pose_now.empty() && fatal == BA_OK) {
      PoseBatch pb;
      std::vector<const ba_pose_request *> rp;
      std::vector<const ba_options *> ro;
      for (auto &r : pose_now) {
        rp.push_back(&r->preq);
        ro.push_back(&r->opt);
      }
      pb.pack(rp, ro);
      if (pb_ok && pb.run((char *)mem + pb_off, stream, nullptr) != BA_OK) fatal = BA_EDEVICE;
      // the headers' download goes to pageable memory: wait for it
      if (hipStreamSynchronize(stream) != hipSuccess) fatal = BA_EDEVICE;
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
    if (fatal == BA_OK) {
      const bool nothing_launched = pose_now.empty() && active.empty();
      if (complete(nothing_launched) != BA_OK) fatal = BA_EDEVICE;
    }
    if (fatal != BA_OK) {
      // fail everything still pending; the device state is unknown
      (void)hipStreamSynchronize(stream);
      std::vector<ReqP> all;
      {
        std::lock_guard<std::mutex> lk(mu);
        all.insert(all.end(), active.begin(), active.end());
        for (auto &kv : ready) all.push_back(kv.second);
        all.insert(all.end(), pose_q.begin(), pose_q.end());
        all.insert(all.end(), up_q.begin(), up_q.end());
        all.insert(all.end(), uploaded.begin(), uploaded.end());
        active.clear();
        ready.clear();
        pose_q.clear();
        up_q.clear();
        uploaded.clear();
      }
      for (auto &c : completing) {
        all.insert(all.end(), c.reqs.begin(), c.reqs.end());
        for (auto &b : c.bufs) pinned_free.push_back(b);
        if (c.ev) (void)hipEventDestroy(c.ev);
      }
      completing.clear();
      for (auto &r : all) r->rc = fatal;
      finish(all);
      dirty = true;
      continue;
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
  if (e == hipSuccess) e = hipStreamCreate(&s->up_stream);
  for (int i = 0; i < kLookahead && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&s->ev_step[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    if (s->mem) (void)hipFree(s->mem);
    if (s->up_stream) (void)hipStreamDestroy(s->up_stream);
    for (auto &ev : s->ev_step)
      if (ev) (void)hipEventDestroy(ev);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    return hip_fail(e, "server allocation");
  }
  s->arena.reset((size_t)hbm_budget_bytes);
  ba_server *raw = s.get();
  const unsigned hw = std::thread::hardware_concurrency();
  const int n_ana = (int)std::max(1u, std::min(8u, hw / 2));
  for (int i = 0; i < n_ana; ++i) s->ana_th.emplace_back([raw] { raw->ana_loop(); });
  s->up_th = std::thread([raw] { raw->up_loop(); });
  s->th = std::thread([raw] { raw->loop(); });
  *out = s.release();
  return BA_OK;
}

int ba_server_submit(ba_server *s, const ba_problem_desc *d, const ba_options *opt, int64_t *ticket) {
  if (!s || !ticket || !d) return fail(BA_EINVAL, "NULL argument");
  if (int e = check_options(opt, false)) return e;
  if (opt->precision != s->precision)
    return fail(BA_EINVAL, "request precision %d differs from the server's %d", opt->precision, s->precision);
  if (d->n_cams < 1 || d->n_pts < 1 || d->n_obs < 1) return fail(BA_EINVAL, "empty problem");
  if (d->n_obs > (int64_t)INT32_MAX - 1) return fail(BA_EINVAL, "n_obs exceeds 2^31 - 2");
  if (!d->K || !d->poses || !d->points_xyz || !d->obs) return fail(BA_EINVAL, "NULL array in problem");
  if ((int64_t)min_problem_bytes(d->n_obs, d->n_pts, d->n_cams, opt->precision) > s->budget)
    return fail(BA_ENOMEM, "problem needs more than the budget of %lld bytes", (long long)s->budget);
  auto r = std::make_shared<Req>();
  r->t_submit = now_ms();
  r->opt = *opt;
  r->n_cams = d->n_cams;
  r->n_pts = d->n_pts;
  r->K_per_cam = d->K_per_cam;
  r->K.assign(d->K, d->K + (d->K_per_cam ? d->n_cams : 1));
  r->poses.assign(d->poses, d->poses + d->n_cams);
  if (d->cam_fixed) r->fixed.assign(d->cam_fixed, d->cam_fixed + d->n_cams);
  r->pts.assign(d->points_xyz, d->points_xyz + 3 * (size_t)d->n_pts);
  r->obs.assign(d->obs, d->obs + d->n_obs);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BA_ESTATE, "server is shutting down");
  r->ticket = s->next_ticket++;
  if (s->first_submit < 0) s->first_submit = r->t_submit;
  s->tickets[r->ticket] = r;
  s->ana_q.push_back(r);
  *ticket = r->ticket;
  s->cv_ana.notify_one();
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
  s->pose_q.push_back(r);
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
  if (r->rc != BA_OK)
    return fail(r->rc, "request %lld failed%s%s", (long long)ticket, r->err.empty() ? "" : ": ", r->err.c_str());
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
  out->queued = (int64_t)(s->ana_q.size() + s->analysing + s->ready.size() + s->pose_q.size());
  out->active = (int64_t)s->active.size();
  out->bytes_in_use = (int64_t)s->arena.used;
  out->peak_bytes = (int64_t)s->peak;
  const double span = s->last_done - s->first_submit;
  out->solves_per_s = (span > 0 && s->n_done > 0) ? s->n_done / (span / 1000.0) : 0.0;
  return BA_OK;
}

void ba_server_destroy(ba_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    std::vector<ReqP> cancelled(s->ana_q.begin(), s->ana_q.end());
    for (auto &kv : s->ready) cancelled.push_back(kv.second);
    cancelled.insert(cancelled.end(), s->pose_q.begin(), s->pose_q.end());
    s->ana_q.clear();
    s->ready.clear();
    s->pose_q.clear();
    for (auto &r : cancelled) {
      r->rc = BA_ESTATE;
      r->err = "cancelled: the server was destroyed";
      r->done = true;
    }
    s->cv_ana.notify_all();
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto &t : s->ana_th) t.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();  // ends once everything admitted has finished
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_ana.notify_all();
  }
  if (s->up_th.joinable()) s->up_th.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->up_stream);
  for (auto &b : s->pinned_free) (void)hipHostFree(b.p);
  for (auto &ev : s->ev_step)
    if (ev) (void)hipEventDestroy(ev);
  (void)hipFree(s->mem);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
