// Pose-only refinement against a fixed map (paper Sec. 6.4.2, localization
// mode): every request of a call runs in one launch, one workgroup each.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_runtime.h"

namespace bax {

int check_pose_request(const ba_pose_request &r, int64_t i) {
  if (r.n < 1 || r.n > BA_POSE_MAX_CORR)
    return fail(BA_EINVAL, "request %lld: n = %d outside [1, %d]", (long long)i, r.n, BA_POSE_MAX_CORR);
  if (!r.X || !r.uv) return fail(BA_EINVAL, "request %lld: NULL correspondence array", (long long)i);
  if (!(std::isfinite(r.K.fx) && std::isfinite(r.K.fy) && std::isfinite(r.K.cx) && std::isfinite(r.K.cy)) ||
      r.K.fx == 0.0 || r.K.fy == 0.0)
    return fail(BA_EINVAL, "request %lld: invalid intrinsics", (long long)i);
  if (int e = check_pose(r.pose0, "request", i)) return e;
  for (int c = 0; c < 3 * r.n; ++c)
    if (!std::isfinite(r.X[c])) return fail(BA_EINVAL, "request %lld: non-finite map point", (long long)i);
  for (int c = 0; c < 2 * r.n; ++c)
    if (!std::isfinite(r.uv[c])) return fail(BA_EINVAL, "request %lld: non-finite pixel", (long long)i);
  return BA_OK;
}

// Packs requests into one device block: [PoseDev x n][X double][uv float].
int PoseBatch::pack(const std::vector<const ba_pose_request *> &reqs,
                    const std::vector<const ba_options *> &opts) {
  n = (int)reqs.size();
  int64_t tot = 0;
  for (auto *r : reqs) tot += r->n;
  n_corr = tot;
  hdr.assign(n, PoseDev{});
  X.resize(3 * tot);
  uv.resize(2 * tot);
  int64_t o = 0;
  for (int i = 0; i < n; ++i) {
    const ba_pose_request &r = *reqs[i];
    PoseDev &d = hdr[i];
    d.K[0] = r.K.fx;
    d.K[1] = r.K.fy;
    d.K[2] = r.K.cx;
    d.K[3] = r.K.cy;
    quat_to_pose12(r.pose0, d.pose);
    d.off = o;
    d.n = r.n;
    d.iters = opts[i]->max_iters;
    d.delta = opts[i]->huber_delta;
    std::memcpy(&X[3 * o], r.X, 3 * (size_t)r.n * sizeof(double));
    for (int c = 0; c < 2 * r.n; ++c) uv[2 * o + c] = (float)r.uv[c];
    o += r.n;
  }
  return BA_OK;
}

size_t PoseBatch::bytes() const {
  const size_t h = ((size_t)n * sizeof(PoseDev) + 255) & ~size_t(255);
  const size_t x = ((size_t)n_corr * 3 * 8 + 255) & ~size_t(255);
  return h + x + (size_t)n_corr * 2 * 4;
}

int PoseBatch::run(char *base, hipStream_t s, KernelTimer *tm) {
  const size_t h = ((size_t)n * sizeof(PoseDev) + 255) & ~size_t(255);
  const size_t x = ((size_t)n_corr * 3 * 8 + 255) & ~size_t(255);
  PoseDev *dh = (PoseDev *)base;
  double *dX = (double *)(base + h);
  float *duv = (float *)(base + h + x);
  hipError_t e = hipMemcpyAsync(dh, hdr.data(), n * sizeof(PoseDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dX, X.data(), X.size() * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(duv, uv.data(), uv.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_pose_gn(n, dh, dX, duv, s, tm);
  if (e == hipSuccess) e = hipMemcpyAsync(hdr.data(), dh, n * sizeof(PoseDev), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "pose batch");
  return BA_OK;
}

}  // namespace bax

using namespace bax;

extern "C" int ba_pose_batch(int32_t n_req, const ba_pose_request *reqs, const ba_options *opt,
                             void *hip_stream, ba_pose *poses_out, int32_t *status_out,
                             double *cost_out, double *device_ms) {
  if (n_req < 1 || !reqs) return fail(BA_EINVAL, "no requests");
  if (int e = check_options(opt, true)) return e;
  std::vector<const ba_pose_request *> rp(n_req);
  for (int i = 0; i < n_req; ++i) {
    if (int e = check_pose_request(reqs[i], i)) return e;
    rp[i] = &reqs[i];
  }
  PoseBatch pb;
  pb.pack(rp, std::vector<const ba_options *>(n_req, opt));
  hipStream_t s = (hipStream_t)hip_stream;
  bool own = false;
  hipError_t e = hipSuccess;
  if (!s) {
    e = hipStreamCreate(&s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    own = true;
  }
  void *mem = nullptr;
  e = hipMalloc(&mem, pb.bytes());
  if (e != hipSuccess) {
    if (own) (void)hipStreamDestroy(s);
    return hip_fail(e, "pose batch allocation");
  }
  EventTimer timer;  // device time of the pose kernel alone
  int rc = pb.run((char *)mem, s, &timer);
  if (rc == BA_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "pose batch");
  }
  if (rc == BA_OK) {
    double ms[K_NUM_KERNELS];
    int32_t nl[K_NUM_KERNELS];
    timer.collect(ms, nl);
    if (device_ms) *device_ms = ms[K_POSE_GN];
    for (int i = 0; i < n_req; ++i) {
      if (poses_out) poses_out[i] = pose12_to_quat(pb.hdr[i].pose);
      if (status_out) status_out[i] = pb.hdr[i].status;
      if (cost_out) cost_out[i] = pb.hdr[i].cost;
    }
  }
  (void)hipFree(mem);
  if (own) (void)hipStreamDestroy(s);
  return rc;
}
