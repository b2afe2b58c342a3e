// Pose-only refinement (paper Sec. 6.4.2, localization mode) without device
// allocation: the requests are staged in a fixed device array that the library
// holds for the life of the process, instead of a block obtained per call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/ba.h"
#include "ba_internal.h"
#include "ba_runtime.h"

namespace bax {
namespace {

// Staging of ba_pose_batch_noalloc: headers, map points and pixels of one call.
// One copy per device; every call on that device reuses it.
__device__ __align__(256) char scratch[BA_POSE_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices] = {};

// Device address of the current device's staging array, looked up on the first call
// on that device.  The array's name is a host-side stand-in: only this address may
// reach kernels and copies.
int scratch_for_current_device(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(BA_EDEVICE, "device %d beyond the staging table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "staging array address");
    g_scratch[dev] = (char *)p;
  }
  *out = g_scratch[dev];
  return BA_OK;
}

}  // namespace
}  // namespace bax

using namespace bax;

extern "C" int ba_pose_batch_noalloc(int32_t n_req, const ba_pose_request *reqs, const ba_options *opt,
                                     void *hip_stream, ba_pose *poses_out, int32_t *status_out,
                                     double *cost_out) {
  if (n_req < 1 || !reqs) return fail(BA_EINVAL, "no requests");
  if (int e = check_options(opt, true)) return e;
  std::vector<const ba_pose_request *> rp(n_req);
  for (int i = 0; i < n_req; ++i) {
    if (int e = check_pose_request(reqs[i], i)) return e;
    rp[i] = &reqs[i];
  }
  PoseBatch pb;
  pb.pack(rp, std::vector<const ba_options *>(n_req, opt));
  if (pb.bytes() > (size_t)BA_POSE_NOALLOC_MAX_BYTES)
    return fail(BA_ENOMEM, "pose batch needs %zu bytes of staging, more than the %zu the no-allocation entry holds",
                pb.bytes(), (size_t)BA_POSE_NOALLOC_MAX_BYTES);
  char *base = nullptr;
  if (int e = scratch_for_current_device(&base)) return e;
  hipStream_t s = (hipStream_t)hip_stream;  // NULL: the device's null stream
  int rc = pb.run(base, s, nullptr);
  if (rc == BA_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "pose batch");
  }
  if (rc != BA_OK) return rc;
  for (int i = 0; i < n_req; ++i) {
    if (poses_out) poses_out[i] = pose12_to_quat(pb.hdr[i].pose);
    if (status_out) status_out[i] = pb.hdr[i].status;
    if (cost_out) cost_out[i] = pb.hdr[i].cost;
  }
  return BA_OK;
}
