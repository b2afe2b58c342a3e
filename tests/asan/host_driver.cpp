// Host-side driver of the C-ABI for the AddressSanitizer build of the library: runs the
// symbolic analysis in every Schur form, the pose-graph and vehicle-rig set-up, the
// pose-only packing and the server's argument checks on small synthetic problems, and
// every validation path on bad input.  Needs no device: calls that would upload return
// BA_EDEVICE once their host work is done.  Exit status 0 when every call returned what
// it should; AddressSanitizer aborts the process on a memory error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ba.h"

namespace {

int g_bad = 0;

void expect(const char *what, int got, int want1, int want2 = 1) {
  if (got == want1 || got == want2) return;
  std::printf("FAIL %s: status %d (%s)\n", what, got, ba_last_error());
  ++g_bad;
}

uint64_t g_rng = 88172645463325252ull;
double urand() {  // xorshift64, uniform in [0, 1)
  g_rng ^= g_rng << 13;
  g_rng ^= g_rng >> 7;
  g_rng ^= g_rng << 17;
  return (double)(g_rng >> 11) * (1.0 / 9007199254740992.0);
}

// n_cams cameras on a line looking down +z, n_pts points ahead; every point is seen by
// `span` consecutive cameras starting at a random one (span = n_cams: every camera).
struct Scene {
  std::vector<ba_intrinsics> K;
  std::vector<ba_pose> poses;
  std::vector<uint8_t> fixed;
  std::vector<double> pts;
  std::vector<ba_obs> obs;
  ba_problem_desc desc() const {
    ba_problem_desc d{};
    d.n_cams = (int32_t)poses.size();
    d.K = K.data();
    d.K_per_cam = 0;
    d.poses = poses.data();
    d.cam_fixed = fixed.data();
    d.n_pts = (int32_t)(pts.size() / 3);
    d.points_xyz = pts.data();
    d.n_obs = (int64_t)obs.size();
    d.obs = obs.data();
    return d;
  }
};

Scene make_scene(int n_cams, int n_pts, int span) {
  Scene s;
  s.K.push_back(ba_intrinsics{500.0, 500.0, 320.0, 240.0});
  for (int i = 0; i < n_cams; ++i) s.poses.push_back(ba_pose{1.0, 0.0, 0.0, 0.0, -0.5 * i, 0.0, 0.0});
  s.fixed.assign(n_cams, 0);
  s.fixed[0] = 1;
  for (int j = 0; j < n_pts; ++j) {
    const int c0 = span >= n_cams ? 0 : (int)(urand() * (n_cams - span + 1));
    const double x = 0.5 * (c0 + 0.5 * span) + 2.0 * (urand() - 0.5), y = 2.0 * (urand() - 0.5),
                 z = 4.0 + 8.0 * urand();
    s.pts.insert(s.pts.end(), {x, y, z});
    for (int c = c0; c < c0 + span && c < n_cams; ++c) {
      const double u = 500.0 * (x - 0.5 * c) / z + 320.0, v = 500.0 * y / z + 240.0;
      s.obs.push_back(ba_obs{c, j, u + 0.3 * (urand() - 0.5), v + 0.3 * (urand() - 0.5)});
    }
  }
  return s;
}

}  // namespace

int main() {
  ba_options opt;
  ba_default_options(&opt);
  // the analysis in each form, on a banded scene and on a dense one
  const Scene band = make_scene(40, 3000, 8), dense = make_scene(24, 1500, 24);
  for (int32_t flags : {0, BA_FLAG_PAIR_LISTS, BA_FLAG_DENSE_SCHUR, BA_FLAG_PCG_WIDE}) {
    for (const Scene *s : {&band, &dense}) {
      ba_options o = opt;
      o.flags = flags;
      ba_problem_info info{};
      int64_t bytes = 0;
      const ba_problem_desc d = s->desc();
      expect("ba_analyse", ba_analyse(&d, &o, &info, &bytes), BA_OK);
      if (bytes <= 0 || info.n_obs != (int32_t)s->obs.size()) {
        std::printf("FAIL ba_analyse sizes: bytes %lld, n_obs %d\n", (long long)bytes, info.n_obs);
        ++g_bad;
      }
      o.prior_abs = 1.0;
      o.prior_seq = 10.0;
      o.prior_seq_k = 3;
      expect("ba_analyse priors", ba_analyse(&d, &o, &info, &bytes), BA_OK);
      ba_problem *p = nullptr;
      const int rc = ba_create(&d, &o, nullptr, &p);
      expect("ba_create", rc, BA_OK, BA_EDEVICE);
      if (p) ba_destroy(p);
    }
  }
  // validation: index out of range, duplicate observation, non-finite, all fixed
  {
    Scene s = make_scene(6, 50, 6);
    ba_problem *p = nullptr;
    s.obs[3].cam = 99;
    ba_problem_desc d = s.desc();
    expect("camera out of range", ba_create(&d, &opt, nullptr, &p), BA_EINVAL);
    s = make_scene(6, 50, 6);
    s.obs[4].cam = s.obs[3].cam;
    s.obs[4].pt = s.obs[3].pt;
    d = s.desc();
    expect("duplicate observation", ba_analyse(&d, &opt, nullptr, nullptr), BA_EINVAL);
    s = make_scene(6, 50, 6);
    s.pts[7] = NAN;
    d = s.desc();
    expect("non-finite point", ba_analyse(&d, &opt, nullptr, nullptr), BA_EINVAL);
    s = make_scene(6, 50, 6);
    std::fill(s.fixed.begin(), s.fixed.end(), 1);
    d = s.desc();
    expect("every camera fixed", ba_analyse(&d, &opt, nullptr, nullptr), BA_EINVAL);
    ba_options bad = opt;
    bad.flags = 1 << 10;
    s = make_scene(6, 50, 6);
    d = s.desc();
    expect("unknown flag", ba_analyse(&d, &bad, nullptr, nullptr), BA_EINVAL);
  }
  // pose graph: a chain of 30 nodes with loop edges
  {
    std::vector<ba_pose> nodes;
    for (int i = 0; i < 30; ++i) nodes.push_back(ba_pose{1.0, 0.0, 0.0, 0.0, -1.0 * i, 0.0, 0.0});
    std::vector<ba_pose_edge> edges;
    for (int i = 0; i + 1 < 30; ++i) edges.push_back(ba_pose_edge{i, i + 1, BA_EDGE_SEQUENTIAL, 0, {1, 0, 0, 0, 1, 0, 0}, 10, 100});
    for (int i = 0; i + 10 < 30; i += 5) edges.push_back(ba_pose_edge{i, i + 10, BA_EDGE_LOOP, 0, {1, 0, 0, 0, 10, 0, 0}, 1, 1});
    std::vector<uint8_t> nf(30, 0);
    nf[0] = 1;
    ba_pose_graph_desc g{30, nodes.data(), nf.data(), (int64_t)edges.size(), edges.data()};
    ba_problem *p = nullptr;
    expect("pose graph", ba_pose_graph_create(&g, &opt, nullptr, &p), BA_OK, BA_EDEVICE);
    if (p) ba_destroy(p);
    edges[3].j = edges[3].i;
    expect("pose graph self edge", ba_pose_graph_create(&g, &opt, nullptr, &p), BA_EINVAL);
  }
  // vehicle rig: 20 frames of 2 cameras
  {
    const Scene s = make_scene(40, 600, 6);
    std::vector<ba_pose> veh, ext{{1, 0, 0, 0, 0, 0, 0}, {1, 0, 0, 0, -0.3, 0, 0}};
    for (int f = 0; f < 20; ++f) veh.push_back(ba_pose{1.0, 0.0, 0.0, 0.0, -1.0 * f, 0.0, 0.0});
    std::vector<ba_rig_obs> ro;
    for (const ba_obs &o : s.obs) ro.push_back(ba_rig_obs{o.cam / 2, o.cam % 2, o.pt, 0, o.u, o.v});
    std::vector<ba_intrinsics> K(2, s.K[0]);
    std::vector<uint8_t> vf(20, 0);
    vf[0] = 1;
    const int32_t pairs[2] = {0, 1};
    ba_rig_desc r{20, 2, K.data(), veh.data(), ext.data(), vf.data(), nullptr, (int32_t)(s.pts.size() / 3),
                  s.pts.data(), (int64_t)ro.size(), ro.data(), 10.0, 10.0, 1, pairs};
    ba_problem *p = nullptr;
    expect("rig", ba_rig_create(&r, &opt, nullptr, &p), BA_OK, BA_EDEVICE);
    if (p) ba_destroy(p);
  }
  // pose-only requests: packing, then the device step
  {
    std::vector<double> X, uv;
    for (int c = 0; c < 200; ++c) {
      const double x = urand() - 0.5, y = urand() - 0.5, z = 3 + urand();
      X.insert(X.end(), {x, y, z});
      uv.insert(uv.end(), {500 * x / z + 320, 500 * y / z + 240});
    }
    ba_pose_request rq{{500, 500, 320, 240}, {1, 0, 0, 0, 0.01, 0, 0}, 200, X.data(), uv.data()};
    std::vector<ba_pose_request> reqs(8, rq);
    ba_options po = opt;
    po.huber_delta = 1.0;
    ba_pose out[8];
    expect("pose batch", ba_pose_batch(8, reqs.data(), &po, nullptr, out, nullptr, nullptr, nullptr), BA_OK, BA_EDEVICE);
    expect("pose batch noalloc", ba_pose_batch_noalloc(8, reqs.data(), &po, nullptr, out, nullptr, nullptr), BA_OK,
           BA_EDEVICE);
    reqs[5].n = 0;
    expect("pose batch n = 0", ba_pose_batch(8, reqs.data(), &po, nullptr, out, nullptr, nullptr, nullptr), BA_EINVAL);
  }
  // triangulation and server argument checks
  {
    const Scene s = make_scene(10, 200, 5);
    const ba_problem_desc d = s.desc();
    std::vector<double> Xo(s.pts.size());
    std::vector<uint8_t> ok(s.pts.size() / 3), inl(s.obs.size());
    expect("triangulate", ba_triangulate(&d, BA_TRI_DLT, nullptr, Xo.data(), ok.data(), nullptr), BA_OK, BA_EDEVICE);
    expect("triangulate method", ba_triangulate(&d, 7, nullptr, Xo.data(), ok.data(), nullptr), BA_EINVAL);
    expect("ransac", ba_triangulate_ransac(&d, BA_TRI_MIDPOINT, 2.0, 64, nullptr, Xo.data(), ok.data(), inl.data(),
                                           nullptr), BA_OK, BA_EDEVICE);
    ba_server *srv = nullptr;
    expect("server budget", ba_server_create(1000, 4, BA_PREC_F32, nullptr, &srv), BA_EINVAL);
    const int rc = ba_server_create(64 << 20, 4, BA_PREC_F32, nullptr, &srv);
    expect("server", rc, BA_OK, BA_EDEVICE);
    if (srv) ba_server_destroy(srv);
  }
  std::printf("host driver: %d unexpected statuses\n", g_bad);
  return g_bad ? 1 : 0;
}
