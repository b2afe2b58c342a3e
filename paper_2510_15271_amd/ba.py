"""Python binding of libba_mi355x.so (ctypes; argument marshalling only).

Every step of the solve runs in the library's HIP kernels.  If the shared
library is missing this module raises on first use; there is no fallback.
Functions mirror the C-ABI in ``include/ba.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libba_mi355x.so")

BA_OK, BA_EINVAL, BA_ENOMEM, BA_EDEVICE, BA_ESTATE = 0, -1, -2, -3, -4
PREC = {"f64": 0, "f32": 1, "f16j": 2, "bf16j": 3}
STATUS_OK, STATUS_DAMPING, STATUS_NUMERICAL, STATUS_PCG_SYNC = 0, 1, 2, 3
POSE_MAX_CORR = 4096
POSE_NOALLOC_MAX_BYTES = 100663296  # staging array of ba_pose_batch_noalloc (96 MiB)


class BAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ba error {code}: {msg}")
        self.code = code


class Intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Pose(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("qw", "qx", "qy", "qz", "tx", "ty", "tz")]


class Options(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("pcg_max_iters", C.c_int32),
                ("pcg_rel_tol", C.c_double), ("lambda0", C.c_double),
                ("huber_delta", C.c_double), ("precision", C.c_int32), ("flags", C.c_int32),
                ("prior_abs", C.c_double), ("prior_seq", C.c_double), ("prior_seq_k", C.c_int32),
                ("reserved", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("accepted", C.c_int32), ("status", C.c_int32),
                ("n_masked", C.c_int32), ("cost0", C.c_double), ("cost", C.c_double),
                ("rms_px", C.c_double), ("lambda_", C.c_double),
                ("iter_cost", C.POINTER(C.c_double)), ("pcg_iters", C.POINTER(C.c_int32)),
                ("solve_ms", C.c_double), ("setup_ms", C.c_double)]


class ProblemDesc(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("K", C.c_void_p), ("K_per_cam", C.c_int32),
                ("poses", C.c_void_p), ("cam_fixed", C.c_void_p), ("n_pts", C.c_int32),
                ("points_xyz", C.c_void_p), ("n_obs", C.c_int64), ("obs", C.c_void_p)]


class DebugIteration(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("pcg_iters", C.c_int32), ("accepted", C.c_int32),
                ("S_rowptr", C.POINTER(C.c_int32)), ("S_col", C.POINTER(C.c_int32)),
                ("S", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)), ("gc", C.POINTER(C.c_double)),
                ("dc", C.POINTER(C.c_double)), ("gp", C.POINTER(C.c_double)), ("dp", C.POINTER(C.c_double)),
                ("r", C.POINTER(C.c_double)), ("Jc", C.POINTER(C.c_double)), ("Jp", C.POINTER(C.c_double))]


class PoseRequest(C.Structure):
    _fields_ = [("K", Intrinsics), ("pose0", Pose), ("n", C.c_int32),
                ("X", C.c_void_p), ("uv", C.c_void_p)]


class ProblemInfo(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_free_cams", C.c_int32), ("n_pts", C.c_int32),
                ("n_obs", C.c_int32), ("n_pairs", C.c_int64), ("n_up_blocks", C.c_int32),
                ("nnzb", C.c_int32), ("n_free_obs", C.c_int32), ("precision", C.c_int32),
                ("schur_form", C.c_int32), ("n_chunks", C.c_int32), ("n_entries", C.c_int64),
                ("pcg_rows", C.c_int32), ("pcg_resident", C.c_int32)]


class PoseEdge(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("type", C.c_int32), ("reserved", C.c_int32),
                ("meas", Pose), ("w_rot", C.c_double), ("w_trans", C.c_double)]


class PoseGraphDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("poses", C.c_void_p), ("node_fixed", C.c_void_p),
                ("n_edges", C.c_int64), ("edges", C.c_void_p)]


class RigDesc(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("n_rig", C.c_int32), ("K", C.c_void_p),
                ("vehicle_poses", C.c_void_p), ("extrinsics", C.c_void_p), ("vehicle_fixed", C.c_void_p),
                ("extrinsic_fixed", C.c_void_p), ("n_pts", C.c_int32), ("points_xyz", C.c_void_p),
                ("n_obs", C.c_int64), ("obs", C.c_void_p), ("prior_ext", C.c_double), ("prior_rig", C.c_double),
                ("n_rig_pairs", C.c_int32), ("rig_pairs", C.c_void_p)]


class RefineStage(C.Structure):
    _fields_ = [("huber_delta", C.c_double), ("cull_px", C.c_double), ("triangulation", C.c_int32),
                ("reserved", C.c_int32)]


TRI = {"midpoint": 0, "dlt": 1}


class RefineRound(C.Structure):
    _fields_ = [("stage", C.c_int32), ("round", C.c_int32), ("iters", C.c_int32),
                ("status", C.c_int32), ("cost", C.c_double), ("n_active_obs", C.c_int64),
                ("n_active_pts", C.c_int32), ("reserved", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("solves_per_s", C.c_double),
                ("done", C.c_int64), ("queued", C.c_int64), ("active", C.c_int64),
                ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64)]


OBS_DTYPE = np.dtype([("cam", "<i4"), ("pt", "<i4"), ("u", "<f8"), ("v", "<f8")])
RIG_OBS_DTYPE = np.dtype([("frame", "<i4"), ("cam", "<i4"), ("pt", "<i4"), ("reserved", "<i4"),
                          ("u", "<f8"), ("v", "<f8")])
EDGE_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("type", "<i4"), ("reserved", "<i4"),
                       ("q", "<f8", (4,)), ("t", "<f8", (3,)), ("w_rot", "<f8"), ("w_trans", "<f8")])

_lib = None


def lib():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with "
                           "`python -m paper_2510_15271_amd.build_lib`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.ba_version.restype = C.c_char_p
    L.ba_last_error.restype = C.c_char_p
    L.ba_default_options.argtypes = [C.POINTER(Options)]
    L.ba_create.argtypes = [C.POINTER(ProblemDesc), C.POINTER(Options), vp, C.POINTER(vp)]
    L.ba_solve.argtypes = [vp]
    L.ba_solve_async.argtypes = [vp]
    L.ba_wait.argtypes = [vp]
    L.ba_reset.argtypes = [vp]
    L.ba_get_result.argtypes = [vp, vp, vp, C.POINTER(Report)]
    L.ba_get_info.argtypes = [vp, C.POINTER(ProblemInfo)]
    L.ba_analyse.argtypes = [C.POINTER(ProblemDesc), C.POINTER(Options), C.POINTER(ProblemInfo),
                             C.POINTER(i64)]
    L.ba_refine.argtypes = [vp, i32, C.POINTER(RefineStage), i32, C.POINTER(RefineRound)]
    L.ba_pose_graph_create.argtypes = [C.POINTER(PoseGraphDesc), C.POINTER(Options), vp, C.POINTER(vp)]
    L.ba_rig_create.argtypes = [C.POINTER(RigDesc), C.POINTER(Options), vp, C.POINTER(vp)]
    L.ba_rig_get_result.argtypes = [vp, vp, vp, vp, C.POINTER(Report)]
    L.ba_get_active.argtypes = [vp, vp]
    L.ba_triangulate.argtypes = [C.POINTER(ProblemDesc), i32, vp, vp, vp, dp]
    L.ba_triangulate_ransac.argtypes = [C.POINTER(ProblemDesc), i32, C.c_double, i32, vp, vp, vp, vp, dp]
    L.ba_problem_bytes.argtypes = [vp]
    L.ba_problem_bytes.restype = i64
    L.ba_destroy.argtypes = [vp]
    L.ba_destroy.restype = None
    L.ba_set_profiling.argtypes = [vp, i32, i32]
    L.ba_set_barrier_polls.argtypes = [vp, i32]
    L.ba_debug_iteration_export.argtypes = [vp, C.POINTER(DebugIteration)]
    L.ba_get_kernel_times.argtypes = [vp, i32, C.POINTER(C.c_char_p), dp, C.POINTER(i32),
                                      C.POINTER(i32)]
    L.ba_pose_batch.argtypes = [i32, C.POINTER(PoseRequest), C.POINTER(Options), vp, vp,
                                C.POINTER(i32), dp, dp]
    L.ba_pose_batch_noalloc.argtypes = [i32, C.POINTER(PoseRequest), C.POINTER(Options), vp, vp,
                                        C.POINTER(i32), dp]
    L.ba_server_create.argtypes = [i64, i32, i32, vp, C.POINTER(vp)]
    L.ba_server_submit.argtypes = [vp, C.POINTER(ProblemDesc), C.POINTER(Options), C.POINTER(i64)]
    L.ba_server_submit_pose.argtypes = [vp, C.POINTER(PoseRequest), C.POINTER(Options),
                                        C.POINTER(i64)]
    L.ba_server_wait.argtypes = [vp, i64, vp, vp, C.POINTER(Report)]
    L.ba_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.ba_server_destroy.argtypes = [vp]
    L.ba_server_destroy.restype = None
    _lib = L
    return L


def _check(rc):
    if rc != BA_OK:
        raise BAError(rc, lib().ba_last_error().decode())


FLAG_NO_GRAPH = 2
FLAG_PAIR_LISTS = 4
FLAG_PCG_WIDE = 8
FLAG_PCG_RESIDENT = 16
FLAG_DENSE_SCHUR = 32
FLAG_PCG_COOPERATIVE = 64


def options(max_iters=10, pcg_max_iters=50, pcg_rel_tol=1e-6, lambda0=1e-4, huber_delta=0.0,
            precision="f32", flags=0, prior_abs=0.0, prior_seq=0.0, prior_seq_k=1) -> Options:
    o = Options()
    lib().ba_default_options(C.byref(o))
    o.max_iters = max_iters
    o.pcg_max_iters = pcg_max_iters
    o.pcg_rel_tol = pcg_rel_tol
    o.lambda0 = lambda0
    o.huber_delta = huber_delta
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.flags = int(flags)
    o.prior_abs = float(prior_abs)
    o.prior_seq = float(prior_seq)
    o.prior_seq_k = int(prior_seq_k)
    return o


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Desc:
    """Holds the contiguous host arrays a ProblemDesc points to."""

    def __init__(self, K, q, t, X, obs_cam, obs_pt, obs_uv, cam_fixed=None):
        K = np.ascontiguousarray(np.atleast_2d(K), dtype=np.float64)
        self.K = K
        self.poses = np.ascontiguousarray(np.concatenate([np.asarray(q, np.float64),
                                                          np.asarray(t, np.float64)], axis=1))
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        n = len(obs_cam)
        obs = np.empty(n, OBS_DTYPE)
        obs["cam"] = obs_cam
        obs["pt"] = obs_pt
        obs["u"] = np.asarray(obs_uv)[:, 0]
        obs["v"] = np.asarray(obs_uv)[:, 1]
        self.obs = obs
        self.fixed = None if cam_fixed is None else np.ascontiguousarray(cam_fixed, dtype=np.uint8)
        d = ProblemDesc()
        d.n_cams = self.poses.shape[0]
        d.K = _ptr(self.K)
        d.K_per_cam = 1 if K.shape[0] == d.n_cams and d.n_cams > 1 else 0
        if K.shape[0] not in (1, d.n_cams):
            raise ValueError("K must have one row or one row per camera")
        d.poses = _ptr(self.poses)
        d.cam_fixed = _ptr(self.fixed)
        d.n_pts = self.X.shape[0]
        d.points_xyz = _ptr(self.X)
        d.n_obs = n
        d.obs = _ptr(self.obs)
        self.desc = d


class _GraphDesc:
    """Holds the contiguous host arrays a PoseGraphDesc points to."""

    def __init__(self, q, t, edge_i, edge_j, meas_q, meas_t, w_rot, w_trans, fixed=None, edge_type=None):
        self.poses = np.ascontiguousarray(np.concatenate([np.asarray(q, np.float64),
                                                          np.asarray(t, np.float64)], axis=1))
        n = len(edge_i)
        e = np.zeros(n, EDGE_DTYPE)
        e["i"], e["j"] = edge_i, edge_j
        e["type"] = 0 if edge_type is None else edge_type
        e["q"], e["t"] = meas_q, meas_t
        e["w_rot"], e["w_trans"] = w_rot, w_trans
        assert EDGE_DTYPE.itemsize == C.sizeof(PoseEdge)
        self.edges = e
        self.fixed = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        d = PoseGraphDesc()
        d.n_nodes = self.poses.shape[0]
        d.poses = _ptr(self.poses)
        d.node_fixed = _ptr(self.fixed)
        d.n_edges = n
        d.edges = _ptr(self.edges)
        self.desc = d


class _RigDesc:
    """Holds the contiguous host arrays a RigDesc points to."""

    def __init__(self, K, qv, tv, qe, te, X, frame, rcam, pt, uv, vehicle_fixed=None, extrinsic_fixed=None,
                 prior_ext=0.0, prior_rig=0.0, rig_pairs=None):
        self.K = np.ascontiguousarray(K, dtype=np.float64)
        self.vp = np.ascontiguousarray(np.concatenate([np.asarray(qv, np.float64), np.asarray(tv, np.float64)], 1))
        self.ep = np.ascontiguousarray(np.concatenate([np.asarray(qe, np.float64), np.asarray(te, np.float64)], 1))
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        o = np.zeros(len(frame), RIG_OBS_DTYPE)
        o["frame"], o["cam"], o["pt"] = frame, rcam, pt
        o["u"], o["v"] = np.asarray(uv)[:, 0], np.asarray(uv)[:, 1]
        self.obs = o
        self.vf = None if vehicle_fixed is None else np.ascontiguousarray(vehicle_fixed, dtype=np.uint8)
        self.ef = None if extrinsic_fixed is None else np.ascontiguousarray(extrinsic_fixed, dtype=np.uint8)
        self.pairs = (np.zeros(0, np.int32) if rig_pairs is None
                      else np.ascontiguousarray(np.asarray(rig_pairs).reshape(-1), dtype=np.int32))
        d = RigDesc()
        d.n_frames, d.n_rig = self.vp.shape[0], self.ep.shape[0]
        d.K = _ptr(self.K)
        d.vehicle_poses, d.extrinsics = _ptr(self.vp), _ptr(self.ep)
        d.vehicle_fixed, d.extrinsic_fixed = _ptr(self.vf), _ptr(self.ef)
        d.n_pts, d.points_xyz = self.X.shape[0], _ptr(self.X)
        d.n_obs, d.obs = len(o), _ptr(self.obs)
        d.prior_ext, d.prior_rig = float(prior_ext), float(prior_rig)
        d.n_rig_pairs, d.rig_pairs = self.pairs.size // 2, _ptr(self.pairs)
        self.desc = d


def rig_desc(s, prior_ext=0.0, prior_rig=0.0, rig_pairs=None) -> _RigDesc:
    return _RigDesc(s.K, s.qv0, s.tv0, s.qe0, s.te0, s.X0, s.frame, s.rcam, s.obs_pt, s.obs_uv, s.fixed_v,
                    s.fixed_e, prior_ext, prior_rig, rig_pairs)


def triangulate(desc: _Desc, method="midpoint", stream=None):
    """ba_triangulate: every point from its observations with the cameras held at the
    description's poses; returns (points (P, 3), ok (P,) bool, device ms)."""
    P = int(desc.desc.n_pts)
    X = np.zeros((P, 3))
    ok = np.zeros(P, np.uint8)
    ms = C.c_double()
    _check(lib().ba_triangulate(C.byref(desc.desc), TRI[method], stream, _ptr(X), _ptr(ok), C.byref(ms)))
    return X, ok.astype(bool), ms.value


def triangulate_ransac(desc: _Desc, tau_px=3.0, n_hyp=64, method="midpoint", stream=None):
    """ba_triangulate_ransac: returns (points (P, 3), ok (P,) bool, inliers (N,) bool, device ms)."""
    P, N = int(desc.desc.n_pts), int(desc.desc.n_obs)
    X = np.zeros((P, 3))
    ok = np.zeros(P, np.uint8)
    inl = np.zeros(N, np.uint8)
    ms = C.c_double()
    _check(lib().ba_triangulate_ransac(C.byref(desc.desc), TRI[method], float(tau_px), int(n_hyp), stream, _ptr(X),
                                       _ptr(ok), _ptr(inl), C.byref(ms)))
    return X, ok.astype(bool), inl.astype(bool), ms.value


def pose_graph_desc(g) -> _GraphDesc:
    return _GraphDesc(g.q0, g.t0, g.edge_i, g.edge_j, g.meas_q, g.meas_t, g.w_rot, g.w_trans,
                      g.fixed, g.edge_type)


def scene_desc(scene) -> _Desc:
    return _Desc(scene.K, scene.q0, scene.t0, scene.X0, scene.obs_cam, scene.obs_pt,
                 scene.obs_uv, scene.cam_fixed)


class Problem:
    """One bundle-adjustment problem resident on the device."""

    def __init__(self, desc: _Desc, opts: Options, stream=None):
        self._desc = desc
        self.opts = opts
        self.n_cams = desc.desc.n_cams
        self.n_pts = desc.desc.n_pts
        h = C.c_void_p()
        _check(lib().ba_create(C.byref(desc.desc), C.byref(opts), stream, C.byref(h)))
        self._h = h

    @classmethod
    def from_pose_graph(cls, graph, stream=None, **kw):
        """ba_pose_graph_create from a synth.PoseGraph (or a _GraphDesc)."""
        gd = graph if isinstance(graph, _GraphDesc) else pose_graph_desc(graph)
        self = cls.__new__(cls)
        self._desc = gd
        self.opts = options(**kw)
        self.n_cams = gd.desc.n_nodes
        self.n_pts = 0
        h = C.c_void_p()
        _check(lib().ba_pose_graph_create(C.byref(gd.desc), C.byref(self.opts), stream, C.byref(h)))
        self._h = h
        return self

    @classmethod
    def from_rig(cls, scene, prior_ext=0.0, prior_rig=0.0, rig_pairs=None, stream=None, **kw):
        """ba_rig_create from a synth.RigScene (or a _RigDesc)."""
        rd = scene if isinstance(scene, _RigDesc) else rig_desc(scene, prior_ext, prior_rig, rig_pairs)
        self = cls.__new__(cls)
        self._desc = rd
        self.opts = options(**kw)
        self.n_frames, self.n_rig = rd.desc.n_frames, rd.desc.n_rig
        self.n_cams = self.n_frames * self.n_rig
        self.n_pts = rd.desc.n_pts
        h = C.c_void_p()
        _check(lib().ba_rig_create(C.byref(rd.desc), C.byref(self.opts), stream, C.byref(h)))
        self._h = h
        return self

    def rig_result(self):
        """Vehicle poses, extrinsics, points and the report (ba_rig_get_result)."""
        vp = np.zeros((self.n_frames, 7))
        ep = np.zeros((self.n_rig, 7))
        pts = np.zeros((self.n_pts, 3))
        ic = np.zeros(self.opts.max_iters + 1)
        pi = np.zeros(self.opts.max_iters, np.int32)
        rep = Report()
        rep.iter_cost = ic.ctypes.data_as(C.POINTER(C.c_double))
        rep.pcg_iters = pi.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ba_rig_get_result(self._h, _ptr(vp), _ptr(ep), _ptr(pts), C.byref(rep)))
        out = _report_dict(rep, vp, pts, ic, pi)
        out["qe"], out["te"] = ep[:, :4], ep[:, 4:]
        return out

    @classmethod
    def from_scene(cls, scene, stream=None, **kw):
        if "huber_delta" not in kw:
            kw["huber_delta"] = scene.huber_delta
        return cls(scene_desc(scene), options(**kw), stream)

    def solve(self):
        _check(lib().ba_solve(self._h))
        return self

    def reset(self):
        _check(lib().ba_reset(self._h))
        return self

    def solve_async(self):
        _check(lib().ba_solve_async(self._h))

    def refine(self, stages, rounds):
        """ba_refine: stages is a sequence of (huber_delta, cull_px[, "midpoint" | "dlt"]);
        returns one dict per (stage, round), stage-major."""
        st = (RefineStage * len(stages))(*[RefineStage(float(g[0]), float(g[1]),
                                                       TRI[g[2]] if len(g) > 2 else 0, 0) for g in stages])
        hist = (RefineRound * max(len(stages) * int(rounds), 1))()
        _check(lib().ba_refine(self._h, len(stages), st, int(rounds), hist))
        return [{f: getattr(h, f) for f, _ in RefineRound._fields_ if f != "reserved"}
                for h in hist[:len(stages) * int(rounds)]]

    def active(self):
        """Observations in the problem (1) or removed by culling (0), caller's order."""
        a = np.zeros(int(getattr(self._desc.desc, "n_obs", 0)), np.uint8)
        _check(lib().ba_get_active(self._h, a.ctypes.data_as(C.c_void_p)))
        return a

    def wait(self):
        _check(lib().ba_wait(self._h))

    def set_profiling(self, mask=-1, stride=1):
        """mask: -1 all kernels, 0 off, or a bit mask over kernel_times() order;
        stride: time every stride-th launch of each selected kernel."""
        m = int(mask)
        if m >= 2 ** 31:
            m -= 2 ** 32
        _check(lib().ba_set_profiling(self._h, m, int(stride)))
        return self

    def set_barrier_polls(self, polls):
        """Poll bound of the resident PCG's grid barrier (a test hook; 0 makes it give up at once)."""
        _check(lib().ba_set_barrier_polls(self._h, int(polls)))
        return self

    def debug_iteration(self):
        """ba_debug_iteration_export: one LM iteration from the current state and its
        intermediate quantities (S blocks in CSR, b, g_c, dc, g_p, dp, sqrt(w) r, J_c, J_p)."""
        info = self.info()
        cf, nnzb, n_obs = info["n_free_cams"], info["nnzb"], info["n_obs"]
        out = dict(S_rowptr=np.zeros(cf + 1, np.int32), S_col=np.zeros(max(nnzb, 1), np.int32),
                   S=np.zeros((max(nnzb, 1), 6, 6)), b=np.zeros(6 * cf), gc=np.zeros(6 * cf),
                   dc=np.zeros(6 * cf), gp=np.zeros((max(self.n_pts, 1), 3)), dp=np.zeros((max(self.n_pts, 1), 3)),
                   r=np.zeros((max(n_obs, 1), 2)), Jc=np.zeros((max(n_obs, 1), 2, 6)),
                   Jp=np.zeros((max(n_obs, 1), 2, 3)))
        d = DebugIteration()
        for k, a in out.items():
            ct = C.c_int32 if a.dtype == np.int32 else C.c_double
            setattr(d, k, a.ctypes.data_as(C.POINTER(ct)))
        _check(lib().ba_debug_iteration_export(self._h, C.byref(d)))
        out["S_col"], out["S"] = out["S_col"][:nnzb], out["S"][:nnzb]
        out["gp"], out["dp"] = out["gp"][:self.n_pts], out["dp"][:self.n_pts]
        out["r"], out["Jc"], out["Jp"] = out["r"][:n_obs], out["Jc"][:n_obs], out["Jp"][:n_obs]
        out.update(lam=d.lambda_, pcg_iters=d.pcg_iters, accepted=d.accepted)
        return out

    def info(self):
        i = ProblemInfo()
        _check(lib().ba_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in ProblemInfo._fields_}

    def kernel_times(self):
        n = 32
        names = (C.c_char_p * n)()
        ms = (C.c_double * n)()
        la = (C.c_int32 * n)()
        cnt = C.c_int32()
        _check(lib().ba_get_kernel_times(self._h, n, names, ms, la, C.byref(cnt)))
        return {names[i].decode(): (ms[i], la[i]) for i in range(cnt.value)}

    @property
    def nbytes(self):
        return int(lib().ba_problem_bytes(self._h))

    def report(self):
        """Report of the last solve without downloading the state."""
        ic = np.zeros(self.opts.max_iters + 1)
        pi = np.zeros(self.opts.max_iters, np.int32)
        rep = Report()
        rep.iter_cost = ic.ctypes.data_as(C.POINTER(C.c_double))
        rep.pcg_iters = pi.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ba_get_result(self._h, None, None, C.byref(rep)))
        return _report_dict(rep, np.zeros((0, 7)), None, ic, pi)

    def result(self):
        poses = np.zeros((self.n_cams, 7))
        pts = np.zeros((self.n_pts, 3))
        ic = np.zeros(self.opts.max_iters + 1)
        pi = np.zeros(self.opts.max_iters, np.int32)
        rep = Report()
        rep.iter_cost = ic.ctypes.data_as(C.POINTER(C.c_double))
        rep.pcg_iters = pi.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ba_get_result(self._h, _ptr(poses), _ptr(pts), C.byref(rep)))
        return _report_dict(rep, poses, pts, ic, pi)

    def close(self):
        if getattr(self, "_h", None):
            lib().ba_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def _report_dict(rep, poses, pts, ic, pi):
    it = rep.iters
    return dict(q=poses[:, :4], t=poses[:, 4:], X=pts, iters=it, accepted=rep.accepted,
                status=rep.status, n_masked=rep.n_masked, cost0=rep.cost0, cost=rep.cost,
                rms_px=rep.rms_px, lam=rep.lambda_, iter_cost=ic[:it + 1].copy(),
                pcg_iters=pi[:it].copy(), solve_ms=rep.solve_ms, setup_ms=rep.setup_ms)


def _pose_request(K, q0, t0, X, uv, keep):
    X = np.ascontiguousarray(X, dtype=np.float64)
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    keep.append((X, uv))
    r = PoseRequest()
    r.K = Intrinsics(*[float(v) for v in K])
    r.pose0 = Pose(*[float(v) for v in q0], *[float(v) for v in t0])
    r.n = X.shape[0]
    r.X = _ptr(X)
    r.uv = _ptr(uv)
    return r


def pose_batch(requests, iters=10, huber_delta=1.0, stream=None):
    """Pose-only Gauss-Newton for a list of synth.PoseRequest-like objects."""
    keep = []
    arr = (PoseRequest * len(requests))()
    for i, q in enumerate(requests):
        arr[i] = _pose_request(q.K, q.q0, q.t0, q.X, q.uv, keep)
    o = options(max_iters=iters, huber_delta=huber_delta)
    poses = np.zeros((len(requests), 7))
    status = np.zeros(len(requests), np.int32)
    cost = np.zeros(len(requests))
    ms = C.c_double()
    _check(lib().ba_pose_batch(len(requests), arr, C.byref(o), stream, _ptr(poses),
                               status.ctypes.data_as(C.POINTER(C.c_int32)),
                               cost.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ms)))
    return dict(q=poses[:, :4], t=poses[:, 4:], status=status, cost=cost, device_ms=ms.value)


def pose_batch_noalloc(requests, iters=10, huber_delta=1.0, stream=None):
    """pose_batch through ba_pose_batch_noalloc (staging in the library's fixed device array)."""
    keep = []
    arr = (PoseRequest * len(requests))()
    for i, q in enumerate(requests):
        arr[i] = _pose_request(q.K, q.q0, q.t0, q.X, q.uv, keep)
    o = options(max_iters=iters, huber_delta=huber_delta)
    poses = np.zeros((len(requests), 7))
    status = np.zeros(len(requests), np.int32)
    cost = np.zeros(len(requests))
    _check(lib().ba_pose_batch_noalloc(len(requests), arr, C.byref(o), stream, _ptr(poses),
                                       status.ctypes.data_as(C.POINTER(C.c_int32)),
                                       cost.ctypes.data_as(C.POINTER(C.c_double))))
    return dict(q=poses[:, :4], t=poses[:, 4:], status=status, cost=cost)


def analyse(desc: "_Desc", opts: "Options"):
    """ba_analyse: the symbolic analysis alone; returns (info dict, device bytes)."""
    i = ProblemInfo()
    b = C.c_int64()
    _check(lib().ba_analyse(C.byref(desc.desc), C.byref(opts), C.byref(i), C.byref(b)))
    return {f: getattr(i, f) for f, _ in ProblemInfo._fields_}, b.value


class Server:
    """Continuous-batching server (see ba_server_* in include/ba.h)."""

    def __init__(self, budget_bytes, max_slots, precision="f32", stream=None):
        h = C.c_void_p()
        self.precision = precision
        _check(lib().ba_server_create(int(budget_bytes), int(max_slots),
                                      PREC[precision] if isinstance(precision, str) else precision,
                                      stream, C.byref(h)))
        self._h = h
        self._meta = {}

    def submit(self, desc: _Desc, opts: Options) -> int:
        t = C.c_int64()
        _check(lib().ba_server_submit(self._h, C.byref(desc.desc), C.byref(opts), C.byref(t)))
        self._meta[t.value] = (desc.desc.n_cams, desc.desc.n_pts, opts.max_iters, False)
        return t.value

    def submit_pose(self, req, iters=10, huber_delta=1.0) -> int:
        keep = []
        r = _pose_request(req.K, req.q0, req.t0, req.X, req.uv, keep)
        o = options(max_iters=iters, huber_delta=huber_delta, precision=self.precision)
        t = C.c_int64()
        _check(lib().ba_server_submit_pose(self._h, C.byref(r), C.byref(o), C.byref(t)))
        self._meta[t.value] = (1, 0, iters, True)
        return t.value

    def wait(self, ticket):
        nc, npt, iters, is_pose = self._meta.pop(ticket)
        poses = np.zeros((nc, 7))
        pts = np.zeros((max(npt, 1), 3))
        ic = np.zeros(iters + 1)
        pi = np.zeros(max(iters, 1), np.int32)
        rep = Report()
        rep.iter_cost = ic.ctypes.data_as(C.POINTER(C.c_double))
        rep.pcg_iters = pi.ctypes.data_as(C.POINTER(C.c_int32))
        _check(lib().ba_server_wait(self._h, ticket, _ptr(poses), _ptr(pts), C.byref(rep)))
        d = _report_dict(rep, poses, pts[:npt], ic, pi)
        d["latency_ms"] = rep.solve_ms
        d["pose_only"] = is_pose
        return d

    def stats(self):
        s = ServerStats()
        _check(lib().ba_server_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().ba_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
