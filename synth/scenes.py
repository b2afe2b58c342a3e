"""Seeded synthetic scenes shaped like the paper's workloads.

The paper evaluates on driving sequences (sequential frames plus loop closures,
Sec. 3.4 and Sec. 6.2-6.3) and on localization against a prior map (Sec. 6.4.2).
Those datasets are not available, so every scene here is synthetic and seeded
with ``numpy.random.default_rng``.  Conventions shared with both solvers:

* pinhole camera, fx = fy = 500, cx = 320, cy = 240, image 640 x 480, pixel
  origin at the top-left corner, y pointing down;
* a pose is world -> camera: P_c = R X + t, stored as a unit quaternion
  (w, x, y, z) plus t;
* observations are (camera index, point index, u, v) in pixels.

Nothing in this module computes a residual, a Jacobian, a loss or a solve.  The
projections below are only used to decide which synthetic points a camera sees
and to write their synthetic pixel coordinates.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

FX = 500.0
FY = 500.0
CX = 320.0
CY = 240.0
IMG_W = 640.0
IMG_H = 480.0
MIN_DEPTH = 0.5  # metres; a synthetic point nearer than this is treated as not visible


@dataclasses.dataclass
class Scene:
    """One bundle-adjustment problem (all arrays float64 / int32 / uint8)."""
    name: str
    K: np.ndarray          # (C, 4) fx, fy, cx, cy per camera
    q_gt: np.ndarray       # (C, 4) ground-truth world->camera rotation, (w, x, y, z)
    t_gt: np.ndarray       # (C, 3)
    q0: np.ndarray         # (C, 4) initial (perturbed) rotation
    t0: np.ndarray         # (C, 3)
    X_gt: np.ndarray       # (P, 3)
    X0: np.ndarray         # (P, 3)
    obs_cam: np.ndarray    # (N,) int32
    obs_pt: np.ndarray     # (N,) int32
    obs_uv: np.ndarray     # (N, 2) float64 pixels
    cam_fixed: np.ndarray  # (C,) uint8
    outlier: np.ndarray    # (N,) bool, True where (u, v) was replaced by a uniform draw
    huber_delta: float     # <= 0: plain least squares
    sigma: float
    meta: dict

    @property
    def n_cams(self) -> int:
        return int(self.K.shape[0])

    @property
    def n_pts(self) -> int:
        return int(self.X0.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])


@dataclasses.dataclass
class PoseRequest:
    """One pose-only localization request against a fixed map."""
    K: np.ndarray        # (4,)
    q_gt: np.ndarray     # (4,)
    t_gt: np.ndarray     # (3,)
    q0: np.ndarray       # (4,)
    t0: np.ndarray       # (3,)
    X: np.ndarray        # (m, 3) map points, world frame
    uv: np.ndarray       # (m, 2)
    outlier: np.ndarray  # (m,) bool


# ----------------------------------------------------------------------------- helpers

def _rotvec_to_matrix(v: np.ndarray) -> np.ndarray:
    return Rotation.from_rotvec(np.asarray(v, dtype=np.float64)).as_matrix()


def _matrix_to_quat_wxyz(R: np.ndarray) -> np.ndarray:
    q = Rotation.from_matrix(R).as_quat()  # (x, y, z, w)
    q = np.atleast_2d(q)
    out = np.concatenate([q[:, 3:4], q[:, 0:3]], axis=1)
    out[out[:, 0] < 0] *= -1.0
    return out


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _cam_to_world_look(forward: np.ndarray) -> np.ndarray:
    """Camera-to-world rotation whose optical axis is ``forward`` (unit, in the
    x-z plane or close to it) with the image y axis along world +y (down)."""
    z = forward / np.linalg.norm(forward, axis=-1, keepdims=True)
    y = np.broadcast_to(np.array([0.0, 1.0, 0.0]), z.shape)
    x = np.cross(y, z)
    x = x / np.linalg.norm(x, axis=-1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=-1)  # columns x, y, z


def _in_view(R_cw: np.ndarray, c: np.ndarray, X: np.ndarray, K=(FX, FY, CX, CY)):
    """Visibility test used while synthesising data: depth > MIN_DEPTH and the
    synthetic pixel inside the image.  Returns (visible, u, v)."""
    fx, fy, cx, cy = K
    Pc = np.einsum("...ij,...j->...i", R_cw, X - c)
    z = Pc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * Pc[..., 0] / z + cx
        v = fy * Pc[..., 1] / z + cy
    vis = (z > MIN_DEPTH) & (u >= 0) & (u < IMG_W) & (v >= 0) & (v < IMG_H)
    return vis, u, v


def _finish(name, R_wc, c, Rt_wc, ct, X_gt, X0, cam, pt, uv, fixed, outlier, delta, sigma, meta,
            K=None) -> Scene:
    C = R_wc.shape[0]
    R_gt = np.transpose(R_wc, (0, 2, 1))
    t_gt = -np.einsum("nij,nj->ni", R_gt, c)
    R0 = np.transpose(Rt_wc, (0, 2, 1))
    t0 = -np.einsum("nij,nj->ni", R0, ct)
    if K is None:
        K = np.tile(np.array([FX, FY, CX, CY]), (C, 1))
    return Scene(
        name=name, K=np.ascontiguousarray(K, dtype=np.float64),
        q_gt=_matrix_to_quat_wxyz(R_gt), t_gt=t_gt,
        q0=_matrix_to_quat_wxyz(R0), t0=t0,
        X_gt=np.ascontiguousarray(X_gt, dtype=np.float64),
        X0=np.ascontiguousarray(X0, dtype=np.float64),
        obs_cam=np.ascontiguousarray(cam, dtype=np.int32),
        obs_pt=np.ascontiguousarray(pt, dtype=np.int32),
        obs_uv=np.ascontiguousarray(uv, dtype=np.float64),
        cam_fixed=np.ascontiguousarray(fixed, dtype=np.uint8),
        outlier=np.ascontiguousarray(outlier, dtype=bool),
        huber_delta=float(delta), sigma=float(sigma), meta=meta)


# ----------------------------------------------------------------------------- arc scenes

def make_arc_scene(n_cams: int, n_pts: int, seed: int, sigma: float = 0.5,
                   rot_perturb: float = 0.01, trans_perturb: float = 0.05,
                   point_perturb: float = 0.05, outlier_frac: float = 0.0,
                   huber_delta: float = 0.0, noiseless: bool = False,
                   name: str | None = None) -> Scene:
    """Cameras on a 2 m arc (radius 6 m about the box centre (0, 0, 6), angles in
    [-1/6, 1/6] rad), each looking at the box centre; points uniform in
    x, y in [-2, 2], z in [2, 10].  Every in-image projection is an observation.
    Camera 0 is fixed and left unperturbed."""
    rng = np.random.default_rng(seed)
    centre = np.array([0.0, 0.0, 6.0])
    if n_cams == 1:
        ang = np.zeros(1)
    else:
        ang = np.linspace(-1.0 / 6.0, 1.0 / 6.0, n_cams)
    c = np.stack([6.0 * np.sin(ang), np.zeros_like(ang), 6.0 - 6.0 * np.cos(ang)], axis=1)
    R_wc = _cam_to_world_look(centre[None, :] - c)
    X = np.stack([rng.uniform(-2, 2, n_pts), rng.uniform(-2, 2, n_pts),
                  rng.uniform(2, 10, n_pts)], axis=1)
    cams, pts, us, vs = [], [], [], []
    for i in range(n_cams):
        vis, u, v = _in_view(R_wc[i].T[None], c[i][None], X)
        idx = np.nonzero(vis)[0]
        cams.append(np.full(idx.size, i, np.int32))
        pts.append(idx.astype(np.int32))
        us.append(u[idx])
        vs.append(v[idx])
    cam = np.concatenate(cams)
    pt = np.concatenate(pts)
    uv = np.stack([np.concatenate(us), np.concatenate(vs)], axis=1)
    if not noiseless:
        uv = uv + sigma * rng.standard_normal(uv.shape)
    outlier = np.zeros(cam.size, bool)
    if outlier_frac > 0 and not noiseless:
        outlier = rng.random(cam.size) < outlier_frac
        k = int(outlier.sum())
        uv[outlier] = np.stack([rng.uniform(0, IMG_W, k), rng.uniform(0, IMG_H, k)], axis=1)
    # initial state: camera 0 fixed and exact; others rotated by Exp(rot * u_hat) on the
    # world->camera side and shifted by trans * v_hat; points shifted by point * w_hat.
    R_cw = np.transpose(R_wc, (0, 2, 1))
    t_cw = -np.einsum("nij,nj->ni", R_cw, c)
    dr = _unit_vectors(rng, n_cams) * rot_perturb
    dt = _unit_vectors(rng, n_cams) * trans_perturb
    dr[0] = 0.0
    dt[0] = 0.0
    R0_cw = np.einsum("nij,njk->nik", _rotvec_to_matrix(dr), R_cw)
    t0_cw = t_cw + dt
    X0 = X + _unit_vectors(rng, n_pts) * point_perturb
    # express initial poses through camera-to-world for _finish
    Rt_wc = np.transpose(R0_cw, (0, 2, 1))
    ct = -np.einsum("nij,nj->ni", Rt_wc, t0_cw)
    fixed = np.zeros(n_cams, np.uint8)
    fixed[0] = 1
    meta = dict(kind="arc", seed=seed, n_cams=n_cams, n_pts=n_pts)
    return _finish(name or f"arc_{n_cams}x{n_pts}", R_wc, c, Rt_wc, ct, X, X0, cam, pt, uv,
                   fixed, outlier, huber_delta, sigma, meta)


def make_config0(noiseless: bool = False) -> Scene:
    """Tiny problem: 10 cameras, 1000 points, sigma 0.5 px, camera 0 fixed."""
    return make_arc_scene(10, 1000, seed=1000, sigma=0.5, noiseless=noiseless, name="config0")


def make_config3_sizes(n_problems: int = 512, seed: int = 1003):
    """Camera and point counts of the serving stream: log-uniform in [5, 200]
    cameras and [1e3, 5e4] points, drawn independently."""
    rng = np.random.default_rng(seed)
    nc = np.floor(np.exp(rng.uniform(math.log(5), math.log(200), n_problems))).astype(int)
    npts = np.floor(np.exp(rng.uniform(math.log(1e3), math.log(5e4), n_problems))).astype(int)
    return nc, npts


def make_config3_problem(r: int, n_cams: int, n_pts: int) -> Scene:
    return make_arc_scene(n_cams, n_pts, seed=10000 * 3 + r, sigma=0.5, name=f"config3_{r}")


# ----------------------------------------------------------------------------- driving scenes

def _drive_poses(headings: np.ndarray, lateral: np.ndarray | None = None,
                 start: np.ndarray | None = None):
    """Positions by integrating 1 m steps along the heading (x-z plane)."""
    n = headings.size
    steps = np.stack([np.sin(headings), np.zeros(n), np.cos(headings)], axis=1)
    c = np.zeros((n, 3))
    if start is not None:
        c[0] = start
    c[1:] = c[0] + np.cumsum(steps[:-1], axis=0)
    if lateral is not None:
        side = np.stack([np.cos(headings), np.zeros(n), -np.sin(headings)], axis=1)
        c = c + lateral[:, None] * side
    R_wc = _cam_to_world_look(steps)
    return R_wc, c


def _place_tracks(rng, R_wc, c, starts, lengths, depth_lo, depth_hi, max_tries=20):
    """Place one point per track so that every frame of the track sees it.

    A pixel is drawn uniformly and back-projected at a uniform depth from the
    last frame of the track; if any frame of the track does not see the point,
    the pixel and depth are drawn again (up to ``max_tries`` times), after which
    the track is shortened to the suffix of frames that see the last draw."""
    n = starts.size
    X = np.zeros((n, 3))
    L = lengths.copy()
    todo = np.arange(n)
    for _ in range(max_tries):
        if todo.size == 0:
            break
        e = starts[todo] + L[todo] - 1
        u = rng.uniform(0, IMG_W, todo.size)
        v = rng.uniform(0, IMG_H, todo.size)
        d = rng.uniform(depth_lo, depth_hi, todo.size)
        ray = np.stack([(u - CX) / FX, (v - CY) / FY, np.ones(todo.size)], axis=1) * d[:, None]
        Xt = c[e] + np.einsum("nij,nj->ni", R_wc[e], ray)
        X[todo] = Xt
        ok = np.ones(todo.size, bool)
        for o in range(int(L[todo].max())):
            m = o < L[todo]
            f = starts[todo] + o
            f = np.where(m, f, 0)
            vis, _, _ = _in_view(np.transpose(R_wc[f], (0, 2, 1)), c[f], Xt)
            ok &= vis | ~m
        todo = todo[~ok]
    # shorten the remaining tracks to the visible suffix ending at the last frame
    for i in todo:
        e = starts[i] + L[i] - 1
        k = 0
        while k < L[i]:
            f = e - k
            vis, _, _ = _in_view(R_wc[f].T[None], c[f][None], X[i][None])
            if not vis[0]:
                break
            k += 1
        starts[i] = e - k + 1
        L[i] = k
    return X, starts, L


def _drift(rng, n: int, rot_step: float, trans_step: float):
    """Cumulative random-walk drift; frame 0 gets none."""
    w = rng.normal(0.0, rot_step, (n, 3))
    tau = rng.normal(0.0, trans_step, (n, 3))
    w[0] = 0.0
    tau[0] = 0.0
    return np.cumsum(w, axis=0), np.cumsum(tau, axis=0)


def _drive_scene(name, rng, R_wc, c, segs, X, sigma, outlier_frac, huber_delta,
                 rot_step, trans_step, point_sigma, meta):
    """segs: list of (point index array, start frame array, length array); the first
    segment of every point defines the frame used for its initial position."""
    C = c.shape[0]
    cams, pts = [], []
    for pidx, s, L in segs:
        for o in range(int(L.max()) if L.size else 0):
            m = o < L
            cams.append((s[m] + o).astype(np.int32))
            pts.append(pidx[m].astype(np.int32))
    cam = np.concatenate(cams)
    pt = np.concatenate(pts)
    # drop observations a second segment cannot see
    R_cw = np.transpose(R_wc, (0, 2, 1))
    vis, u, v = _in_view(R_cw[cam], c[cam], X[pt])
    cam, pt, u, v = cam[vis], pt[vis], u[vis], v[vis]
    order = np.lexsort((pt, cam))  # camera-major order, as an image database would hold it
    cam, pt, u, v = cam[order], pt[order], u[order], v[order]
    uv = np.stack([u, v], axis=1) + sigma * rng.standard_normal((cam.size, 2))
    outlier = np.zeros(cam.size, bool)
    if outlier_frac > 0:
        outlier = rng.random(cam.size) < outlier_frac
        k = int(outlier.sum())
        uv[outlier] = np.stack([rng.uniform(0, IMG_W, k), rng.uniform(0, IMG_H, k)], axis=1)
    # drifted initial trajectory (camera-to-world side), frame 0 exact and fixed
    wdr, tdr = _drift(rng, C, rot_step, trans_step)
    Rt_wc = np.einsum("nij,njk->nik", _rotvec_to_matrix(wdr), R_wc)
    ct = c + tdr
    # initial points: true point seen from its first frame, carried to the world with
    # the drifted pose of that frame, plus isotropic noise
    first = np.full(X.shape[0], -1, np.int64)
    for pidx, s, L in reversed(segs):
        first[pidx] = s
    Pc = np.einsum("nij,nj->ni", R_cw[first], X - c[first])
    X0 = np.einsum("nij,nj->ni", Rt_wc[first], Pc) + ct[first]
    X0 = X0 + rng.normal(0.0, point_sigma, X0.shape)
    fixed = np.zeros(C, np.uint8)
    fixed[0] = 1
    meta = dict(meta)
    meta.update(n_obs=int(cam.size))
    return _finish(name, R_wc, c, Rt_wc, ct, X, X0, cam, pt, uv, fixed, outlier,
                   huber_delta, sigma, meta)


def _track_lengths(rng, n, p, n_frames, starts):
    L = 1 + rng.geometric(p, n)
    return np.minimum(L, n_frames - starts)


def make_config1(n_pts: int = 250_000, n_cams: int = 500, seed: int = 1001,
                 sigma: float = 0.7, name: str | None = None, outlier_frac: float = 0.0,
                 huber_delta: float = 0.0) -> Scene:
    """Sequential drive: cameras 1 m apart along a curve with heading
    0.3 sin(2 pi s / 500) rad, optical axis along the direction of travel; track
    length 1 + Geom(1/7) over consecutive frames (mean 8); points 3-40 m from the
    last frame of their track; drift 0.002 rad and 0.01 m per frame per axis.
    The default 250k points gives about 2M observations; 200k is the literal count.
    outlier_frac > 0 replaces that fraction of the pixels by uniform ones."""
    rng = np.random.default_rng(seed)
    s_idx = np.arange(n_cams, dtype=np.float64)
    R_wc, c = _drive_poses(0.3 * np.sin(2 * np.pi * s_idx / 500.0))
    starts = rng.integers(0, n_cams - 1, n_pts)
    L = _track_lengths(rng, n_pts, 1.0 / 7.0, n_cams, starts)
    X, starts, L = _place_tracks(rng, R_wc, c, starts, L, 3.0, 40.0)
    keep = L >= 2
    pidx = np.arange(n_pts)
    # points whose visible suffix fell below two frames are dropped and the rest renumbered
    remap = np.cumsum(keep) - 1
    X = X[keep]
    segs = [(remap[pidx[keep]], starts[keep], L[keep])]
    meta = dict(kind="drive", seed=seed, n_cams=n_cams, n_pts_requested=n_pts,
                n_pts=int(keep.sum()), mean_track=float(L[keep].mean()))
    return _drive_scene(name or f"config1_{n_pts}", rng, R_wc, c, segs, X, sigma, outlier_frac,
                        huber_delta, 0.002, 0.01, 0.05, meta)


def make_small_drive(n_cams: int = 40, n_pts: int = 3000, seed: int = 77, sigma: float = 0.7,
                     outlier_frac: float = 0.0, huber_delta: float = 0.0,
                     mean_track: float = 8.0, name: str | None = None) -> Scene:
    """A short sequential drive with the same recipe as the 2M-observation scene,
    sized for oracle-speed tests (several tiles and ragged tails)."""
    rng = np.random.default_rng(seed)
    s_idx = np.arange(n_cams, dtype=np.float64)
    R_wc, c = _drive_poses(0.3 * np.sin(2 * np.pi * s_idx / 500.0))
    starts = rng.integers(0, n_cams - 1, n_pts)
    L = _track_lengths(rng, n_pts, 1.0 / (mean_track - 1.0), n_cams, starts)
    X, starts, L = _place_tracks(rng, R_wc, c, starts, L, 3.0, 40.0)
    keep = L >= 2
    remap = np.cumsum(keep) - 1
    X = X[keep]
    segs = [(remap[np.arange(n_pts)[keep]], starts[keep], L[keep])]
    meta = dict(kind="drive", seed=seed, n_cams=n_cams, n_pts=int(keep.sum()))
    return _drive_scene(name or f"drive_{n_cams}x{n_pts}", rng, R_wc, c, segs, X, sigma,
                        outlier_frac, huber_delta, 0.002, 0.01, 0.05, meta)


def make_config2(n_pts: int = 1_500_000, laps_frames: int = 1500, seed: int = 1002,
                 sigma: float = 0.7, outlier_frac: float = 0.05, overlap_frac: float = 0.25,
                 name: str | None = None) -> Scene:
    """Loop-closed drive: one closed circular loop of ``laps_frames`` frames (1 m
    apart) driven twice, the second pass 1 m to the inside; 3000 cameras in all.
    Track length 1 + Geom(1/5) (mean 6).  ``overlap_frac`` of the points are seen on
    both passes (one track segment per pass, at corresponding frames), which puts
    loop-closure blocks into the reduced camera system.  5 % of observations are
    replaced by uniform outliers; Huber delta 1 px."""
    rng = np.random.default_rng(seed)
    n = laps_frames
    h = 2 * np.pi * np.arange(n) / n
    radius = n / (2 * np.pi)
    R1, c1 = _drive_poses(h, start=np.array([0.0, 0.0, 0.0]))
    # exact circle (integration of 1 m chords is close to it; use the closed form so the
    # second pass retraces the first)
    c1 = np.stack([radius * (1 - np.cos(h)), np.zeros(n), radius * np.sin(h)], axis=1)
    inward = np.stack([np.cos(h), np.zeros(n), -np.sin(h)], axis=1)  # camera +x, towards the centre
    c2 = c1 + 1.0 * inward
    R_wc = np.concatenate([R1, R1], axis=0)
    c = np.concatenate([c1, c2], axis=0)
    C = 2 * n
    n_loop = int(round(overlap_frac * n_pts))
    n_single = n_pts - n_loop
    # single-pass points anywhere along the 2n frames
    s_a = rng.integers(0, C - 1, n_single)
    L_a = _track_lengths(rng, n_single, 1.0 / 5.0, C, s_a)
    X_a, s_a, L_a = _place_tracks(rng, R_wc, c, s_a, L_a, 3.0, 40.0)
    # loop points: placed on pass 1, re-observed on pass 2 at corresponding frames
    s_b = rng.integers(0, n - 1, n_loop)
    L_b = _track_lengths(rng, n_loop, 1.0 / 5.0, n, s_b)
    X_b, s_b, L_b = _place_tracks(rng, R_wc[:n], c[:n], s_b, L_b, 3.0, 40.0)
    keep_a = L_a >= 2
    keep_b = L_b >= 2
    X = np.concatenate([X_a[keep_a], X_b[keep_b]], axis=0)
    ia = np.arange(int(keep_a.sum()))
    ib = np.arange(int(keep_b.sum())) + ia.size
    segs = [(ia, s_a[keep_a], L_a[keep_a]),
            (ib, s_b[keep_b], L_b[keep_b]),
            (ib, s_b[keep_b] + n, L_b[keep_b])]
    meta = dict(kind="loop", seed=seed, n_cams=C, n_pts=int(X.shape[0]),
                n_loop_pts=int(keep_b.sum()))
    return _drive_scene(name or "config2", rng, R_wc, c, segs, X, sigma, outlier_frac, 1.0,
                        0.002, 0.01, 0.05, meta)


# ----------------------------------------------------------------------------- pose-only

def make_config4_requests(n_req: int = 4096, seed: int = 1004, sigma: float = 1.0,
                          outlier_frac: float = 0.10, m_lo: int = 100, m_hi: int = 2000,
                          rot_perturb: float = 0.01, trans_perturb: float = 0.05,
                          noiseless: bool = False):
    """Pose-only localization requests: m = floor(exp U(ln m_lo, ln m_hi))
    correspondences each; map points back-projected from uniform pixels at uniform
    depth in [2, 30] m under a random ground-truth pose; sigma 1 px; 10 % outliers;
    initial pose perturbed by 0.01 rad and 0.05 m."""
    rng = np.random.default_rng(seed)
    ms = np.floor(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), n_req))).astype(int)
    reqs = []
    for r in range(n_req):
        rr = np.random.default_rng(10000 * 4 + r + (seed - 1004) * 1_000_003)
        m = int(ms[r])
        R_wc = _rotvec_to_matrix(rr.normal(0, 0.5, 3))
        cpos = rr.normal(0, 10.0, 3)
        u = rr.uniform(0, IMG_W, m)
        v = rr.uniform(0, IMG_H, m)
        d = rr.uniform(2.0, 30.0, m)
        ray = np.stack([(u - CX) / FX, (v - CY) / FY, np.ones(m)], axis=1) * d[:, None]
        X = ray @ R_wc.T + cpos
        uv = np.stack([u, v], axis=1)
        if not noiseless:
            uv = uv + sigma * rr.standard_normal((m, 2))
        out = np.zeros(m, bool)
        if outlier_frac > 0 and not noiseless:
            out = rr.random(m) < outlier_frac
            k = int(out.sum())
            uv[out] = np.stack([rr.uniform(0, IMG_W, k), rr.uniform(0, IMG_H, k)], axis=1)
        R_cw = R_wc.T
        t_cw = -R_cw @ cpos
        R0 = _rotvec_to_matrix(_unit_vectors(rr, 1)[0] * rot_perturb) @ R_cw
        t0 = t_cw + _unit_vectors(rr, 1)[0] * trans_perturb
        reqs.append(PoseRequest(K=np.array([FX, FY, CX, CY]),
                                q_gt=_matrix_to_quat_wxyz(R_cw)[0], t_gt=t_cw,
                                q0=_matrix_to_quat_wxyz(R0)[0], t0=t0,
                                X=X, uv=uv, outlier=out))
    return reqs


# ----------------------------------------------------------------------------- storage

def save_scene(path: str, s: Scene) -> None:
    np.savez(path, name=s.name, K=s.K, q_gt=s.q_gt, t_gt=s.t_gt, q0=s.q0, t0=s.t0,
             X_gt=s.X_gt, X0=s.X0, obs_cam=s.obs_cam, obs_pt=s.obs_pt, obs_uv=s.obs_uv,
             cam_fixed=s.cam_fixed, outlier=s.outlier, huber_delta=s.huber_delta,
             sigma=s.sigma)


def load_scene(path: str) -> Scene:
    z = np.load(path, allow_pickle=False)
    return Scene(name=str(z["name"]), K=z["K"], q_gt=z["q_gt"], t_gt=z["t_gt"], q0=z["q0"],
                 t0=z["t0"], X_gt=z["X_gt"], X0=z["X0"], obs_cam=z["obs_cam"],
                 obs_pt=z["obs_pt"], obs_uv=z["obs_uv"], cam_fixed=z["cam_fixed"],
                 outlier=z["outlier"], huber_delta=float(z["huber_delta"]),
                 sigma=float(z["sigma"]), meta={})


# ----------------------------------------------------------------------------- pose graphs

@dataclasses.dataclass
class PoseGraph:
    """A pose graph: nodes with ground-truth and initial world->node poses, hard-fixed
    nodes, and edges (i, j) with a measured relative pose of T_i T_j^-1 and the
    weights of its rotation and translation entries."""
    name: str
    q_gt: np.ndarray      # (n, 4) ground-truth world->node rotation (w, x, y, z)
    t_gt: np.ndarray      # (n, 3)
    q0: np.ndarray        # (n, 4) initial poses (integrated noisy odometry)
    t0: np.ndarray        # (n, 3)
    fixed: np.ndarray     # (n,) uint8
    edge_i: np.ndarray    # (E,) int32
    edge_j: np.ndarray    # (E,) int32
    meas_q: np.ndarray    # (E, 4) measured relative rotation
    meas_t: np.ndarray    # (E, 3) measured relative translation
    w_rot: np.ndarray     # (E,)
    w_trans: np.ndarray   # (E,)
    edge_type: np.ndarray  # (E,) int32: 0 sequential, 1 loop closure, 2 extrinsic
    meta: dict

    @property
    def n_nodes(self) -> int:
        return int(self.q0.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edge_i.shape[0])


EDGE_SEQUENTIAL, EDGE_LOOP, EDGE_EXTRINSIC = 0, 1, 2


def _rig_extrinsics(n_rig: int):
    """Vehicle->camera transforms of a rig: camera c yawed by c * 60 degrees
    (alternating sides) about the vehicle's down axis, mounted 0.5 m from the
    vehicle origin along its optical axis."""
    yaws = [0.0] + [(1 if k % 2 else -1) * 60.0 * ((k + 1) // 2) for k in range(1, n_rig)]
    out = []
    for yaw in yaws:
        Ry = Rotation.from_euler("y", yaw, degrees=True)  # camera axes in the vehicle frame
        p = Ry.apply(np.array([0.0, 0.0, 0.5]))
        R_e = Ry.inv()
        out.append((R_e, -R_e.apply(p)))
    return out


def make_pose_graph(n_frames: int = 1500, laps: int = 2, n_rig: int = 3, mode: str = "camera",
                    seq_k: int = 2, loop_every: int = 2, odo_rot: float = 1e-3, odo_trans: float = 1e-2,
                    loop_rot: float = 1e-3, loop_trans: float = 2e-2, weight_scale: float = 1e-4,
                    seed: int = 1005, noiseless: bool = False, name: str | None = None) -> PoseGraph:
    """Pose graph of a vehicle with an ``n_rig``-camera rig driving a circular loop of
    ``n_frames`` frames (1 m apart) ``laps`` times, each lap 1 m inside the previous one.

    Nodes: one per camera and frame (``mode="camera"``) or one per frame with the
    vehicle pose (``mode="rig"``).  The initial trajectory integrates odometry whose
    per-frame relative motions carry Gaussian noise (odo_rot rad, odo_trans m per
    axis, as a left perturbation).  Edges:
      - sequential: node pairs of frames f, f + k (k = 1..seq_k, same camera), measured
        from the initial trajectory;
      - loop closure: every ``loop_every``-th frame of laps 2.. with the frame at the same
        angle one lap earlier (front camera, or vehicle in rig mode), measured as the
        true relative pose with noise (loop_rot, loop_trans);
      - extrinsic (camera mode): the front camera with each other camera of the same
        frame, measured by the exact rig calibration.
    Weights are weight_scale / sigma^2 of each entry group; extrinsic edges get 100
    times the sequential ones.  Node 0 is fixed.  Pose compositions here only
    synthesise measurements (scipy Rotation); no solver arithmetic lives here."""
    rng = np.random.default_rng(seed)
    T = n_frames * laps
    f = np.arange(T)
    h = 2 * np.pi * (f % n_frames) / n_frames
    radius = n_frames / (2 * np.pi)
    lap = f // n_frames
    c = np.stack([radius * (1 - np.cos(h)), np.zeros(T), radius * np.sin(h)], axis=1)
    c = c + lap[:, None] * np.stack([np.cos(h), np.zeros(T), -np.sin(h)], axis=1)
    fwd = np.stack([np.sin(h), np.zeros(T), np.cos(h)], axis=1)
    R_wv = _cam_to_world_look(fwd)              # vehicle-to-world rotation per frame
    Rv = Rotation.from_matrix(np.transpose(R_wv, (0, 2, 1)))  # world->vehicle
    tv = -Rv.apply(c)
    # noisy odometry: D_f = T_{f+1} T_f^-1 perturbed on the left, integrated from frame 0
    Rd = Rv[1:] * Rv[:-1].inv()
    td = tv[1:] - Rd.apply(tv[:-1])
    if noiseless:
        nr, nt = np.zeros((T - 1, 3)), np.zeros((T - 1, 3))
    else:
        nr, nt = rng.normal(0.0, odo_rot, (T - 1, 3)), rng.normal(0.0, odo_trans, (T - 1, 3))
    En = Rotation.from_rotvec(nr)
    Rd_n = En * Rd
    td_n = En.apply(td) + nt
    R0 = [Rv[0]]
    t0 = [tv[0]]
    for k in range(T - 1):
        R0.append(Rd_n[k] * R0[-1])
        t0.append(Rd_n[k].apply(t0[-1]) + td_n[k])
    R0 = Rotation.concatenate(R0)
    t0 = np.array(t0)
    ext = _rig_extrinsics(n_rig) if mode == "camera" else [(Rotation.identity(), np.zeros(3))]
    nc = len(ext)

    def node_pose(Rw, tw, cam):
        Re, te = ext[cam]
        return Re * Rw, Re.apply(tw) + te

    def node(fr, cam):
        return fr * nc + cam

    gt = [node_pose(Rv[fr], tv[fr], cam) for fr in range(T) for cam in range(nc)]
    ini = [node_pose(R0[fr], t0[fr], cam) for fr in range(T) for cam in range(nc)]
    R_gt = Rotation.concatenate([g[0] for g in gt])
    t_gt = np.array([g[1] for g in gt])
    R_in = Rotation.concatenate([g[0] for g in ini])
    t_in = np.array([g[1] for g in ini])

    def rel(Ra, ta, Rb, tb):  # A = T_a T_b^-1
        RA = Ra * Rb.inv()
        return RA, ta - RA.apply(tb)

    ei, ej, mq, mt, wr, wt, ty = [], [], [], [], [], [], []

    def add(i, j, RA, tA, w_r, w_t, typ):
        ei.append(i)
        ej.append(j)
        mq.append(RA.as_quat()[[3, 0, 1, 2]])
        mt.append(tA)
        wr.append(w_r)
        wt.append(w_t)
        ty.append(typ)

    ws_r, ws_t = weight_scale / odo_rot ** 2, weight_scale / odo_trans ** 2
    for fr in range(T):
        for k in range(1, seq_k + 1):
            if fr + k >= T:
                continue
            for cam in range(nc):
                a, b = node(fr, cam), node(fr + k, cam)
                RA, tA = rel(R_in[a], t_in[a], R_in[b], t_in[b])
                add(a, b, RA, tA, ws_r, ws_t, EDGE_SEQUENTIAL)
    for fr in range(n_frames, T):
        if (fr - n_frames) % loop_every:
            continue
        a, b = node(fr, 0), node(fr - n_frames, 0)
        RA, tA = rel(R_gt[a], t_gt[a], R_gt[b], t_gt[b])
        if not noiseless:
            E = Rotation.from_rotvec(rng.normal(0.0, loop_rot, 3))
            RA, tA = E * RA, E.apply(tA) + rng.normal(0.0, loop_trans, 3)
        add(a, b, RA, tA, weight_scale / loop_rot ** 2, weight_scale / loop_trans ** 2, EDGE_LOOP)
    if nc > 1:
        for fr in range(T):
            for cam in range(1, nc):
                a, b = node(fr, 0), node(fr, cam)
                RA, tA = rel(ext[0][0], ext[0][1], ext[cam][0], ext[cam][1])
                add(a, b, RA, tA, 100 * ws_r, 100 * ws_t, EDGE_EXTRINSIC)
    n = T * nc
    fixed = np.zeros(n, np.uint8)
    fixed[0] = 1
    q_gt = R_gt.as_quat()[:, [3, 0, 1, 2]]
    q0 = R_in.as_quat()[:, [3, 0, 1, 2]]
    meta = dict(kind="pose_graph", mode=mode, n_frames=n_frames, laps=laps, n_rig=n_rig, seq_k=seq_k,
                seed=seed, n_nodes=n, n_edges=len(ei))
    return PoseGraph(name=name or f"pose_graph_{mode}_{T}x{nc}", q_gt=q_gt, t_gt=t_gt, q0=q0, t0=t_in,
                     fixed=fixed, edge_i=np.array(ei, np.int32), edge_j=np.array(ej, np.int32),
                     meas_q=np.array(mq), meas_t=np.array(mt), w_rot=np.array(wr), w_trans=np.array(wt),
                     edge_type=np.array(ty, np.int32), meta=meta)


# ----------------------------------------------------------------------------- vehicle-rig drives

@dataclasses.dataclass
class RigScene:
    """Observations of a multi-camera rig on a vehicle: rig camera c at frame f has the
    world->camera pose E_c T_v(f) (extrinsic E_c = vehicle -> camera, T_v(f) = world ->
    vehicle).  Quaternions are (w, x, y, z)."""
    name: str
    K: np.ndarray          # (nr, 4)
    qv_gt: np.ndarray      # (F, 4) world -> vehicle
    tv_gt: np.ndarray      # (F, 3)
    qe_gt: np.ndarray      # (nr, 4) vehicle -> camera
    te_gt: np.ndarray      # (nr, 3)
    qv0: np.ndarray        # initial vehicle poses (drifted)
    tv0: np.ndarray
    qe0: np.ndarray        # initial extrinsics (calibration error)
    te0: np.ndarray
    X_gt: np.ndarray       # (P, 3)
    X0: np.ndarray
    frame: np.ndarray      # (N,) int32
    rcam: np.ndarray       # (N,) int32
    obs_pt: np.ndarray     # (N,) int32
    obs_uv: np.ndarray     # (N, 2)
    fixed_v: np.ndarray    # (F,) uint8
    fixed_e: np.ndarray    # (nr,) uint8
    sigma: float
    meta: dict

    @property
    def n_frames(self) -> int:
        return int(self.qv0.shape[0])

    @property
    def n_rig(self) -> int:
        return int(self.qe0.shape[0])

    @property
    def n_pts(self) -> int:
        return int(self.X0.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.frame.shape[0])


def make_rig_drive(n_frames: int = 200, n_pts: int = 20000, n_rig: int = 3, seed: int = 1006,
                   sigma: float = 0.7, ext_rot: float = 0.01, ext_trans: float = 0.02,
                   mean_track: float = 8.0, cross_frames: int = 20, name: str | None = None) -> RigScene:
    """A drive of ``n_frames`` frames 1 m apart (heading 0.3 sin(2 pi s / 500), as the
    sequential drive) with an ``n_rig``-camera rig (yaws 0, +-60 degrees, 0.5 m from the
    vehicle origin).  Each point is tracked by one rig camera over consecutive frames
    (track length 1 + Geom, mean ``mean_track``, points 3-40 m away); the other rig
    cameras observe it too wherever it is in their view during the track's frames and
    the ``cross_frames`` frames after them (a point ahead of the vehicle passes into a
    side camera), which ties the extrinsics together.  Pixel noise sigma.
    Initial state: vehicle poses with the drive's random-walk drift (0.002 rad, 0.01 m
    per frame), extrinsics off their true values by Exp of (ext_trans, ext_rot) noise per
    axis (the calibration error the refinement corrects), points carried with the
    drifted pose plus 0.05 m noise.  Frame 0 is fixed; the extrinsics are free."""
    rng = np.random.default_rng(seed)
    s_idx = np.arange(n_frames, dtype=np.float64)
    R_wv, cv = _drive_poses(0.3 * np.sin(2 * np.pi * s_idx / 500.0))
    ext = _rig_extrinsics(n_rig)
    Rv = Rotation.from_matrix(np.transpose(R_wv, (0, 2, 1)))
    tv = -Rv.apply(cv)
    cams, pts, uvs, Xs, tracks = [], [], [], [], []
    per = n_pts // n_rig
    base = 0
    for c, (Re, te) in enumerate(ext):
        Rc = Re * Rv                          # world -> camera c at every frame
        tcm = Re.apply(tv) + te
        R_wc = np.transpose(Rc.as_matrix(), (0, 2, 1))
        cc = -np.einsum("nij,nj->ni", R_wc, tcm)  # camera centres
        starts = rng.integers(0, n_frames - 1, per)
        L = _track_lengths(rng, per, 1.0 / (mean_track - 1.0), n_frames, starts)
        X, starts, L = _place_tracks(rng, R_wc, cc, starts, L, 3.0, 40.0)
        keep = L >= 2
        X, starts, L = X[keep], starts[keep], L[keep]
        tracks.append((base, X, starts, L, c))
        Xs.append(X)
        base += X.shape[0]
    # every rig camera's view of every point over its track's frames (plus cross_frames)
    cam_R_wc, cam_c = [], []
    for Re, te in ext:
        Rc = Re * Rv
        R_wc = np.transpose(Rc.as_matrix(), (0, 2, 1))
        cam_R_wc.append(R_wc)
        cam_c.append(-np.einsum("nij,nj->ni", R_wc, Re.apply(tv) + te))
    for b0, X, starts, L, c0 in tracks:
        for c in range(n_rig):
            span = L if c == c0 else np.minimum(L + cross_frames, n_frames - starts)
            for o in range(int(span.max()) if span.size else 0):
                m = o < span
                f = (starts[m] + o).astype(np.int32)
                j = np.nonzero(m)[0]
                vis, u, v = _in_view(np.transpose(cam_R_wc[c][f], (0, 2, 1)), cam_c[c][f], X[j])
                cams.append(np.stack([f[vis], np.full(int(vis.sum()), c, np.int32)], axis=1))
                pts.append((b0 + j[vis]).astype(np.int32))
                uvs.append(np.stack([u[vis], v[vis]], axis=1))
    fc = np.concatenate(cams)
    pt = np.concatenate(pts)
    uv = np.concatenate(uvs) + sigma * rng.standard_normal((pt.size, 2))
    X_gt = np.concatenate(Xs)
    # drifted vehicle trajectory (frame 0 exact), perturbed extrinsics
    wdr, tdr = _drift(rng, n_frames, 0.002, 0.01)
    Rt_wv = np.einsum("nij,njk->nik", _rotvec_to_matrix(wdr), R_wv)
    ct = cv + tdr
    Rv0 = Rotation.from_matrix(np.transpose(Rt_wv, (0, 2, 1)))
    tv0 = -Rv0.apply(ct)
    Ee = [(Rotation.from_rotvec(rng.normal(0, ext_rot, 3)) * Re, te + rng.normal(0, ext_trans, 3))
          for Re, te in ext]
    # initial points: true point seen from its first frame and camera, carried with the
    # drifted vehicle pose and the perturbed extrinsic of that camera
    first_f = np.zeros(X_gt.shape[0], np.int64)
    cam_of = np.zeros(X_gt.shape[0], np.int32)
    for b0, X, starts, L, c0 in tracks:
        first_f[b0:b0 + X.shape[0]] = starts
        cam_of[b0:b0 + X.shape[0]] = c0
    X0 = np.empty_like(X_gt)
    for c, (Re, te) in enumerate(ext):
        m = cam_of == c
        f = first_f[m]
        Pc = Re.apply(Rv[f].apply(X_gt[m]) + tv[f]) + te          # true camera frame
        Re0, te0 = Ee[c]
        Pv = Re0.inv().apply(Pc - te0)                                 # through the initial extrinsic
        X0[m] = Rv0[f].inv().apply(Pv - tv0[f])                        # and the drifted vehicle pose
    X0 = X0 + rng.normal(0.0, 0.05, X0.shape)
    fixed_v = np.zeros(n_frames, np.uint8)
    fixed_v[0] = 1
    q = lambda R: R.as_quat()[..., [3, 0, 1, 2]]
    meta = dict(kind="rig_drive", seed=seed, n_frames=n_frames, n_rig=n_rig, n_pts=int(X_gt.shape[0]),
                n_obs=int(pt.size))
    return RigScene(name=name or f"rig_drive_{n_frames}x{n_rig}", K=np.tile(np.array([FX, FY, CX, CY]), (n_rig, 1)),
                    qv_gt=q(Rv), tv_gt=tv, qe_gt=np.stack([q(R) for R, _ in ext]),
                    te_gt=np.stack([t for _, t in ext]), qv0=q(Rv0), tv0=tv0,
                    qe0=np.stack([q(R) for R, _ in Ee]), te0=np.stack([t for _, t in Ee]),
                    X_gt=X_gt, X0=X0, frame=fc[:, 0].astype(np.int32), rcam=fc[:, 1].astype(np.int32),
                    obs_pt=pt, obs_uv=uv, fixed_v=fixed_v, fixed_e=np.zeros(n_rig, np.uint8),
                    sigma=float(sigma), meta=meta)
