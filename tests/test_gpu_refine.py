"""Iterative refinement on the device (BA rounds alternating with culling by a
reprojection threshold and midpoint re-triangulation, robust then strict stage)
against the FP64 oracle, through the C-ABI.  Needs an MI355X."""
import sys

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_config1, make_small_drive

pytestmark = pytest.mark.gpu

# robust stage: Huber 1 px, outliers beyond 8 px; strict stage: no loss, 3 px
STAGES = [(1.0, 8.0), (0.0, 3.0)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(res):
    return O.quat_to_rot(res["q"]), res["t"], res["X"]


def test_refine_f64_matches_oracle_round_by_round(balib):
    """10 % uniform outliers on a 20-camera drive, FP64, two stages of two rounds:
    every round's final cost within 1e-9 of the oracle's, the active-observation
    and point counts equal, the final mask identical and the final state within
    1e-7.  Rounds drop points (two-observation tracks with an outlier) and cull
    whole tracks, the degenerate cases of the step."""
    s = make_small_drive(20, 1000, seed=61, outlier_frac=0.1, huber_delta=1.0)
    ref, hist = O.refine(O.Problem.from_scene(s), STAGES, 2, O.LMOptions(max_iters=6, solve="exact"))
    _say("device refine f64:", s.name, s.n_obs)
    p = balib.Problem.from_scene(s, max_iters=6, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64")
    dh = p.refine(STAGES, 2)
    act = p.active()
    res = p.result()
    for h, (si, rd, cost, na, npt) in zip(dh, hist):
        _say("round", si, rd, "cost", h["cost"], cost, "obs", h["n_active_obs"], na, "pts", h["n_active_pts"], npt)
        assert (h["stage"], h["round"]) == (si, rd)
        assert abs(h["cost"] - cost) <= 1e-9 * cost
        assert (h["n_active_obs"], h["n_active_pts"]) == (na, npt)
    assert hist[0][4] < s.n_pts  # some points left the problem
    assert np.array_equal(act.astype(bool), ref.active)
    R, t, X = _state(res)
    assert np.max(np.abs(X - ref.X)) <= 1e-7 * (1 + np.max(np.abs(ref.X)))
    assert np.max(np.abs(R - ref.R)) <= 1e-7
    assert np.max(np.abs(t - ref.t)) <= 1e-7 * (1 + np.max(np.abs(ref.t)))
    # the report's rms is over the observations still in the problem
    assert abs(res["rms_px"] - O.rms(ref)) <= 1e-6 * O.rms(ref)
    # reset puts every observation back
    p.reset()
    assert p.active().all()
    p.close()


def test_refine_f32_removes_outliers_to_noise_level(balib):
    """FP32 with the benchmark's PCG schedule on a 60-camera drive with 10 %
    outliers: at least 99 % of the planted outliers are out, the RMS over what
    remains matches sigma sqrt((2N - d)/N) within 5 %, and the final mask agrees
    with the FP64 oracle run with the same schedule on 99.9 % of observations."""
    s = make_small_drive(60, 6000, seed=62, outlier_frac=0.1, huber_delta=1.0)
    opts = O.LMOptions(max_iters=8, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6)
    ref, hist = O.refine(O.Problem.from_scene(s), STAGES, 2, opts)
    _say("device refine f32:", s.name, s.n_obs)
    p = balib.Problem.from_scene(s, max_iters=8, precision="f32")
    dh = p.refine(STAGES, 2)
    act = p.active().astype(bool)
    res = p.result()
    p.close()
    removed = (~act & s.outlier).sum() / s.outlier.sum()
    n = int(act.sum())
    pts = int(np.count_nonzero(np.bincount(s.obs_pt[act], minlength=s.n_pts) > 0))
    d = 6 * int((s.cam_fixed == 0).sum()) + 3 * pts - 1
    expected = s.sigma * np.sqrt((2 * n - d) / n)
    agree = np.mean(act == ref.active)
    _say("outliers removed", removed, "rms", res["rms_px"], "expected", expected, "mask agreement", agree,
         [(h["n_active_obs"], h["n_active_pts"]) for h in dh], [(h[3], h[4]) for h in hist])
    assert removed >= 0.99
    assert abs(res["rms_px"] - expected) <= 0.05 * expected
    assert agree >= 0.999
    assert dh[-1]["n_active_obs"] == n and dh[-1]["n_active_pts"] == pts


def test_refine_full_size_culling_matches_oracle_at_device_state(balib):
    """The 2M-observation drive with 5 % outliers, FP32, one robust round (Huber
    1 px, 10 LM iterations, cull at 8 px).  A second problem solved the same way
    gives the state the culling step saw (solves are deterministic).  Against the
    oracle at that state: every decision on an observation of a point that lost
    none, and every kept observation, agrees with the oracle's FP64 threshold test
    except within 1e-3 px of the threshold (the device reads FP32 pixels); each
    point that lost one was re-triangulated or dropped, and for 200 sampled such
    points the oracle's midpoint from the same observations gives the same outcome
    and the same point within 1e-4 relative."""
    s = make_config1(outlier_frac=0.05, huber_delta=1.0)
    tau = 8.0
    _say("device refine full size:", s.name, s.n_obs)
    a = balib.Problem.from_scene(s, max_iters=10, precision="f32")
    h = a.refine([(1.0, tau)], 1)[0]
    act = a.active().astype(bool)
    Xa = a.result()["X"]
    a.close()
    _say("device solve at the same settings")
    b = balib.Problem.from_scene(s, max_iters=10, precision="f32")
    rb = b.solve().result()
    b.close()
    assert rb["cost"] == h["cost"]
    p = O.Problem.from_scene(s)
    R, t, X = _state(rb)
    r, valid, _ = O.residuals(p, R, t, X)
    norm = np.sqrt(np.sum(r * r, axis=1))
    keep = valid & (norm <= tau)
    near = np.abs(norm - tau) <= 1e-3
    lost_pt = np.zeros(s.n_pts, bool)
    lost_pt[s.obs_pt[~keep & ~near]] = True
    # observations of points that lost none: same decision
    m = ~lost_pt[s.obs_pt] & ~near
    assert np.array_equal(act[m], keep[m])
    # kept observations pass the threshold
    assert np.all(keep[act & ~near])
    # points that lost an observation: all of the threshold survivors kept, or none
    dropped = np.zeros(s.n_pts, bool)
    cnt_keep = np.bincount(s.obs_pt[keep], minlength=s.n_pts)
    cnt_act = np.bincount(s.obs_pt[act], minlength=s.n_pts)
    lp = np.nonzero(lost_pt)[0]
    ok_counts = (cnt_act[lp] == 0) | (cnt_act[lp] == cnt_keep[lp])
    dropped[lp] = cnt_act[lp] == 0
    _say("lost points", lp.size, "dropped", int(dropped.sum()), "count mismatches", int((~ok_counts).sum()))
    assert ok_counts.mean() >= 0.999
    assert h["n_active_obs"] == int(act.sum())
    rng = np.random.default_rng(5)
    sample = rng.choice(lp[ok_counts], size=min(200, int(ok_counts.sum())), replace=False)
    q = O.Problem.from_scene(s)
    q.R, q.t, q.X = R, t, X.copy()
    q.active = keep.copy()
    bad = 0
    for j in sample:
        Xo, ok = O.triangulate_midpoint(q, int(j)) if cnt_keep[j] >= 2 else (None, False)
        if ok != (not dropped[j]):
            bad += 1
            continue
        if ok:
            assert np.linalg.norm(Xa[j] - Xo) <= 1e-4 * np.linalg.norm(Xo)
    _say("sampled re-triangulations", sample.size, "outcome mismatches", bad)
    assert bad <= 1


@pytest.mark.parametrize("method,tol", [("midpoint", 1e-8), ("dlt", 1e-7)])
def test_triangulate_from_scratch_matches_oracle(balib, method, tol):
    """ba_triangulate on a 20-camera drive at the true poses (noisy pixels): the same
    points succeed as in the oracle and each point agrees within the stated relative
    tolerance: FP64 rounding times the conditioning of the short-baseline systems (the
    3x3 midpoint matrix reaches condition numbers near 1e6 on tracks along the direction
    of travel; the DLT's 4x4 normal matrix squares the conditioning of A)."""
    s = make_small_drive(20, 1000, seed=71)
    p = O.Problem.from_scene(s)
    p.R, p.t = O.quat_to_rot(s.q_gt), np.array(s.t_gt)
    ref, ok_ref = O.triangulate_points(p, method)
    d = balib.scene_desc(s)
    d.poses[:, :4], d.poses[:, 4:] = s.q_gt, s.t_gt
    _say("device triangulation:", method, s.n_pts)
    X, ok, ms = balib.triangulate(d, method)
    assert np.array_equal(ok, ok_ref)
    err = np.linalg.norm(X[ok] - ref[ok], axis=1) / (1 + np.linalg.norm(ref[ok], axis=1))
    _say(method, "ok", int(ok.sum()), "max rel err", err.max(), "device ms", ms)
    assert err.max() <= tol
    assert np.array_equal(X[~ok], s.X0[~ok])


@pytest.mark.parametrize("method", ["midpoint", "dlt"])
def test_triangulate_full_size_sampled(balib, method):
    """All 250k points of the 2M-observation drive at the true poses in one launch; 300
    sampled points against the oracle (midpoint 1e-8, DLT 1e-6 relative; outcome equal)."""
    s = make_config1()
    d = balib.scene_desc(s)
    d.poses[:, :4], d.poses[:, 4:] = s.q_gt, s.t_gt
    _say("device triangulation full size:", method, s.n_pts, s.n_obs)
    X, ok, ms = balib.triangulate(d, method)
    p = O.Problem.from_scene(s)
    p.R, p.t = O.quat_to_rot(s.q_gt), np.array(s.t_gt)
    f = O.triangulate_midpoint if method == "midpoint" else O.triangulate_dlt
    tol = 1e-8 if method == "midpoint" else 1e-6
    rng = np.random.default_rng(2)
    worst, bad = 0.0, 0
    for j in rng.choice(s.n_pts, 300, replace=False):
        Xo, oko = f(p, int(j))
        if oko != ok[j]:
            bad += 1
            continue
        if oko:
            worst = max(worst, np.linalg.norm(X[j] - Xo) / (1 + np.linalg.norm(Xo)))
    _say(method, "ok", int(ok.sum()), "of", s.n_pts, "sample max rel err", worst, "outcome mismatches", bad,
         "device ms", ms)
    assert bad == 0 and worst <= tol


def test_refine_dlt_f64_matches_oracle(balib):
    """The refinement with DLT re-triangulation, FP64: round counts and costs as the
    oracle's (1e-9) and the final mask identical."""
    s = make_small_drive(20, 1000, seed=61, outlier_frac=0.1, huber_delta=1.0)
    stages = [(1.0, 8.0, "dlt"), (0.0, 3.0, "dlt")]
    ref, hist = O.refine(O.Problem.from_scene(s), stages, 2, O.LMOptions(max_iters=6, solve="exact"))
    p = balib.Problem.from_scene(s, max_iters=6, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64")
    dh = p.refine(stages, 2)
    act = p.active()
    p.close()
    for h, (si, rd, cost, na, npt) in zip(dh, hist):
        _say("dlt round", si, rd, h["cost"], cost, h["n_active_obs"], na, h["n_active_pts"], npt)
        assert abs(h["cost"] - cost) <= 1e-9 * cost
        assert (h["n_active_obs"], h["n_active_pts"]) == (na, npt)
    assert np.array_equal(act.astype(bool), ref.active)


@pytest.mark.parametrize("method,tol", [("midpoint", 1e-7), ("dlt", 1e-7)])
def test_ransac_triangulation_matches_oracle(balib, method, tol):
    """ba_triangulate_ransac on a 20-camera drive with 10 % uniform outliers at the true
    poses (64 hypotheses, 3 px): the same tracks succeed, every inlier flag agrees with
    the oracle's, and the points agree within 1e-7 relative: FP64 rounding times the
    conditioning of the final solve, which for a track whose inliers are two adjacent
    frames along the direction of travel approaches 1e8 (measured: midpoint 7.6e-9,
    DLT 3.1e-11)."""
    s = make_small_drive(20, 1000, seed=72, outlier_frac=0.1)
    p = O.Problem.from_scene(s)
    p.R, p.t = O.quat_to_rot(s.q_gt), np.array(s.t_gt)
    d = balib.scene_desc(s)
    d.poses[:, :4], d.poses[:, 4:] = s.q_gt, s.t_gt
    _say("device ransac triangulation:", method, s.n_pts, s.n_obs)
    X, ok, inl, ms = balib.triangulate_ransac(d, 3.0, 64, method)
    ref_ok = np.zeros(s.n_pts, bool)
    ref_in = np.zeros(s.n_obs, bool)
    worst = 0.0
    for j in range(s.n_pts):
        Xo, oko, ino = O.triangulate_ransac(p, j, 3.0, 64, method)
        ref_ok[j] = oko
        ref_in[np.nonzero(p.pt == j)[0]] = ino
        if oko and ok[j]:
            worst = max(worst, np.linalg.norm(X[j] - Xo) / (1 + np.linalg.norm(Xo)))
    _say(method, "ok", int(ok.sum()), "inliers", int(inl.sum()), "outliers flagged",
         float((~inl & s.outlier).sum() / s.outlier.sum()), "max rel err", worst, "device ms", ms)
    assert np.array_equal(ok, ref_ok) and np.array_equal(inl, ref_in)
    assert worst <= tol


def test_ransac_triangulation_full_size_sampled(balib):
    """All 250k tracks of the 2M-observation drive with 5 % outliers at the true poses in
    one launch (midpoint, 64 hypotheses, 3 px); 60 sampled tracks against the oracle:
    outcome and inlier flags identical, points within 1e-8."""
    s = make_config1(outlier_frac=0.05, huber_delta=1.0)
    d = balib.scene_desc(s)
    d.poses[:, :4], d.poses[:, 4:] = s.q_gt, s.t_gt
    _say("device ransac triangulation full size:", s.n_pts, s.n_obs)
    X, ok, inl, ms = balib.triangulate_ransac(d, 3.0, 64)
    p = O.Problem.from_scene(s)
    p.R, p.t = O.quat_to_rot(s.q_gt), np.array(s.t_gt)
    rng = np.random.default_rng(4)
    worst = 0.0
    for j in rng.choice(s.n_pts, 60, replace=False):
        Xo, oko, ino = O.triangulate_ransac(p, int(j), 3.0, 64)
        assert oko == ok[j]
        assert np.array_equal(ino, inl[np.nonzero(p.pt == j)[0]])
        if oko:
            worst = max(worst, np.linalg.norm(X[j] - Xo) / (1 + np.linalg.norm(Xo)))
    _say("ok", int(ok.sum()), "outliers flagged", float((~inl & s.outlier).sum() / s.outlier.sum()),
         "inliers kept", float((inl & ~s.outlier).sum() / (~s.outlier).sum()), "max rel err", worst, "device ms", ms)
    assert worst <= 1e-8
