"""The dense co-visibility Schur form (BA_FLAG_DENSE_SCHUR; chosen by itself when
every camera sees most points) against the FP64 oracle, through the C-ABI.  Its
products run on the matrix cores (FP64 / FP32 MFMA, FP16 / BF16 operands in the
16-bit storage modes).  Needs an MI355X."""
import sys

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_arc_scene, make_config0, make_small_drive

pytestmark = pytest.mark.gpu

DENSE = 32  # BA_FLAG_DENSE_SCHUR
PAIR_LISTS = 4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(balib, s, **kw):
    _say("device solve:", s.name, s.n_cams, s.n_pts, s.n_obs, kw)
    p = balib.Problem.from_scene(s, **kw)
    info = p.info()
    res = p.solve().result()
    p.close()
    return info, res


def _with_fixed(s, cams):
    s.cam_fixed = s.cam_fixed.copy()
    s.cam_fixed[list(cams)] = 1
    return s


def test_form_selection(balib):
    """Arc scenes (every camera sees most points) take the dense form; a sequential
    drive keeps the chunk form unless the flag forces the dense one; pair lists
    exclude it."""
    for s, flags, form in [(make_config0(), 0, 2), (make_small_drive(40, 3000, seed=5), 0, 1),
                           (make_small_drive(40, 3000, seed=5), DENSE, 2), (make_config0(), PAIR_LISTS, 0)]:
        p = balib.Problem.from_scene(s, flags=flags)
        info = p.info()
        p.close()
        _say(s.name, flags, "form", info["schur_form"], "pairs", info["n_pairs"], "nnzb", info["nnzb"])
        assert info["schur_form"] == form
        if form == 2:
            assert info["nnzb"] == info["n_free_cams"] ** 2


SCENES = [("config0", lambda: make_config0(), 0),
          # 3 camera tiles (16, 16, 8) with fixed cameras inside two of them
          ("arc40-fixed", lambda: _with_fixed(make_arc_scene(40, 1500, seed=71), [5, 21]), 0),
          # one camera tile, 5000 points in 4 point ranges
          ("arc12x5000", lambda: make_arc_scene(12, 5000, seed=72), 0),
          # forced on a drive: sparse co-visibility, zero rows in most tiles
          ("drive-forced", lambda: make_small_drive(40, 3000, seed=5), DENSE),
          ("huber-arc", lambda: make_arc_scene(20, 1500, seed=73, outlier_frac=0.05, huber_delta=1.0), 0)]


@pytest.mark.parametrize("name,make,flags", SCENES, ids=[c[0] for c in SCENES])
def test_dense_f64_per_iteration_cost_and_first_iteration(balib, name, make, flags):
    """FP64: every C_n of 12 LM iterations within 1e-9 of the explicit-Schur oracle
    solved exactly, and the first iteration's S, b, dc and dp element by element
    (S, b within 1e-12 of the largest magnitude; dc, dp within 1e-10 of the exact
    solve, the PCG run to 1e-14)."""
    s = make()
    ref = O.lm_schur(O.Problem.from_scene(s), O.LMOptions(max_iters=12, solve="exact"))
    kw = dict(max_iters=12, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64", flags=flags)
    info, res = _run(balib, s, **kw)
    assert info["schur_form"] == 2
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say(name, "max rel cost diff", rel.max(), "pcg", list(res["pcg_iters"]))
    assert rel.max() <= 1e-9
    # first iteration, element by element
    p = O.Problem.from_scene(s)
    H, g, _, _, _ = O.normal_equations(p)
    fidx, nf = O._free_index(p.fixed)
    ncam = 6 * nf
    D = O.damping_diag(H.diagonal())
    S, b, Vinv, W = O.schur_blocks(H, g, D, 1e-4, ncam)
    dc = np.linalg.solve(S, b)
    dp = np.asarray(Vinv @ (-g[ncam:] - W.T @ dc)).ravel().reshape(-1, 3)
    q = balib.Problem.from_scene(s, **{**kw, "max_iters": 1})
    dev = q.debug_iteration()
    q.close()
    Sd = np.zeros_like(S)
    for a in range(nf):
        for k in range(dev["S_rowptr"][a], dev["S_rowptr"][a + 1]):
            c = dev["S_col"][k]
            Sd[6 * a:6 * a + 6, 6 * c:6 * c + 6] = dev["S"][k]
    errs = {"S": np.abs(Sd - S).max() / np.abs(S).max(), "b": np.abs(dev["b"] - b).max() / np.abs(b).max(),
            "dc": np.abs(dev["dc"] - dc).max() / np.abs(dc).max(),
            "dp": np.abs(dev["dp"] - dp).max() / np.abs(dp).max()}
    _say(name, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["S"] <= 1e-12 and errs["b"] <= 1e-12
    assert errs["dc"] <= 1e-10 and errs["dp"] <= 1e-10


@pytest.mark.parametrize("prec", ["f32", "f16j", "bf16j"])
def test_dense_reduced_precision_final_rms(balib, prec):
    """30 cameras x 2000 points, 20 LM iterations with PCG 50 / 1e-6: the final RMS,
    recomputed by the oracle at the device's state, within 1e-3 px of the FP64
    oracle's run of the same schedule (FP32 products, FP16 / BF16 operands)."""
    s = make_arc_scene(30, 2000, seed=74)
    ref = O.lm_schur(O.Problem.from_scene(s), O.LMOptions(max_iters=20, solve="pcg", pcg_max_iters=50,
                                                          pcg_rel_tol=1e-6))
    info, res = _run(balib, s, max_iters=20, precision=prec)
    assert info["schur_form"] == 2
    p = O.Problem.from_scene(s)
    rms = O.rms(p, O.quat_to_rot(res["q"]), res["t"], res["X"])
    rms_ref = O.rms(p, ref.R, ref.t, ref.X)
    _say(prec, "rms", rms, "oracle", rms_ref, "reported", res["rms_px"])
    assert abs(rms - rms_ref) <= 1e-3


def test_dense_problems_in_a_served_mix(balib):
    """Dense-form problems among chunk-form ones in the server: each result equals,
    bit for bit, the same problem solved alone."""
    scenes = [make_arc_scene(24, 3000, seed=75), make_small_drive(30, 2000, seed=76),
              make_arc_scene(9, 800, seed=77), make_arc_scene(40, 1200, seed=78)]
    iters = [7, 6, 9, 5]
    srv = balib.Server(512 << 20, 3, precision="f32")
    tk = [srv.submit(balib.scene_desc(s), balib.options(max_iters=it, precision="f32"))
          for s, it in zip(scenes, iters)]
    res = [srv.wait(t) for t in tk]
    srv.close()
    for s, it, r in zip(scenes, iters, res):
        info, a = _run(balib, s, max_iters=it, precision="f32")
        _say(s.name, "form", info["schur_form"], "mix", r["iter_cost"][-1], "alone", a["iter_cost"][-1])
        assert np.array_equal(r["iter_cost"], a["iter_cost"])
        assert np.array_equal(r["X"], a["X"]) and np.array_equal(r["t"], a["t"])


def test_dense_with_resident_pcg_equals_per_launch(balib):
    """The dense form under the resident PCG (rows of 24 blocks, 6 tiles): the same
    run bit for bit as the launch-per-iteration PCG, in FP64 and FP32."""
    s = make_arc_scene(25, 2000, seed=79)
    for prec in ("f64", "f32"):
        out = []
        for flags in (0, 16):
            info, r = _run(balib, s, max_iters=6, precision=prec, flags=flags)
            out.append((info, r))
        (ia, a), (ib, b) = out
        assert ia["schur_form"] == ib["schur_form"] == 2
        assert ia["pcg_resident"] == 0 and ib["pcg_resident"] == 1
        assert np.array_equal(a["iter_cost"], b["iter_cost"])
        assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["q"], b["q"])
        assert list(a["pcg_iters"]) == list(b["pcg_iters"])


def test_dense_with_pose_priors_f64(balib):
    """Absolute and sequential pose priors (Sec. 4.3 objective) with the dense form,
    FP64: every C_n within 1e-9 of the explicit-Schur oracle."""
    s = make_arc_scene(18, 1200, seed=80)
    kw = dict(prior_abs=20.0, prior_seq=500.0, seq_k=3)
    ref = O.lm_schur(O.Problem.from_scene(s, **kw), O.LMOptions(max_iters=8, solve="exact"))
    info, res = _run(balib, s, max_iters=8, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64",
                     prior_abs=20.0, prior_seq=500.0, prior_seq_k=3)
    assert info["schur_form"] == 2
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say("dense priors rel", rel.max())
    assert rel.max() <= 1e-9


def test_dense_refine_f64_matches_oracle_round_by_round(balib):
    """The two-stage refinement (culling with midpoint re-triangulation) on an arc
    scene with 10 % outliers in the dense form, FP64: each round's cost within 1e-9 of
    the oracle's, the active counts equal and the final mask identical."""
    s = make_arc_scene(16, 1500, seed=81, outlier_frac=0.1, huber_delta=1.0)
    stages = [(1.0, 8.0), (0.0, 3.0)]
    ref, hist = O.refine(O.Problem.from_scene(s), stages, 2, O.LMOptions(max_iters=6, solve="exact"))
    p = balib.Problem.from_scene(s, max_iters=6, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64")
    assert p.info()["schur_form"] == 2
    dh = p.refine(stages, 2)
    act = p.active()
    p.close()
    for h, (si, rd, cost, na, npt) in zip(dh, hist):
        _say("round", si, rd, "cost", h["cost"], cost, "obs", h["n_active_obs"], na)
        assert abs(h["cost"] - cost) <= 1e-9 * cost
        assert (h["n_active_obs"], h["n_active_pts"]) == (na, npt)
    assert np.array_equal(act.astype(bool), ref.active)
