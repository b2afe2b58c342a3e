"""The resident PCG (BA_FLAG_PCG_RESIDENT: every iteration of a linear solve in one
launch, workgroups meeting at a grid barrier) against the launch-per-iteration PCG
and the FP64 oracle, through the C-ABI.  Needs an MI355X."""
import sys

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_config1, make_pose_graph, make_small_drive

pytestmark = pytest.mark.gpu

RESIDENT = 16  # BA_FLAG_PCG_RESIDENT


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(balib, scene, flags, **kw):
    _say("device solve:", scene.name, scene.n_cams, scene.n_pts, scene.n_obs, "flags", flags, kw)
    p = balib.Problem.from_scene(scene, flags=flags, **kw)
    info = p.info()
    res = p.solve().result()
    p.close()
    return info, res


def _same(a, b):
    assert np.array_equal(a["iter_cost"], b["iter_cost"])
    assert list(a["pcg_iters"]) == list(b["pcg_iters"])
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["t"], b["t"])
    assert np.array_equal(a["X"], b["X"])
    assert a["status"] == b["status"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("extra", [0, 2, 8, 64, 66])
def test_small_drive_resident_equals_per_launch(balib, prec, extra):
    """40-camera drive (10 tiles of 4 rows, the last ragged; with BA_FLAG_PCG_WIDE one
    full and one ragged 32-row tile; with BA_FLAG_NO_GRAPH launched without a graph;
    with BA_FLAG_PCG_COOPERATIVE started as a cooperative launch, in a graph or not):
    the resident solve repeats the per-launch solve bit for bit, and in FP64 every C_n
    is within 1e-9 of the explicit-Schur oracle solved exactly."""
    s = make_small_drive(40, 3000, seed=5)
    kw = dict(max_iters=8, pcg_max_iters=400, pcg_rel_tol=1e-14, precision=prec)
    ia, a = _run(balib, s, extra, **kw)
    ib, b = _run(balib, s, extra | RESIDENT, **kw)
    _say("info", ia["pcg_rows"], ia["pcg_resident"], ib["pcg_rows"], ib["pcg_resident"], "pcg", b["pcg_iters"])
    assert ia["pcg_resident"] == 0 and ib["pcg_resident"] == (2 if extra & 64 else 1)
    assert ib["pcg_rows"] == (32 if extra == 8 else 4)
    _same(a, b)
    if prec == "f64":
        ref = O.lm_schur(O.Problem.from_scene(s), O.LMOptions(max_iters=8, solve="exact"))
        rel = np.abs(b["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
        _say("max rel cost diff vs oracle", rel.max())
        assert rel.max() <= 1e-9


def test_small_drive_resident_early_stop_and_cap(balib):
    """A loose tolerance (the solve stops after a few iterations) and a cap of 3
    iterations: the resident solve stops where the per-launch one does."""
    s = make_small_drive(30, 2000, seed=21)
    for kw in (dict(pcg_rel_tol=1e-2, pcg_max_iters=50), dict(pcg_rel_tol=1e-12, pcg_max_iters=3)):
        _, a = _run(balib, s, 0, max_iters=5, precision="f32", **kw)
        _, b = _run(balib, s, RESIDENT, max_iters=5, precision="f32", **kw)
        _say(kw, "pcg", a["pcg_iters"], b["pcg_iters"])
        _same(a, b)


def test_full_size_drive_resident_equals_per_launch(balib):
    """The 2M-observation drive in the benchmark's configuration (FP32, 10 LM
    iterations, PCG 50 / 1e-6): 125 resident workgroups, the same run bit for bit as
    the launch-per-iteration PCG (also when started as a cooperative launch), and a
    cost that falls below half its start."""
    s = make_config1()
    ia, a = _run(balib, s, 0, max_iters=10, precision="f32")
    ib, b = _run(balib, s, RESIDENT, max_iters=10, precision="f32")
    _say("info", ib["pcg_rows"], ib["pcg_resident"], "rms", a["rms_px"], b["rms_px"], "pcg", b["pcg_iters"])
    assert ib["pcg_resident"] == 1
    _same(a, b)
    assert b["cost"] < 0.5 * b["cost0"]
    ic, c = _run(balib, s, RESIDENT | 64, max_iters=10, precision="f32")
    assert ic["pcg_resident"] == 2
    _same(a, c)


def test_pose_graph_too_many_tiles_falls_back(balib):
    """The 1500-frame rig pose graph has more 32-row tiles (282) than the device holds
    1024-thread workgroups at once: the flag is ignored and the solve is the
    per-launch one."""
    g = make_pose_graph(1500)
    out = []
    for flags in (0, RESIDENT):
        p = balib.Problem.from_pose_graph(g, max_iters=5, precision="f32", flags=flags)
        info = p.info()
        out.append((info, p.solve().result()))
        p.close()
    _say("tiles of", out[1][0]["pcg_rows"], "rows; resident", out[1][0]["pcg_resident"])
    assert out[1][0]["pcg_resident"] == 0
    assert np.array_equal(out[0][1]["iter_cost"], out[1][1]["iter_cost"])


def test_refine_resident_equals_per_launch(balib):
    """The two-stage refinement (robust Huber 1 px / 8 px culling, then strict 3 px) on
    a 60-camera drive with 10 % outliers, FP32, with the benchmark's PCG schedule: the
    resident PCG gives the same rounds, activity mask, poses and points bit for bit."""
    s = make_small_drive(60, 6000, seed=62, outlier_frac=0.1, huber_delta=1.0)
    out = []
    for flags in (0, RESIDENT):
        _say("device refine:", s.name, s.n_obs, "flags", flags)
        p = balib.Problem.from_scene(s, max_iters=8, precision="f32", flags=flags)
        info = p.info()
        hist = p.refine([(1.0, 8.0), (0.0, 3.0)], 2)
        out.append((info, hist, p.active().copy(), p.result()))
        p.close()
    (ia, ha, aa, ra), (ib, hb, ab, rb) = out
    _say("resident", ib["pcg_resident"], "rounds", [h["n_active_obs"] for h in hb])
    assert ia["pcg_resident"] == 0 and ib["pcg_resident"] == 1
    assert ha == hb
    assert np.array_equal(aa, ab)
    assert np.array_equal(ra["q"], rb["q"]) and np.array_equal(ra["t"], rb["t"])
    assert np.array_equal(ra["X"], rb["X"])


@pytest.mark.parametrize("coop", [0, 64])
def test_barrier_time_out_rejects_the_step_and_stops(balib, coop):
    """The barrier's poll bound set to 0 from the host (no workgroup is starved: each
    gives up at its first barrier and exits): the first LM iteration rejects its step
    and the solve ends there with BA_STATUS_PCG_SYNC, one iteration reported and the
    initial state kept.  With the default bound restored the next solve equals a
    fresh one bit for bit.  The same with a cooperative launch."""
    s = make_small_drive(40, 3000, seed=5)
    kw = dict(max_iters=6, precision="f32", flags=RESIDENT | coop)
    p = balib.Problem.from_scene(s, **kw)
    assert p.info()["pcg_resident"] == (2 if coop else 1)
    init = p.result()
    p.set_barrier_polls(0)
    _say("device solve: barrier poll bound 0")
    r = p.solve().result()
    _say("status", r["status"], "iters", r["iters"], "costs", r["iter_cost"], "pcg", r["pcg_iters"])
    assert r["status"] == balib.STATUS_PCG_SYNC
    assert r["iters"] == 1 and r["accepted"] == 0
    assert len(r["iter_cost"]) == 2 and r["iter_cost"][0] == r["iter_cost"][1] == r["cost0"] == r["cost"]
    assert np.array_equal(r["q"], init["q"]) and np.array_equal(r["t"], init["t"])
    assert np.array_equal(r["X"], init["X"])
    p.set_barrier_polls(1 << 20)
    b = p.reset().solve().result()
    p.close()
    _, a = _run(balib, s, RESIDENT, max_iters=6, precision="f32")
    assert b["status"] == 0 and b["iters"] == 6
    _same(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pose_graph_sixteen_row_tiles_resident_equals_per_launch(balib, prec):
    """1080-node pose graph: 16 reduced-system rows per workgroup (68 tiles, four waves
    reducing the partial sums); the resident solve repeats the per-launch one bit for bit."""
    g = make_pose_graph(180)
    out = []
    for flags in (0, RESIDENT):
        _say("device pose-graph solve: 1080 nodes, flags", flags, prec)
        p = balib.Problem.from_pose_graph(g, max_iters=6, pcg_max_iters=100, pcg_rel_tol=1e-8,
                                          precision=prec, flags=flags)
        info = p.info()
        out.append((info, p.solve().result()))
        p.close()
    (ia, a), (ib, b) = out
    _say("rows", ib["pcg_rows"], "resident", ib["pcg_resident"], "pcg", list(b["pcg_iters"]))
    assert ia["pcg_rows"] == 16 and ib["pcg_rows"] == 16
    assert ia["pcg_resident"] == 0 and ib["pcg_resident"] == 1
    assert np.array_equal(a["iter_cost"], b["iter_cost"])
    assert list(a["pcg_iters"]) == list(b["pcg_iters"])
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["t"], b["t"])
