"""Pose-graph optimisation on the device (nodes and relative-pose edges through the
LM / reduced-system / PCG path) against the FP64 oracle, through the C-ABI.
Needs an MI355X."""
import sys

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_pose_graph

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_problem(g, prior_abs=0.0):
    return O.pose_graph_problem(O.quat_to_rot(g.q0), g.t0, g.fixed, np.stack([g.edge_i, g.edge_j], axis=1),
                                O.quat_to_rot(g.meas_q), g.meas_t, g.w_rot, g.w_trans, prior_abs=prior_abs)


def _solve(balib, g, **kw):
    _say("device pose graph:", g.name, g.n_nodes, g.n_edges, kw)
    p = balib.Problem.from_pose_graph(g, **kw)
    info = p.info()
    res = p.solve().result()
    p.close()
    return res, info


@pytest.mark.parametrize("mode,flags,prior_abs", [("camera", 0, 0.0), ("camera", 4, 0.0),
                                                   ("rig", 0, 0.0), ("camera", 0, 0.5)])
def test_pose_graph_f64_per_iteration_cost(balib, mode, flags, prior_abs):
    """24 frames of a 3-camera rig (72 nodes; sequential k = 1, 2, loop-closure edges
    pointing backwards, extrinsic edges) or the same drive as 24 rig nodes, FP64, 15
    LM iterations: every C_n within 1e-9 of the oracle solved exactly, and the final
    poses within 1e-8; in both Schur forms, and with an absolute prior."""
    g = make_pose_graph(12, mode=mode)
    ref = O.lm_schur(_oracle_problem(g, prior_abs), O.LMOptions(max_iters=15, solve="exact"))
    res, info = _solve(balib, g, max_iters=15, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64",
                       flags=flags, prior_abs=prior_abs)
    assert info["n_pts"] == 0 and info["n_obs"] == 0
    assert info["schur_form"] == (0 if flags & 4 else 1)
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say("max rel cost diff", rel.max(), "cost", ref.iter_cost[0], "->", ref.iter_cost[-1])
    assert rel.max() <= 1e-9
    assert ref.iter_cost[-1] < 0.75 * ref.iter_cost[0]
    R = O.quat_to_rot(res["q"])
    assert np.max(np.abs(R - ref.R)) <= 1e-8 and np.max(np.abs(res["t"] - ref.t)) <= 1e-8 * (1 + np.abs(ref.t).max())
    assert res["n_masked"] == 0 and res["rms_px"] == 0.0


@pytest.mark.parametrize("flags,rows", [(0, 16), (8, 32)])
def test_pose_graph_sparse_tiles_f64_pcg_schedule(balib, flags, rows):
    """1080 nodes (360 frames of the 3-camera rig): the reduced system has many sparse
    rows, so the PCG runs 16 rows per workgroup (32, half a wave per row, with
    BA_FLAG_PCG_WIDE).  FP64 with PCG capped at 100 products and tol 1e-8 against the
    oracle's textbook PCG with the same schedule: PCG counts identical and every C_n
    within 1e-8."""
    g = make_pose_graph(180)
    ref = O.lm_schur(_oracle_problem(g), O.LMOptions(max_iters=6, solve="pcg", pcg_max_iters=100,
                                                     pcg_rel_tol=1e-8))
    res, info = _solve(balib, g, max_iters=6, pcg_max_iters=100, pcg_rel_tol=1e-8, precision="f64",
                       flags=flags)
    assert info["pcg_rows"] == rows
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say("sparse tiles: max rel cost diff", rel.max(), list(res["pcg_iters"]), ref.pcg_iters)
    assert list(res["pcg_iters"]) == list(ref.pcg_iters)
    assert rel.max() <= 1e-8


def test_pose_graph_f32_final_cost(balib):
    """600 nodes, 1641 edges, FP32 with the benchmark's PCG schedule (50 / 1e-6), 10
    iterations: the final cost within 1e-4 of the FP64 oracle run with that schedule,
    recomputed by the oracle at the device's state."""
    g = make_pose_graph(100)
    p = _oracle_problem(g)
    ref = O.lm_schur(p, O.LMOptions(max_iters=10, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6))
    res, _ = _solve(balib, g, max_iters=10, precision="f32")
    c_dev = O.prior_cost(p, O.quat_to_rot(res["q"]), res["t"])
    _say("f32 pose graph", c_dev, ref.iter_cost[-1], res["pcg_iters"])
    assert abs(c_dev - ref.iter_cost[-1]) <= 1e-4 * ref.iter_cost[-1]
    assert abs(res["cost"] - c_dev) <= 1e-5 * c_dev


def test_pose_graph_full_size_cost_matches_oracle_at_device_state(balib):
    """The benchmark's graph (3000 frames of a 3-camera rig: 9000 nodes, 24,741 edges),
    FP32, 10 LM iterations, PCG 50 / 1e-6: the accepted costs never increase, the
    device's final cost equals the oracle's at the device state within 1e-5, and the
    loop closures pull the second lap onto the first (cost below half the start)."""
    g = make_pose_graph(1500)
    res, info = _solve(balib, g, max_iters=10, precision="f32")
    assert info["pcg_rows"] == 32
    p = _oracle_problem(g)
    c = O.prior_cost(p, O.quat_to_rot(res["q"]), res["t"])
    _say("full-size pose graph: device", res["cost"], "oracle", c, "start", res["iter_cost"][0], info["nnzb"])
    assert abs(res["cost"] - c) <= 1e-5 * c
    assert all(b <= a for a, b in zip(res["iter_cost"], res["iter_cost"][1:]))
    assert res["cost"] < 0.5 * res["iter_cost"][0]
