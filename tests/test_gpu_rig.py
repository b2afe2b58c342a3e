"""Vehicle-rig BA on the device (composed cameras through the BA kernels, projection
onto vehicle poses and shared extrinsics, rig PCG, rig update) against the FP64
oracle, through the C-ABI.  Needs an MI355X."""
import sys

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_rig_drive

pytestmark = pytest.mark.gpu

PAIRS = np.array([[0, 1], [0, 2]])


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(s, delta=0.0, **kw):
    return O.RigProblem(K=s.K, Rv=O.quat_to_rot(s.qv0), tv=np.array(s.tv0), Re=O.quat_to_rot(s.qe0),
                        te=np.array(s.te0), X=np.array(s.X0), frame=s.frame.astype(np.int64),
                        rcam=s.rcam.astype(np.int64), pt=s.obs_pt.astype(np.int64), uv=s.obs_uv,
                        fixed_v=s.fixed_v.astype(bool), fixed_e=s.fixed_e.astype(bool), delta=delta, **kw)


def _solve(balib, s, **kw):
    _say("device rig:", s.name, s.n_frames, s.n_rig, s.n_pts, s.n_obs, {k: v for k, v in kw.items() if k != "rig_pairs"})
    p = balib.Problem.from_rig(s, **kw)
    res = p.solve().rig_result()
    info = p.info()
    p.close()
    return res, info


@pytest.mark.parametrize("delta,flags", [(0.0, 0), (1.0, 0), (0.0, 4)])
def test_rig_f64_per_iteration_cost(balib, delta, flags):
    """12 frames of a 3-camera rig, extrinsic prior and rigidity pairs, FP64, 10 LM
    iterations: every C_n within 1e-9 of the oracle (dense solve of the rig system),
    vehicle poses and extrinsics within 1e-8; least squares and Huber, both Schur forms
    of the composed cameras."""
    s = make_rig_drive(12, 300, seed=21)
    q = _oracle(s, delta=delta, prior_ext=10.0, rig_pairs=PAIRS, prior_rig=10.0)
    ref = O.lm_rig(q, O.LMOptions(max_iters=10))
    res, info = _solve(balib, s, prior_ext=10.0, prior_rig=10.0, rig_pairs=PAIRS, max_iters=10, pcg_max_iters=400,
                       pcg_rel_tol=1e-14, precision="f64", huber_delta=delta, flags=flags)
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say("max rel cost diff", rel.max(), ref.iter_cost[0], "->", ref.iter_cost[-1], ref.accepted)
    assert rel.max() <= 1e-9
    Re, te = ref.ext
    assert np.max(np.abs(O.quat_to_rot(res["q"]) - ref.R)) <= 1e-8
    assert np.max(np.abs(res["t"] - ref.t)) <= 1e-8 * (1 + np.abs(ref.t).max())
    assert np.max(np.abs(O.quat_to_rot(res["qe"]) - Re)) <= 1e-8
    assert np.max(np.abs(res["te"] - te)) <= 1e-8


def test_rig_f64_one_extrinsic_fixed_no_priors(balib):
    """The gauge fixed by holding extrinsic 0 instead of priors: per-iteration cost
    within 1e-9 of the oracle."""
    s = make_rig_drive(10, 250, seed=22)
    s.fixed_e[0] = 1
    ref = O.lm_rig(_oracle(s), O.LMOptions(max_iters=8))
    res, _ = _solve(balib, s, max_iters=8, pcg_max_iters=400, pcg_rel_tol=1e-14, precision="f64")
    rel = np.abs(res["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    _say("max rel cost diff", rel.max())
    assert rel.max() <= 1e-9
    assert np.max(np.abs(O.quat_to_rot(res["qe"][0]) - O.quat_to_rot(s.qe0[0]))) <= 1e-14


def test_rig_f32_drive_cost_matches_oracle_at_device_state(balib):
    """200 frames of the 3-camera rig (the benchmark's rig workload), FP32, 10 LM
    iterations, PCG 50 / 1e-6: the device's cost equals the oracle's rig cost at the
    device's state within 1e-5, the accepted costs never increase, and the relative
    extrinsics E_c E_0^-1 end closer to the truth than they started."""
    s = make_rig_drive(200, 20000, seed=1006)
    res, info = _solve(balib, s, prior_ext=100.0, prior_rig=100.0, rig_pairs=PAIRS, max_iters=10, precision="f32")
    q = _oracle(s, prior_ext=100.0, rig_pairs=PAIRS, prior_rig=100.0)
    c, _ = O.rig_cost_and_masked(q, O.quat_to_rot(res["q"]), res["t"], O.quat_to_rot(res["qe"]), res["te"], res["X"])
    _say("rig f32: device", res["cost"], "oracle", c, "start", res["iter_cost"][0], info)
    assert abs(res["cost"] - c) <= 1e-5 * c
    assert all(b <= a for a, b in zip(res["iter_cost"], res["iter_cost"][1:]))

    def rel_err(qe, te):
        R = O.quat_to_rot(qe)
        Rg = O.quat_to_rot(s.qe_gt)
        return max(np.linalg.norm(R[k] @ R[0].T - Rg[k] @ Rg[0].T) for k in range(1, s.n_rig))

    e0, e1 = rel_err(s.qe0, s.te0), rel_err(res["qe"], res["te"])
    _say("relative extrinsic rotation error", e0, "->", e1)
    assert e1 < 0.5 * e0
