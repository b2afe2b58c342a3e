"""Serving loop (continuous batching under a device-memory budget) and the
pose-only batch, through the C-ABI.  Needs an MI355X."""
import sys
import time

import numpy as np
import pytest

from oracle import ba_oracle as O
from synth import make_arc_scene, make_config4_requests, make_small_drive

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mix():
    """Problems of uneven size: arc scenes (dense co-visibility) and short drives."""
    scenes = [make_arc_scene(5, 300, seed=101), make_arc_scene(12, 2000, seed=102),
              make_small_drive(30, 2000, seed=103), make_arc_scene(8, 700, seed=104),
              make_small_drive(45, 3500, seed=105), make_arc_scene(20, 1500, seed=106)]
    iters = [6, 10, 8, 12, 10, 7]
    return scenes, iters


def _alone(balib, s, iters, prec):
    p = balib.Problem.from_scene(s, max_iters=iters, precision=prec)
    r = p.solve().result()
    p.close()
    return r


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_each_result_is_identical_alone_and_in_the_mix(balib, prec):
    """Requests arrive while others run (a second wave is submitted after the
    first results come back); every result equals, bit for bit, the same problem
    solved alone.  Stated tolerance: 0 (all reductions are fixed-order)."""
    scenes, iters = _mix()
    srv = balib.Server(512 << 20, 4, precision=prec)
    t = []
    for s, it in zip(scenes[:3], iters[:3]):
        t.append(srv.submit(balib.scene_desc(s), balib.options(max_iters=it, precision=prec)))
    first = srv.wait(t[0])
    for s, it in zip(scenes[3:], iters[3:]):
        t.append(srv.submit(balib.scene_desc(s), balib.options(max_iters=it, precision=prec)))
    res = [first] + [srv.wait(x) for x in t[1:]]
    st = srv.stats()
    srv.close()
    _say("stats", st)
    assert st["done"] == len(scenes)
    for s, it, r in zip(scenes, iters, res):
        a = _alone(balib, s, it, prec)
        _say(s.name, "mix", r["iter_cost"][-1], "alone", a["iter_cost"][-1])
        assert r["iters"] == it
        assert np.array_equal(r["iter_cost"], a["iter_cost"])
        assert np.array_equal(r["X"], a["X"]) and np.array_equal(r["t"], a["t"])
        assert np.array_equal(r["pcg_iters"], a["pcg_iters"])


def test_server_results_match_oracle(balib):
    """FP64 through the server: per-iteration cost within 1e-9 of the oracle."""
    s = make_small_drive(25, 1500, seed=111)
    srv = balib.Server(256 << 20, 2, precision="f64")
    tk = srv.submit(balib.scene_desc(s), balib.options(max_iters=6, pcg_max_iters=300,
                                                       pcg_rel_tol=1e-14, precision="f64"))
    r = srv.wait(tk)
    srv.close()
    ref = O.lm_schur(O.Problem.from_scene(s), O.LMOptions(max_iters=6, solve="exact"))
    rel = np.abs(r["iter_cost"] - np.array(ref.iter_cost)) / np.array(ref.iter_cost)
    assert rel.max() <= 1e-9


def test_admission_respects_budget_and_slots(balib):
    """A budget that holds about two problems and one slot fewer than requests:
    every request completes, the peak never exceeds the budget, and a request
    larger than the whole budget is refused at submission."""
    scenes = [make_small_drive(30, 2500, seed=120 + i) for i in range(6)]
    p = balib.Problem.from_scene(scenes[0], max_iters=5)
    one = p.nbytes
    p.close()
    budget = int(2.5 * one)
    srv = balib.Server(budget, 3)
    tk = [srv.submit(balib.scene_desc(s), balib.options(max_iters=5)) for s in scenes]
    for x in tk:
        r = srv.wait(x)
        assert r["iters"] == 5
    st = srv.stats()
    _say("budget", budget, "one", one, "stats", st)
    assert st["peak_bytes"] <= budget
    assert st["done"] == 6 and st["queued"] == 0 and st["active"] == 0
    big = make_small_drive(80, 9000, seed=130)
    with pytest.raises(balib.BAError) as e:  # refused at submission or, once analysed, at wait
        srv.wait(srv.submit(balib.scene_desc(big), balib.options(max_iters=5)))
    assert e.value.code == balib.BA_ENOMEM
    # invalid content fails its own ticket and no other
    bad = make_small_drive(20, 1000, seed=131)
    bad.obs_cam = bad.obs_cam.copy()
    bad.obs_pt = bad.obs_pt.copy()
    bad.obs_cam[1], bad.obs_pt[1] = bad.obs_cam[0], bad.obs_pt[0]  # one (camera, point) observed twice
    good = make_small_drive(20, 1000, seed=132)
    tb = srv.submit(balib.scene_desc(bad), balib.options(max_iters=3))
    tg = srv.submit(balib.scene_desc(good), balib.options(max_iters=3))
    with pytest.raises(balib.BAError) as e:
        srv.wait(tb)
    assert e.value.code == balib.BA_EINVAL and "twice" in str(e.value)
    assert srv.wait(tg)["iters"] == 3
    srv.close()


def test_small_request_passes_one_waiting_for_memory(balib):
    """A budget for one large problem and one small one: large A runs, large B (submitted
    next) waits for memory, and small C, submitted after B, is admitted beside A instead
    of waiting behind B, so it finishes before A does; every result equals, bit for bit,
    the problem solved alone."""
    A = make_small_drive(60, 6000, seed=140)
    B = make_small_drive(60, 6000, seed=141)
    Cs = make_small_drive(15, 600, seed=142)
    iters = {"A": 300, "B": 5, "C": 3}
    sizes = {}
    for name, s in (("A", A), ("B", B), ("C", Cs)):
        p = balib.Problem.from_scene(s, max_iters=iters[name])
        sizes[name] = p.nbytes
        p.close()
    budget = sizes["A"] + sizes["C"] + (1 << 20)
    _say("bytes", sizes, "budget", budget)
    assert sizes["B"] > sizes["C"] + (1 << 20)  # A and B do not fit together
    srv = balib.Server(budget, 4)
    t0 = time.perf_counter()
    ta = srv.submit(balib.scene_desc(A), balib.options(max_iters=iters["A"]))
    tb = srv.submit(balib.scene_desc(B), balib.options(max_iters=iters["B"]))
    time.sleep(0.05)  # A is running and B analysed and waiting when C arrives
    t_c = time.perf_counter()
    tc = srv.submit(balib.scene_desc(Cs), balib.options(max_iters=iters["C"]))
    rc, ra, rb = srv.wait(tc), srv.wait(ta), srv.wait(tb)
    st = srv.stats()
    srv.close()
    done_a = ra["latency_ms"] / 1e3
    done_c = (t_c - t0) + rc["latency_ms"] / 1e3
    _say("A done at", done_a, "s, C done at", done_c, "s, B latency", rb["latency_ms"], "ms", st)
    assert done_c < done_a
    assert st["peak_bytes"] <= budget
    for name, s, r in (("A", A, ra), ("B", B, rb), ("C", Cs, rc)):
        a = _alone(balib, s, iters[name], "f32")
        assert np.array_equal(r["iter_cost"], a["iter_cost"]), name
        assert np.array_equal(r["X"], a["X"]) and np.array_equal(r["t"], a["t"]), name


def test_pose_requests_through_server_equal_batch(balib):
    reqs = make_config4_requests(40, seed=1004)
    ref = balib.pose_batch(reqs, iters=10, huber_delta=1.0)
    srv = balib.Server(64 << 20, 4)
    tk = [srv.submit_pose(q, iters=10, huber_delta=1.0) for q in reqs]
    for i, x in enumerate(tk):
        r = srv.wait(x)
        assert np.array_equal(r["q"][0], ref["q"][i]) and np.array_equal(r["t"][0], ref["t"][i])
        assert r["cost"] == ref["cost"][i]
    st = srv.stats()
    srv.close()
    _say("pose stats", st)
    assert st["done"] == len(reqs)


def test_pose_requests_with_different_options_keep_their_own(balib):
    """Pose requests admitted in one scheduler step but asking for different
    iteration counts and Huber thresholds: each result equals, bit for bit,
    ba_pose_batch run alone with that request's own options."""
    reqs = make_config4_requests(24, seed=1005)
    opts = [(10, 1.0), (4, 0.0), (7, 2.5)]
    refs = {o: balib.pose_batch(reqs, iters=o[0], huber_delta=o[1]) for o in opts}
    srv = balib.Server(64 << 20, 4)
    tk = [srv.submit_pose(q, iters=opts[i % 3][0], huber_delta=opts[i % 3][1]) for i, q in enumerate(reqs)]
    for i, x in enumerate(tk):
        r = srv.wait(x)
        ref = refs[opts[i % 3]]
        assert r["iters"] == opts[i % 3][0]
        assert np.array_equal(r["q"][0], ref["q"][i]) and np.array_equal(r["t"][0], ref["t"][i]), i
        assert r["cost"] == ref["cost"][i] and r["status"] == ref["status"][i]
    srv.close()
    # the options matter: the three references differ
    assert not np.array_equal(refs[opts[0]]["t"], refs[opts[1]]["t"])
    assert not np.array_equal(refs[opts[0]]["cost"], refs[opts[2]]["cost"])


def test_destroy_with_queued_requests(balib):
    """Destroying a server cancels what is queued and finishes what runs."""
    scenes = [make_small_drive(20, 1000, seed=140 + i) for i in range(5)]
    srv = balib.Server(256 << 20, 1)
    for s in scenes:
        srv.submit(balib.scene_desc(s), balib.options(max_iters=3))
    srv.close()
