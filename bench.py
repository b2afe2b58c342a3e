#!/usr/bin/env python3
"""Benchmark of the bundle-adjustment hot path on one MI355X.

A step is one full solve of the sequential-drive problem (500 cameras, 250k
points, ~1.97M observations, camera 0 fixed): 10 Levenberg-Marquardt
iterations, each linearising, forming the Schur complement, running block-
Jacobi PCG (50 products, rel. tol 1e-6), back-substituting and evaluating the
trial cost.  The problem is uploaded once; each step restores the initial state
on the device (ba_reset) and solves.  Prints one JSON line: the drive's LM
iterations/s as `value`, the dominant kernel and the whole LM loop against the
HBM roofline (algorithmic bytes of the method: 48 B per observation, 48 B per
point, and the reduced system's upper triangle, 144 B per FP32 6x6 block, once to
form it and once per PCG iteration), and the other legs: the tiny FP64 scene, the
11.2M-observation loop scene in FP32 / FP16-J / BF16-J, the refinement, vehicle-rig
and pose-graph legs, the serving streams and the oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--precision f32|f64|f16j|bf16j]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BA LM iterations/sec and observations/sec at 2M obs; p50/p99 latency for mixed-size stream"
HBM_PEAK_GBS = 8000.0
LM_ITERS = 10


def model_bytes_pcg_iteration(info: dict, precision: str) -> float:
    """Algorithmic bytes of one PCG iteration in the byte model of the method: the
    reduced system's upper triangle with its diagonal read once, one 6x6 block of the
    compute type per block (144 B in FP32); vectors are negligible beside it."""
    T = 8 if precision == "f64" else 4
    return (info["n_up_blocks"] + info["n_free_cams"]) * 36 * T


def model_bytes_lm_iteration(info: dict, precision: str, pcg_iters: float) -> float:
    """Algorithmic bytes of one LM iteration in the same model: the observations
    (16 B each) read three times (linearise + Schur, back-substitution, trial cost),
    the points (12 B) read three times and written once, and the reduced system read
    once to form it plus once per PCG iteration."""
    return (48 * info["n_obs"] + 48 * info["n_pts"]
            + (1 + pcg_iters) * model_bytes_pcg_iteration(info, precision))


def host_cpu() -> dict:
    """The host's logical core count and CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cores": os.cpu_count(), "cpu_model": model}


def design_bytes(kernel: str, info: dict, precision: str) -> float:
    """Bytes a kernel of this design moves per launch (each input it reads once,
    each output it writes once), from the problem's sizes: both triangles of S, the
    stored linearisation records and the chunk partials included."""
    T = 8 if precision == "f64" else 4
    S = {"f64": 8, "f32": 4, "f16j": 2, "bf16j": 2}[precision]
    N, P, Cf, C = info["n_obs"], info["n_pts"], info["n_free_cams"], info["n_cams"]
    Nf = info["n_free_obs"]
    rec = 7 * S + 2 * T            # compact record: sqrt(w) J_pi (4), P_c (3), sqrt(w) r (2)
    if kernel == "linearize":      # obs cam/pt/uv/slot + points in; records, V, g_p, D_p out
        return N * (12 + 2 * T) + P * 24 + Nf * rec + P * 12 * T + C * 96
    if kernel == "point_prep":     # V, D_p, records, obs cam/pt/slot in; V*^-1, Q out
        return P * 9 * T + Nf * rec + N * 12 + P * 6 * T + Nf * 6 * T
    if kernel == "schur_diag":     # per free observation: slot, point, record, Q, g_p; S diagonal, M^-1 out
        return Nf * (4 + 4 + rec + 6 * T + 3 * T) + Cf * (36 * T + 36 * 8 + 6 * 6 * T)
    if kernel == "schur_off":      # pair list + records and Q once; S blocks out
        return info["n_pairs"] * 8 + Nf * (rec + 6 * T) + info["n_up_blocks"] * 2 * 36 * T
    if kernel == "schur_chunk":    # records, point blocks, items once; partials out
        return (Nf * rec + N * 12 + P * (15 * T + 6 * T) + (Nf + info["n_pairs"]) * 4
                + info["n_entries"] * (16 + 36 * T))
    if kernel == "schur_reduce":   # partials in; S blocks out (both triangles), M^-1
        return info["n_entries"] * (4 + 36 * T) + info["nnzb"] * 36 * T + Cf * 36 * 8
    if kernel == "pcg_cg":         # S once; r, u, w, s, p, x in and out once, M^-1 once
        return info["nnzb"] * (36 * T + 4) + Cf * (6 * T * 12 + 36 * 8)
    if kernel == "pcg_spmv":       # S once + column vectors
        return info["nnzb"] * (36 * T + 4) + Cf * 6 * T * 4
    if kernel == "cull":           # activity, cameras, pixels, point ranges, points, poses read once,
        # tile counts written (the activity and point write-backs depend on the data: not counted)
        return N * (1 + 4 + 2 * T) + P * (4 + 24) + C * 96 + 8 * ((P + 255) // 256)
    if kernel == "point_trial":    # records, x, V*^-1, g_p, D_p, X in; X' out; obs re-read for cost
        return Nf * rec + N * (12 + 2 * T) + P * (12 * T + 48) + Cf * 6 * T
    return 0.0


REFINE_STAGES = [(4.0, 16.0), (0.0, 3.0)]  # (Huber delta px, outlier threshold px): robust, then strict
REFINE_ROUNDS = 2
REFINE_ITERS = 30  # LM iterations per round


def refine_leg(ba, precision: str, n_pts: int, flags: int = 0, reps: int = 3) -> dict:
    """The two-stage iterative refinement (each round: 30 LM iterations, then
    culling with midpoint re-triangulation) on the same drive with 5 % of the
    pixels replaced by uniform outliers.  Whole-call wall time over `reps` runs
    (each from the initial state, graphs replayed), then one more run with the
    culling kernel timed by HIP events."""
    import numpy as np
    from synth import make_config1
    print("bench: generating the outlier drive", flush=True, file=sys.stderr)
    s = make_config1(n_pts=n_pts, outlier_frac=0.05, huber_delta=1.0)
    p = ba.Problem.from_scene(s, max_iters=REFINE_ITERS, pcg_max_iters=50, pcg_rel_tol=1e-6,
                              precision=precision, flags=flags)
    info = p.info()
    p.refine(REFINE_STAGES, REFINE_ROUNDS)  # warm-up (graph capture)
    walls = []
    for _ in range(reps):
        p.reset()
        t0 = time.perf_counter()
        hist = p.refine(REFINE_STAGES, REFINE_ROUNDS)
        walls.append(time.perf_counter() - t0)
        print(f"bench: refine {1000 * walls[-1]:.2f} ms", flush=True, file=sys.stderr)
    act = p.active().astype(bool)
    rep = p.report()
    names = list(p.kernel_times().keys())
    p.reset()
    p.set_profiling(1 << names.index("cull"))
    p.refine(REFINE_STAGES, REFINE_ROUNDS)
    cull_ms, n_cull = p.kernel_times()["cull"]
    p.set_profiling(0)
    p.close()
    wall = float(np.median(walls))
    n_rounds = len(REFINE_STAGES) * REFINE_ROUNDS
    cull_s = cull_ms / 1000.0 / max(n_cull, 1)
    abytes = design_bytes("cull", info, precision)
    return {"workload": f"sequential drive BA with 5 % uniform outliers: {info['n_cams']} cameras, "
                        f"{info['n_pts']} points, {info['n_obs']} observations",
            "stages": [{"huber_delta_px": d, "cull_px": t} for d, t in REFINE_STAGES],
            "rounds_per_stage": REFINE_ROUNDS, "lm_iters_per_round": REFINE_ITERS,
            "ms": round(1000 * wall, 3), "lm_iters_per_s": round(n_rounds * REFINE_ITERS / wall, 2),
            "rounds": [[h["stage"], h["round"], h["iters"], h["cost"], h["n_active_obs"], h["n_active_pts"]]
                       for h in hist],
            "outliers_removed": round(float((~act & s.outlier).sum() / s.outlier.sum()), 5),
            "inliers_removed": round(float((~act & ~s.outlier).sum() / (~s.outlier).sum()), 5),
            "final_rms_px": rep["rms_px"],
            "cull": {"avg_launch_us": round(cull_s * 1e6, 2), "launches": n_cull,
                     "algorithmic_bytes": abytes,
                     "achieved_gbs": round(abytes / cull_s / 1e9, 1),
                     "frac_of_hbm_peak": round(abytes / cull_s / 1e9 / HBM_PEAK_GBS, 4),
                     "share_of_refine": round(cull_ms / 1000.0 / wall, 5)}}


def pose_graph_leg(ba, precision: str, n_frames: int, flags: int = 0, steps: int = 10) -> dict:
    """Pose-graph optimisation of a 3-camera rig driving a circular loop twice
    (camera-frame nodes; sequential k = 1, 2, loop-closure and extrinsic edges): 10 LM
    iterations with PCG 50 / 1e-6 per solve, inputs resident in HBM (ba_reset +
    ba_solve), `steps` timed solves; then one solve with the PCG step timed by HIP events."""
    import numpy as np
    from synth import make_pose_graph
    print("bench: generating the pose graph", flush=True, file=sys.stderr)
    g = make_pose_graph(n_frames)
    p = ba.Problem.from_pose_graph(g, max_iters=LM_ITERS, pcg_max_iters=50, pcg_rel_tol=1e-6,
                                   precision=precision, flags=flags)
    info = p.info()
    p.reset().solve()  # warm-up (graph capture)
    walls, dev = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        p.reset().solve()
        walls.append(time.perf_counter() - t0)
        dev.append(p.report()["solve_ms"])
    rep = p.report()
    names = list(p.kernel_times().keys())
    p.set_profiling(1 << names.index("pcg_cg"))
    p.reset().solve()
    cg_ms, cg_n = p.kernel_times()["pcg_cg"]
    p.set_profiling(0)
    p.close()
    wall = float(np.median(walls))
    cg_s = cg_ms / 1000.0 / max(cg_n, 1)
    abytes = model_bytes_pcg_iteration(info, precision)
    return {"workload": f"pose graph: {g.meta['n_frames'] * g.meta['laps']} frames x 3 cameras = "
                        f"{info['n_cams']} nodes (1 fixed), {g.n_edges} edges "
                        f"(sequential k = 1, 2; loop closures; extrinsic)",
            "lm_iters": LM_ITERS, "ms_per_solve": round(1000 * wall, 3),
            "device_ms_per_solve": round(float(np.median(dev)), 3),
            "lm_iters_per_s": round(LM_ITERS / wall, 2), "edges_per_s": round(g.n_edges * LM_ITERS / wall, 1),
            "nnzb": info["nnzb"], "cost0": rep["cost0"], "cost": rep["cost"],
            "pcg_iters": [int(x) for x in rep["pcg_iters"]],
            "pcg_cg": {"avg_launch_us": round(cg_s * 1e6, 2), "algorithmic_bytes": abytes,
                       "achieved_gbs": round(abytes / cg_s / 1e9, 1),
                       "frac_of_hbm_peak": round(abytes / cg_s / 1e9 / HBM_PEAK_GBS, 4)}}


def rig_leg(ba, precision: str, flags: int = 0, steps: int = 10) -> dict:
    """Extrinsic refinement in the vehicle-rig configuration: 200 frames of a 3-camera
    rig (~20k points, ~192k observations), vehicle poses and shared extrinsics unknown,
    extrinsic prior and rigidity pairs (weights 100), 10 LM iterations with PCG
    50 / 1e-6 per solve, `steps` timed solves from the initial state; then one solve
    with every kernel timed by HIP events (per LM iteration, microseconds)."""
    import numpy as np
    from scipy.spatial.transform import Rotation
    from synth import make_rig_drive
    print("bench: generating the rig drive", flush=True, file=sys.stderr)
    s = make_rig_drive(200, 20000, seed=1006)
    pairs = np.array([[0, 1], [0, 2]])
    p = ba.Problem.from_rig(s, prior_ext=100.0, prior_rig=100.0, rig_pairs=pairs, max_iters=LM_ITERS,
                            pcg_max_iters=50, pcg_rel_tol=1e-6, precision=precision, flags=flags)
    info = p.info()
    p.reset().solve()  # warm-up (graph capture)
    walls, dev = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        p.reset().solve()
        walls.append(time.perf_counter() - t0)
        dev.append(p.report()["solve_ms"])
    res = p.rig_result()
    p.set_profiling(-1)
    p.reset().solve()
    per_iter_us = {k: round(v[0] / LM_ITERS * 1000, 2) for k, v in p.kernel_times().items() if v[1]}
    p.set_profiling(0)
    p.close()

    def rel_rot_err(q):  # largest ||R_c R_0^T - R_c,true R_0,true^T||_F over the side cameras
        R = Rotation.from_quat(np.asarray(q)[:, [1, 2, 3, 0]]).as_matrix()
        G = Rotation.from_quat(np.asarray(s.qe_gt)[:, [1, 2, 3, 0]]).as_matrix()
        return float(max(np.linalg.norm(R[k] @ R[0].T - G[k] @ G[0].T) for k in range(1, len(R))))

    wall = float(np.median(walls))
    return {"workload": f"vehicle-rig BA: {s.n_frames} frames x {s.n_rig} cameras, {info['n_pts']} points, "
                        f"{info['n_obs']} observations; vehicle poses and shared extrinsics, extrinsic prior "
                        f"and rigidity pairs",
            "lm_iters": LM_ITERS, "ms_per_solve": round(1000 * wall, 3),
            "device_ms_per_solve": round(float(np.median(dev)), 3),
            "lm_iters_per_s": round(LM_ITERS / wall, 2), "obs_per_s": round(info["n_obs"] * LM_ITERS / wall, 1),
            "cost0": res["cost0"], "cost": res["cost"],
            "rel_extrinsic_rot_err": [round(rel_rot_err(s.qe0), 6), round(rel_rot_err(res["qe"]), 6)],
            "kernel_us_per_iter": per_iter_us}


def config0_leg(ba, steps: int = 5) -> dict:
    """The tiny arc scene (10 cameras, 1000 points, ~9k observations) in FP64: 20 LM
    iterations with PCG run to 1e-14, device time per LM iteration (median of `steps`
    solves from the initial state), and every C_n against the dense FP64 oracle's run
    stored in tests/golden/config0_oracle.json."""
    import numpy as np
    from synth import make_config0
    s = make_config0()
    p = ba.Problem.from_scene(s, max_iters=20, pcg_max_iters=200, pcg_rel_tol=1e-14, precision="f64",
                              flags=ba.FLAG_PCG_RESIDENT)
    info = p.info()
    p.reset().solve()  # warm-up (graph capture)
    walls, dev = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        p.reset().solve()
        walls.append(time.perf_counter() - t0)
        dev.append(p.report()["solve_ms"])
    r = p.report()
    p.close()
    out = {"workload": f"tiny arc BA: {info['n_cams']} cameras (1 fixed), {info['n_pts']} points, "
                       f"{info['n_obs']} observations, FP64, 20 LM iterations, PCG 200 / 1e-14",
           "device_us_per_lm_iteration": round(float(np.median(dev)) * 1000 / 20, 2),
           "wall_us_per_lm_iteration": round(float(np.median(walls)) * 1e6 / 20, 2),
           "final_rms_px": r["rms_px"]}
    gold = os.path.join(ROOT, "tests", "golden", "config0_oracle.json")
    with open(gold) as f:
        g = json.load(f)
    rel = [abs(a - b) / b for a, b in zip(r["iter_cost"], g["iter_cost"])]
    out["vs_oracle"] = {"max_rel_cost_err": max(rel), "final_rms_err_px": abs(r["rms_px"] - g["final_rms_px"]),
                        "oracle": "dense normal equations, FP64"}
    return out


def loop_leg(ba, precisions, steps: int = 2) -> dict:
    """The loop-closed drive (3000 cameras on two overlapping laps, 1.5M points, ~11.2M
    observations, 5 % outliers, Huber 1 px): 15 LM iterations with PCG 50 / 1e-6 per
    solve in each precision mode, inputs resident in HBM; LM iterations/s over `steps`
    solves, the whole loop against the byte model, and the final cost and RMS against
    the FP64 oracle's run of the same schedule (tests/golden/config2_oracle.json)."""
    import numpy as np
    from synth import make_config2
    print("bench: generating the loop scene", flush=True, file=sys.stderr)
    s = make_config2()
    gold = os.path.join(ROOT, "tests", "golden", "config2_oracle.json")
    with open(gold) as f:
        g = json.load(f)
    out = {}
    for prec in precisions:
        print(f"bench: loop scene, {prec}", flush=True, file=sys.stderr)
        p = ba.Problem.from_scene(s, max_iters=15, pcg_max_iters=50, pcg_rel_tol=1e-6, precision=prec)
        info = p.info()
        p.reset().solve()  # warm-up (graph capture)
        walls, dev = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            p.reset().solve()
            walls.append(time.perf_counter() - t0)
            dev.append(p.report()["solve_ms"])
        r = p.report()
        p.close()
        wall = float(np.median(walls))
        dev_lm_s = float(np.median(dev)) / 1000.0 / 15
        pcg_per_lm = float(np.mean(r["pcg_iters"]))
        lm_bytes = model_bytes_lm_iteration(info, prec, pcg_per_lm)
        rel = [abs(a - b) / b for a, b in zip(r["iter_cost"], g["iter_cost"])]
        out[prec] = {"lm_iters_per_s": round(15 / wall, 2), "obs_per_s": round(info["n_obs"] * 15 / wall, 1),
                     "device_us_per_lm_iteration": round(dev_lm_s * 1e6, 2),
                     "loop_roofline": {"bound": "hbm", "bytes_per_lm_iteration": round(lm_bytes),
                                       "achieved": round(lm_bytes / dev_lm_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(lm_bytes / dev_lm_s / 1e9 / HBM_PEAK_GBS, 4)},
                     "final_cost": r["cost"], "final_rms_px": r["rms_px"],
                     "vs_oracle": {"final_rms_px": g["final_rms_px"],
                                   "final_rms_err_px": abs(r["rms_px"] - g["final_rms_px"]),
                                   "max_rel_cost_err": max(rel),
                                   "same_pcg_iters": [int(x) for x in r["pcg_iters"]] == g["pcg_iters"]}}
    out["workload"] = (f"loop-closed Huber drive BA: {info['n_cams']} cameras (1 fixed), {info['n_pts']} points, "
                       f"{info['n_obs']} observations, 5 % outliers, Huber 1 px, 15 LM iterations, PCG 50 / 1e-6")
    return out


def cpu_baseline(budget_s: float = 30.0) -> dict:
    """The FP64 oracle (explicit Schur complement + block-Jacobi PCG, the same
    schedule) timed on one host core for one LM iteration of the same scene."""
    code = r"""
import json, time, sys
sys.path.insert(0, %r)
from synth import make_config1
from oracle import ba_oracle as O
s = make_config1()
p = O.Problem.from_scene(s)
t = time.perf_counter()
r = O.lm_schur(p, O.LMOptions(max_iters=1, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6))
dt = time.perf_counter() - t
print(json.dumps({"seconds": dt, "n_obs": p.n_obs, "iters": 1}))
""" % ROOT
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                             timeout=max(120.0, 6 * budget_s))
        d = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # the baseline is reported, never required
        return {"value": None, "unit": "LM iterations/s", "cores": 1, "kind": "oracle", **host_cpu(),
                "sample": f"failed: {e}"}
    sec = d["seconds"]
    return {"value": 1.0 / sec, "unit": "LM iterations/s", "cores": 1, "kind": "oracle", **host_cpu(),
            "obs_per_s": d["n_obs"] / sec,
            "sample": f"1 LM iteration (linearise, explicit Schur, PCG 50/1e-6, back-substitution, "
                      f"trial cost) of the same {d['n_obs']}-observation scene, FP64 NumPy/SciPy, "
                      f"{sec:.1f} s on 1 thread"}


def cpu_serving_baseline(sizes, budget_s: float = 30.0) -> dict:
    """The oracle on the serving streams, on the host: the pose-only GN oracle over a
    pool of one single-threaded process per host core (the first 512 requests of the
    4096-request stream, timed whole); and the explicit-Schur LM oracle (PCG 50 / 1e-6)
    timed for one LM iteration on a sample of BA-stream requests at fixed size ranks,
    fitted as seconds per observation pair (pairs ~ N (N / P - 1) / 2), extrapolated to
    20 iterations of every request, and replayed as the saturated stream (all arrivals at
    t = 0, first come first served) on as many single-threaded workers as host cores.
    `sizes`: (n_obs, n_pts) of every BA-stream request in stream order."""
    import numpy as np
    code = r"""
import json, os, sys, time
import multiprocessing as mp
sys.path.insert(0, %r)
import numpy as np
from synth import make_config3_problem, make_config3_sizes, make_config4_requests
from oracle import ba_oracle as O

def pose(q):
    return O.pose_only_gn(q.K, q.q0, q.t0, q.X, q.uv, 1.0, 10)[2]

if __name__ == "__main__":
    n = os.cpu_count()
    reqs = make_config4_requests(4096)[:512]
    with mp.Pool(n) as pool:
        pool.map(pose, reqs[:n])
        t = time.perf_counter()
        pool.map(pose, reqs, chunksize=8)
        dt = time.perf_counter() - t
    out = {"pose_requests": len(reqs), "pose_seconds": dt, "cores": n}
    nc, npt = make_config3_sizes()
    sample = json.loads(sys.argv[1])
    times = []
    for r in sample:
        s = make_config3_problem(r, int(nc[r]), int(npt[r]))
        p = O.Problem.from_scene(s)
        t = time.perf_counter()
        O.lm_schur(p, O.LMOptions(max_iters=1, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6))
        times.append([r, p.n_obs, p.n_pts, time.perf_counter() - t])
    out["ba_sample"] = times
    print(json.dumps(out))
""" % ROOT
    nobs = np.array([x[0] for x in sizes], float)
    npts = np.array([x[1] for x in sizes], float)
    pairs = nobs * np.maximum(nobs / npts - 1.0, 0.0) / 2.0
    order = np.argsort(pairs)
    # seven requests at the 2nd-40th size percentiles keep the sample to tens of seconds
    sample = [int(order[int(q * (len(order) - 1))]) for q in (0.02, 0.06, 0.10, 0.15, 0.20, 0.30, 0.40)]
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    try:
        out = subprocess.run([sys.executable, "-c", code, json.dumps(sample)], env=env, capture_output=True,
                             text=True, timeout=max(300.0, 10 * budget_s))
        d = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # the baseline is reported, never required
        return {"kind": "oracle", "sample": f"failed: {e}", **host_cpu()}
    n = d["cores"]
    res = {"kind": "oracle", "cores": n, **host_cpu(),
           "pose_stream": {"requests_per_s": round(d["pose_requests"] / d["pose_seconds"], 1),
                           "sample": f"the first {d['pose_requests']} requests of the 4096-request stream, "
                                     f"10 GN iterations, one single-threaded process per core"}}
    samp = np.array([[x[1], x[2], x[3]] for x in d["ba_sample"]], float)
    sp = samp[:, 0] * np.maximum(samp[:, 0] / samp[:, 1] - 1.0, 0.0) / 2.0
    c = float((sp * samp[:, 2]).sum() / (sp * sp).sum())  # seconds per pair per LM iteration
    est = 20.0 * c * pairs  # seconds per request, 20 LM iterations
    free_at = np.zeros(n)
    lat = []
    for e in est:  # saturated stream, first come first served on n workers
        w = int(np.argmin(free_at))
        free_at[w] += e
        lat.append(free_at[w])
    lat = np.sort(np.array(lat))
    res["ba_stream"] = {"solves_per_s": round(len(est) / float(free_at.max()), 4),
                        "p50_ms": round(1000 * float(np.percentile(lat, 50)), 1),
                        "p99_ms": round(1000 * float(np.percentile(lat, 99)), 1),
                        "seconds_per_pair_iteration": c,
                        "sample": f"one LM iteration of requests {sample} (the 2nd to 40th percentiles of "
                                  f"pair count), {', '.join(f'{x[3]:.2f} s' for x in d['ba_sample'])}; "
                                  f"extrapolated: seconds per observation pair fitted, 20 iterations "
                                  f"of every request, saturated stream replayed on {n} workers"}
    return res


def serving_leg(ba, n_ba: int, precision: str, precisions=("f16j", "bf16j"), slots: int = 16,
                poisson=(0.5, 0.8), cpu: bool = True) -> dict:
    """p50/p99 latency (submission to result on the host) and throughput of the
    continuous-batching server under an 8 GB budget: the 4096-request pose-only
    localization stream submitted at once, and the first n_ba problems of the
    512-problem BA stream (cameras and points log-uniform, 20 LM iterations, PCG
    50 / 1e-6), first saturated (all submitted at t = 0), then with seeded Poisson
    arrivals at 0.5 and 0.8 of the saturated rate; then saturated again in each of
    `precisions`, with every problem's final RMS set against the same problem's in
    `precision` (the FP32 form with FP64 reductions by default)."""
    import numpy as np
    from synth import make_config3_problem, make_config3_sizes, make_config4_requests
    out = {}
    reqs = make_config4_requests(4096)
    srv = ba.Server(8 << 30, 64, precision)
    t0 = time.perf_counter()
    tk = [srv.submit_pose(r, iters=10, huber_delta=1.0) for r in reqs]
    for t in tk:
        srv.wait(t)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out["pose_stream"] = {"requests": len(reqs), "correspondences": int(sum(len(r.X) for r in reqs)),
                          "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                          "requests_per_s": round(len(reqs) / wall, 1), "gn_iters": 10}
    if n_ba <= 0:
        return out
    nc, npt = make_config3_sizes()
    print(f"bench: generating {n_ba} BA stream problems", flush=True, file=sys.stderr)
    descs = [ba.scene_desc(make_config3_problem(r, int(nc[r]), int(npt[r]))) for r in range(n_ba)]
    nobs = [int(d.desc.n_obs) for d in descs]

    def run(gaps, prec):
        opts = ba.options(max_iters=20, pcg_max_iters=50, pcg_rel_tol=1e-6, precision=prec)
        srv = ba.Server(8 << 30, slots, prec)
        t0 = time.perf_counter()
        tks = []
        for d, g in zip(descs, gaps):
            if g > 0:
                time.sleep(g)
            tks.append(srv.submit(d, opts))
        res, refused = [], 0
        for t in tks:
            try:
                res.append(srv.wait(t))
            except ba.BAError:
                res.append(None)
                refused += 1
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        print(f"bench: BA stream {prec}: {wall:.2f} s, p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms",
              flush=True, file=sys.stderr)
        return wall, st, res, refused

    def summary(wall, st, refused):
        return {"p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
                "solves_per_s": round(n_ba / wall, 2), "wall_s": round(wall, 3), "refused": refused,
                "peak_bytes": st["peak_bytes"]}

    wall, st, base, refused = run([0.0] * n_ba, precision)
    rate = n_ba / wall
    out["ba_stream"] = {"problems": n_ba, "obs_total": sum(nobs), "obs_max": max(nobs), "lm_iters": 20,
                        "budget_bytes": 8 << 30, "slots": slots, "precision": precision,
                        "schur_forms": "dense co-visibility (chosen per problem)"}
    out["ba_stream_saturated"] = summary(wall, st, refused)
    rms = np.array([r["rms_px"] if r else np.nan for r in base])
    sizes = [(int(d.desc.n_obs), int(d.desc.n_pts)) for d in descs]
    out["ba_stream_saturated"]["final_rms_px_median"] = round(float(np.nanmedian(rms)), 6)
    for frac in poisson:
        rng = np.random.default_rng(3000 + int(round(10 * frac)))
        gaps = rng.exponential(1.0 / (frac * rate), n_ba)
        gaps[0] = 0.0
        wall, st, _, refused = run(list(gaps), precision)
        out[f"ba_stream_poisson_{frac}"] = {**summary(wall, st, refused), "offered_per_s": round(frac * rate, 2)}
    for prec in precisions:
        wall, st, res, refused = run([0.0] * n_ba, prec)
        d = np.array([abs(r["rms_px"] - rms[i]) if r else np.nan for i, r in enumerate(res)])
        out[f"ba_stream_saturated_{prec}"] = {**summary(wall, st, refused),
                                              "final_rms_diff_vs_" + precision + "_px_max": float(np.nanmax(d)),
                                              "final_rms_diff_vs_" + precision + "_px_median": float(np.nanmedian(d))}
    if cpu:
        print("bench: timing the oracle on the serving streams", flush=True, file=sys.stderr)
        out["cpu_baseline"] = cpu_serving_baseline(sizes)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16j", "bf16j"])
    ap.add_argument("--points", type=int, default=None)
    ap.add_argument("--workload", default="drive", choices=["drive", "loop"],
                    help="drive: 500-camera sequential drive, ~2M observations, 10 LM iterations "
                         "(the metric's workload); loop: 3000-camera loop-closed drive, ~11M "
                         "observations, Huber, 15 LM iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="enqueue kernels instead of replaying a graph")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time only whole steps (lets solves replay their graph)")
    ap.add_argument("--graph-only", action="store_true",
                    help="no warm-up solve enqueued kernel by kernel: every solve replays graphs "
                         "(for a kernel trace of the mode the product runs)")
    ap.add_argument("--serving", type=int, default=512, metavar="N",
                    help="BA problems of the mixed-size stream in the serving leg (0: pose stream only, -1: skip)")
    ap.add_argument("--serving-precisions", default="f16j,bf16j",
                    help="storage modes whose saturated BA stream is set against the FP32 one")
    ap.add_argument("--serving-poisson", default="0.5,0.8",
                    help="Poisson arrival rates of the BA stream, as fractions of the saturated rate")
    ap.add_argument("--serving-slots", type=int, default=16, help="problems the server batches at once")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (3 times), to calibrate HBM counters")
    ap.add_argument("--prior-abs", type=float, default=0.0,
                    help="weight of the absolute pose prior (0: off)")
    ap.add_argument("--prior-seq", type=float, default=0.0,
                    help="weight of the sequential pose prior between frames i and i+k (0: off)")
    ap.add_argument("--prior-seq-k", type=int, default=1)
    ap.add_argument("--no-rig", action="store_true",
                    help="skip the vehicle-rig leg (200 frames x 3 cameras)")
    ap.add_argument("--no-pose-graph", action="store_true",
                    help="skip the pose-graph leg (9000 nodes, 24.7k edges)")
    ap.add_argument("--no-refine", action="store_true",
                    help="skip the iterative-refinement leg (outlier drive, two stages)")
    ap.add_argument("--no-config0", action="store_true",
                    help="skip the tiny FP64 leg (10 cameras, 1000 points, 20 LM iterations)")
    ap.add_argument("--loop-precisions", default="f32,f16j,bf16j",
                    help="precision modes of the loop-scene leg (11.2M observations), comma-separated; "
                         "empty to skip it")
    ap.add_argument("--per-launch-pcg", action="store_true",
                    help="one launch per PCG iteration instead of one resident launch per linear "
                         "solve (BA_FLAG_PCG_RESIDENT, the default for this lone solve)")
    ap.add_argument("--profile-all", action="store_true",
                    help="print per-kernel device times of one extra solve to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the problem is not sharded)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    from paper_2510_15271_amd import ba, build_lib
    if not os.path.exists(ba.LIB_PATH):
        build_lib.build()
    from synth import make_config1, make_config2

    print("bench: generating scene", flush=True, file=sys.stderr)
    global LM_ITERS
    if args.workload == "drive":
        scene = make_config1(n_pts=args.points or 250_000)
    else:
        scene = make_config2(n_pts=args.points or 1_500_000)
        LM_ITERS = 15
    prob = ba.Problem.from_scene(scene, max_iters=LM_ITERS, pcg_max_iters=50, pcg_rel_tol=1e-6,
                                 precision=args.precision,
                                 flags=(ba.FLAG_NO_GRAPH if args.no_graph else 0) |
                                       (0 if args.per_launch_pcg else ba.FLAG_PCG_RESIDENT),
                                 prior_abs=args.prior_abs, prior_seq=args.prior_seq,
                                 prior_seq_k=args.prior_seq_k)
    info = prob.info()
    names = list(prob.kernel_times().keys())

    # warm-up; the first one also times every kernel to find the dominant one (with
    # --graph-only no launch is enqueued outside a graph: the PCG is taken as dominant)
    if args.graph_only:
        for w in range(max(1, args.warmup)):
            prob.reset().solve()
        kt = {k: (0.0, 0) for k in names}
        dominant = "pcg_cg"
    else:
        prob.set_profiling(-1)
        for w in range(max(1, args.warmup)):
            prob.reset().solve()
            if w == 0:
                kt = prob.kernel_times()
                prob.set_profiling(0)
        dominant = max(kt, key=lambda k: kt[k][0])
    if args.profile_all:
        tot = sum(v[0] for v in kt.values())
        for k, (ms, n) in sorted(kt.items(), key=lambda x: -x[1][0]):
            print(f"  {k:12s} {ms:9.3f} ms  {n:5d} launches  {100 * ms / tot:5.1f} %",
                  file=sys.stderr)

    # timed region: the dominant kernel is timed with HIP events on its stream.  The
    # PCG step is bracketed once per run of launches (50 per LM iteration); other
    # kernels launched more than 100 times per solve are sampled every 10th launch.
    stride = 1 if dominant == "pcg_cg" else (10 if kt[dominant][1] >= 100 else 1)
    prob.set_profiling(0 if args.no_kernel_timing else 1 << names.index(dominant), stride)
    dev_ms = []
    dom_ms, dom_launch, pcg_iters = 0.0, 0, 0
    print(f"bench: timing {args.steps} steps", flush=True, file=sys.stderr)
    t0 = time.perf_counter()
    steps_log = []  # printed after the timed region
    for _ in range(args.steps):
        prob.reset().solve()
        r = prob.report()
        dev_ms.append(r["solve_ms"])
        ms, nl = prob.kernel_times()[dominant]
        steps_log.append((r["iters"], r["solve_ms"], ms, nl))
        dom_ms += ms
        dom_launch += nl
        pcg_iters += int(sum(r["pcg_iters"]))
    wall = time.perf_counter() - t0
    for it, sm, ms, nl in steps_log:
        print(f"bench: step {it} iters, {sm:.3f} ms device, {dominant} {ms:.3f} ms over {nl} launches",
              file=sys.stderr)
    sys.stderr.flush()
    prob.set_profiling(0)

    ms_per_step = 1000.0 * wall / args.steps
    lm_per_s = LM_ITERS * args.steps / wall
    avg_launch_s = dom_ms / 1000.0 / max(dom_launch, 1)
    resident = dominant == "pcg_cg" and bool(info["pcg_resident"])
    pcg_per_lm = pcg_iters / (args.steps * LM_ITERS)
    # algorithmic bytes per launch of the dominant kernel: for the PCG, the reduced
    # system's upper triangle once per PCG iteration (a resident launch runs a whole
    # linear solve, so it is charged the iterations it ran); another dominant kernel is
    # charged its design bytes (each input and output once)
    if dominant in ("pcg_cg", "pcg_spmv"):
        per_unit = model_bytes_pcg_iteration(info, args.precision)
        units = pcg_iters / max(dom_launch, 1) if resident else 1.0
        bytes_model = "method: S upper triangle with diagonal, 36 values per 6x6 block, once per PCG iteration"
        dbytes = design_bytes(dominant, info, args.precision) * units
    else:
        per_unit, units = design_bytes(dominant, info, args.precision), 1.0
        bytes_model = "design: each input and output of the kernel once"
        dbytes = per_unit
    abytes = per_unit * units
    achieved = abytes / avg_launch_s / 1e9 if abytes and avg_launch_s > 0 else None
    traffic = None
    tname = f"{dominant}_resident" if resident else dominant
    tfile = os.path.join(ROOT, "profiles", f"traffic_{tname}_{args.workload}_{args.precision}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            traffic = json.load(f).get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dominant,
                "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "algorithmic_bytes": round(abytes), "bytes_per_unit": round(per_unit),
                "units_per_launch": round(units, 3), "bytes_model": bytes_model,
                "design_bytes": round(dbytes),
                "design_frac": round(dbytes / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4) if avg_launch_s > 0 else None}
    if resident and units > 0:
        roofline["avg_pcg_iteration_us"] = round(avg_launch_s * 1e6 / units, 3)
    # the whole LM loop against the same model (device time of the iteration loop)
    lm_bytes = model_bytes_lm_iteration(info, args.precision, pcg_per_lm)
    dev_lm_s = sum(dev_ms) / len(dev_ms) / 1000.0 / LM_ITERS
    loop_roofline = {"bound": "hbm", "bytes_per_lm_iteration": round(lm_bytes),
                     "pcg_iterations_per_lm_iteration": round(pcg_per_lm, 2),
                     "device_us_per_lm_iteration": round(dev_lm_s * 1e6, 2),
                     "achieved": round(lm_bytes / dev_lm_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(lm_bytes / dev_lm_s / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC,
        "value": round(lm_per_s, 2),
        "unit": "LM iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f16j": "f32+f16 storage",
                  "bf16j": "f32+bf16 storage"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{'sequential' if args.workload == 'drive' else 'loop-closed Huber'} "
                               f"drive BA: {info['n_cams']} cameras (1 fixed), "
                               f"{info['n_pts']} points, {info['n_obs']} observations, "
                               f"{LM_ITERS} LM iterations, PCG 50 / 1e-6",
                   "n_obs": info["n_obs"], "n_pairs": info["n_pairs"],
                   "nnzb": info["nnzb"], "precision": args.precision,
                   "schur_form": "point chunks" if info["schur_form"] else "pair lists",
                   "pose_priors": ({"abs": args.prior_abs, "seq": args.prior_seq, "seq_k": args.prior_seq_k}
                                   if args.prior_abs > 0 or args.prior_seq > 0 else None),
                   "graph": not args.no_graph,
                   "pcg": "resident (one launch per linear solve)" if info["pcg_resident"]
                          else "one launch per iteration"},
        "obs_per_s": round(info["n_obs"] * lm_per_s, 1),
        "device_ms_per_step": round(sum(dev_ms) / len(dev_ms), 3),
        "final_rms_px": r["rms_px"],
        "final_cost": r["cost"],
        "roofline": roofline,
        "loop_roofline": loop_roofline,
    }
    gold = os.path.join(ROOT, "tests", "golden", f"config{1 if args.workload == 'drive' else 2}_oracle.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        if g["n_obs"] == info["n_obs"] and len(g["iter_cost"]) == LM_ITERS + 1:
            # the FP64 oracle's run of the same scene and schedule, stored by tests/golden
            out["vs_oracle"] = {"final_rms_px": g["final_rms_px"],
                                "final_rms_err_px": abs(r["rms_px"] - g["final_rms_px"]),
                                "max_rel_cost_err": max(abs(a - b) / b for a, b in zip(r["iter_cost"],
                                                                                         g["iter_cost"])),
                                "same_pcg_iters": [int(x) for x in r["pcg_iters"]] == g["pcg_iters"]}
    prob.close()
    if not args.no_config0 and args.workload == "drive":
        print("bench: tiny FP64 scene", flush=True, file=sys.stderr)
        out["config0"] = config0_leg(ba)
    if args.loop_precisions and args.workload == "drive":
        out["loop"] = loop_leg(ba, [x for x in args.loop_precisions.split(",") if x])
    if not args.no_refine and args.workload == "drive":
        out["refine"] = refine_leg(ba, args.precision, args.points or 250_000,
                                   (ba.FLAG_NO_GRAPH if args.no_graph else 0) |
                                   (0 if args.per_launch_pcg else ba.FLAG_PCG_RESIDENT))
    if not args.no_rig and args.workload == "drive":
        out["rig"] = rig_leg(ba, args.precision, ba.FLAG_NO_GRAPH if args.no_graph else 0)
    if not args.no_pose_graph and args.workload == "drive":
        out["pose_graph"] = pose_graph_leg(ba, args.precision, 1500, ba.FLAG_NO_GRAPH if args.no_graph else 0)
    if args.serving >= 0:
        print("bench: serving streams", flush=True, file=sys.stderr)
        out["serving"] = serving_leg(ba, args.serving, args.precision,
                                     [x for x in args.serving_precisions.split(",") if x], args.serving_slots,
                                     [float(x) for x in args.serving_poisson.split(",") if x],
                                     not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", flush=True, file=sys.stderr)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
