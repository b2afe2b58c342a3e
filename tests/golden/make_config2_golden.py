"""Writes tests/golden/config2_oracle.json: the FP64 oracle's run of the
11M-observation loop-closed drive (Huber delta 1 px, 5 % outliers) with the benchmark's schedule (15 LM
iterations, explicit Schur complement, block-Jacobi PCG capped at 50 products,
rel. tol 1e-6).  Calls only synth/ and oracle/.  Takes about an hour on one core and ~25 GB of memory.

    python tests/golden/make_config2_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ba_oracle as O  # noqa: E402
from synth import make_config2  # noqa: E402


def main():
    s = make_config2()
    p = O.Problem.from_scene(s)
    t = time.time()
    r = O.lm_schur(p, O.LMOptions(max_iters=15, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6))
    out = dict(scene="make_config2() (1.5M points, seed 1002)", n_obs=int(p.n_obs),
               schedule="15 LM iterations, PCG 50 / 1e-6, lambda0 1e-4, Huber delta 1 px",
               iter_cost=[float(c) for c in r.iter_cost], accepted=[bool(a) for a in r.accepted],
               pcg_iters=[int(i) for i in r.pcg_iters],
               final_rms_px=O.rms(p, r.R, r.t, r.X),
               final_inlier_rms_px=O.rms(p, r.R, r.t, r.X, inlier_px=3.0),
               n_masked=O.cost_and_masked(p, r.R, r.t, r.X)[1],
               seconds=time.time() - t)
    with open(os.path.join(HERE, "config2_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
