"""Writes tests/golden/config1_oracle.json: the FP64 oracle's run of the
2M-observation sequential drive with the benchmark's schedule (10 LM
iterations, explicit Schur complement, block-Jacobi PCG capped at 50 products,
rel. tol 1e-6).  Calls only synth/ and oracle/.  Takes a few minutes on one core.

    python tests/golden/make_config1_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ba_oracle as O  # noqa: E402
from synth import make_config1  # noqa: E402


def main():
    s = make_config1()
    p = O.Problem.from_scene(s)
    t = time.time()
    r = O.lm_schur(p, O.LMOptions(max_iters=10, solve="pcg", pcg_max_iters=50, pcg_rel_tol=1e-6))
    out = dict(scene="make_config1() (250k points, seed 1001)", n_obs=int(p.n_obs),
               schedule="10 LM iterations, PCG 50 / 1e-6, lambda0 1e-4",
               iter_cost=[float(c) for c in r.iter_cost], accepted=[bool(a) for a in r.accepted],
               pcg_iters=[int(i) for i in r.pcg_iters],
               final_rms_px=O.rms(p, r.R, r.t, r.X),
               n_masked=O.cost_and_masked(p, r.R, r.t, r.X)[1],
               seconds=time.time() - t)
    with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
