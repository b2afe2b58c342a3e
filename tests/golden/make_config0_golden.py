"""Writes tests/golden/config0_oracle.json: the FP64 dense normal-equation oracle's
run of the tiny arc scene (10 cameras, 1000 points, camera 0 fixed) for 20 LM
iterations (lambda0 1e-4).  Calls only synth/ and oracle/.  Takes seconds.

    python tests/golden/make_config0_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ba_oracle as O  # noqa: E402
from synth import make_config0  # noqa: E402


def main():
    s = make_config0()
    p = O.Problem.from_scene(s)
    t = time.time()
    r = O.lm_dense(p, O.LMOptions(max_iters=20))
    out = dict(scene="make_config0() (10 cameras, 1000 points, seed 1000)", n_obs=int(p.n_obs),
               schedule="20 LM iterations, dense normal equations, lambda0 1e-4",
               iter_cost=[float(c) for c in r.iter_cost], accepted=[bool(a) for a in r.accepted],
               final_rms_px=O.rms(p, r.R, r.t, r.X), seconds=time.time() - t)
    with open(os.path.join(HERE, "config0_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
