"""The allocation-free pose-only entry (ba_pose_batch_noalloc) against ba_pose_batch,
through the C-ABI.  Needs an MI355X."""
import sys

import numpy as np
import pytest

from synth import make_config4_requests

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["t"], b["t"])
    assert np.array_equal(a["status"], b["status"]) and np.array_equal(a["cost"], b["cost"])


def test_pose_batch_noalloc_equals_pose_batch_on_two_calls(balib):
    """Two calls in a row, the second with fewer and smaller requests and other
    options: each equals ba_pose_batch on the same input bit for bit (one kernel, one
    input; the staging array keeps the first call's contents beyond the second's)."""
    big = make_config4_requests(600, seed=1004)
    print("noalloc: 600 requests,", sum(len(r.X) for r in big), "correspondences", flush=True)
    a = balib.pose_batch(big, iters=10, huber_delta=1.0)
    b = balib.pose_batch_noalloc(big, iters=10, huber_delta=1.0)
    _same(a, b)
    small = make_config4_requests(37, seed=1007)
    for r in small:
        r.X, r.uv = r.X[: len(r.X) // 2 + 1], r.uv[: len(r.uv) // 2 + 1]
    print("noalloc: 37 requests,", sum(len(r.X) for r in small), "correspondences", flush=True)
    a2 = balib.pose_batch(small, iters=6, huber_delta=0.0)
    b2 = balib.pose_batch_noalloc(small, iters=6, huber_delta=0.0)
    _same(a2, b2)
    assert np.all(np.isfinite(b2["cost"])) and np.all(b2["status"] == 0)
    sys.stdout.flush()
