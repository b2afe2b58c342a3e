"""The symbolic analysis alone (ba_analyse), CPU only: the observation-pair count and the
stored block pattern against counts made here with NumPy, the Schur form chosen for
banded and dense co-visibility, and the forcing flags."""
import numpy as np
import pytest

from synth import make_arc_scene, make_config0, make_small_drive


def _pairs_and_pattern(s):
    """Observation pairs of one point in two free cameras, and the number of stored
    6x6 blocks of S (co-visible free-camera pairs, both triangles, plus the diagonal)."""
    free = ~s.cam_fixed.astype(bool)
    fidx = -np.ones(s.n_cams, np.int64)
    fidx[free] = np.arange(free.sum())
    m = free[s.obs_cam]
    cnt = np.bincount(s.obs_pt[m], minlength=s.n_pts)
    pairs = int((cnt * (cnt - 1) // 2).sum())
    nf = int(free.sum())
    cov = np.zeros((nf, nf), bool)
    order = np.argsort(s.obs_pt[m], kind="stable")
    pt, cam = s.obs_pt[m][order], fidx[s.obs_cam[m][order]]
    starts = np.flatnonzero(np.r_[True, pt[1:] != pt[:-1]])
    for a, b in zip(starts, np.r_[starts[1:], len(pt)]):
        c = cam[a:b]
        cov[np.ix_(c, c)] = True
    np.fill_diagonal(cov, True)
    return pairs, int(cov.sum()), nf


@pytest.mark.parametrize("make,flags,form", [
    (lambda: make_small_drive(40, 3000, seed=5), 0, 1),      # banded: point chunks
    (lambda: make_small_drive(40, 3000, seed=5), 4, 0),      # BA_FLAG_PAIR_LISTS
    (lambda: make_small_drive(40, 3000, seed=5), 32, 2),     # BA_FLAG_DENSE_SCHUR forces it
    (make_config0, 0, 2),                                    # every camera sees most points
    (lambda: make_arc_scene(30, 2000, seed=74), 4, 0),       # pair lists exclude the dense form
])
def test_analysis_sizes_and_form(balib, make, flags, form):
    s = make()
    info, nbytes = balib.analyse(balib.scene_desc(s), balib.options(flags=flags))
    pairs, nnzb, nf = _pairs_and_pattern(s)
    assert info["schur_form"] == form
    assert info["n_pairs"] == pairs
    assert info["n_free_cams"] == nf and info["n_obs"] == s.n_obs
    # the dense form holds every block; the sparse forms exactly the co-visible ones
    assert info["nnzb"] == (nf * nf if form == 2 else nnzb)
    assert info["n_up_blocks"] == (info["nnzb"] - nf) // 2
    assert nbytes > 0


def test_analysis_rejects_invalid_input(balib):
    s = make_small_drive(20, 800, seed=9)
    s.obs_cam = s.obs_cam.copy()
    s.obs_pt = s.obs_pt.copy()
    s.obs_cam[1], s.obs_pt[1] = s.obs_cam[0], s.obs_pt[0]
    with pytest.raises(balib.BAError) as e:
        balib.analyse(balib.scene_desc(s), balib.options())
    assert e.value.code == balib.BA_EINVAL and "twice" in str(e.value)


@pytest.mark.parametrize("n_cams,mean_track,flags,rows", [
    (40, 8.0, 0, 4),       # few rows: 4 per tile
    (40, 8.0, 8, 32),      # BA_FLAG_PCG_WIDE
    (1100, 8.0, 0, 16),    # 1024 or more free cameras, sparse rows
    (1100, 24.0, 0, 16),   # ... and rows of about 47 blocks: 4-row tiles would outnumber the CUs
])
def test_pcg_rows_per_tile(balib, n_cams, mean_track, flags, rows):
    """Rows of the reduced system per PCG workgroup: 4 below 1024 free cameras, 16 from
    there on whatever the row density, 32 with BA_FLAG_PCG_WIDE."""
    s = make_small_drive(n_cams, 20 * n_cams, seed=9, mean_track=mean_track)
    info, _ = balib.analyse(balib.scene_desc(s), balib.options(flags=flags))
    _, nnzb, nf = _pairs_and_pattern(s) if n_cams < 200 else (0, info["nnzb"], info["n_free_cams"])
    assert info["pcg_rows"] == rows, (info["pcg_rows"], nnzb / nf)
    if mean_track > 20:
        assert nnzb > 24 * nf  # the rows are dense: the rule does not ask for sparse rows
