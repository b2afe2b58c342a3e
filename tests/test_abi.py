"""C-ABI checks that need no GPU: every symbol of include/ba.h is exported, and
argument validation rejects bad input before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import make_arc_scene, make_config4_requests

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(balib):
    names = _declared_functions()
    assert len(names) >= 19
    lib = ctypes.CDLL(balib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_defaults(balib):
    assert b"gfx950" in balib.lib().ba_version()
    o = balib.options()
    assert o.max_iters == 10 and o.pcg_max_iters == 50 and o.precision == 1


def _expect(balib, code, fn):
    with pytest.raises(balib.BAError) as e:
        fn()
    assert e.value.code == code
    return str(e.value)


@pytest.mark.parametrize("mutate,needle", [
    (lambda d: d.obs["cam"].__setitem__(0, 99), "camera 99"),
    (lambda d: d.obs["pt"].__setitem__(3, 10**6), "out of range"),
    (lambda d: d.obs["u"].__setitem__(2, np.nan), "non-finite"),
    (lambda d: d.X.__setitem__((1, 1), np.inf), "non-finite"),
    (lambda d: d.poses.__setitem__((1, 0), 2.0), "quaternion"),
    (lambda d: d.K.__setitem__((0, 0), 0.0), "intrinsics"),
])
def test_create_rejects_invalid_input(balib, mutate, needle):
    s = make_arc_scene(3, 20, seed=1)
    d = balib.scene_desc(s)
    mutate(d)
    msg = _expect(balib, balib.BA_EINVAL, lambda: balib.Problem(d, balib.options()))
    assert needle in msg


def test_create_rejects_duplicates_empty_and_all_fixed(balib):
    s = make_arc_scene(3, 20, seed=1)
    d = balib.scene_desc(s)
    d.obs[1] = d.obs[0]
    assert "twice" in _expect(balib, balib.BA_EINVAL, lambda: balib.Problem(d, balib.options()))
    d = balib.scene_desc(s)
    d.desc.n_obs = 0
    _expect(balib, balib.BA_EINVAL, lambda: balib.Problem(d, balib.options()))
    s2 = make_arc_scene(3, 20, seed=1)
    s2.cam_fixed[:] = 1
    assert "fixed" in _expect(balib, balib.BA_EINVAL,
                              lambda: balib.Problem(balib.scene_desc(s2), balib.options()))


def test_options_validation(balib):
    s = make_arc_scene(3, 20, seed=1)
    for kw in [dict(max_iters=0), dict(pcg_max_iters=0), dict(lambda0=0.0),
               dict(pcg_rel_tol=-1.0), dict(precision=7), dict(huber_delta=np.inf), dict(flags=5), dict(flags=128),
               dict(prior_abs=-1.0), dict(prior_seq=np.nan), dict(prior_seq=1.0, prior_seq_k=0),
               dict(prior_seq=1.0, prior_seq_k=65)]:
        _expect(balib, balib.BA_EINVAL, lambda: balib.Problem(balib.scene_desc(s), balib.options(**kw)))


def test_pose_batch_validation(balib):
    reqs = make_config4_requests(2, seed=1004)
    reqs[1].X = reqs[1].X.copy()
    reqs[1].X[0, 0] = np.nan
    _expect(balib, balib.BA_EINVAL, lambda: balib.pose_batch(reqs))
    r = make_config4_requests(1, seed=1004)[0]
    r.X = np.zeros((balib.POSE_MAX_CORR + 1, 3))
    r.uv = np.zeros((balib.POSE_MAX_CORR + 1, 2))
    _expect(balib, balib.BA_EINVAL, lambda: balib.pose_batch([r]))
    _expect(balib, balib.BA_EINVAL, lambda: balib.pose_batch_noalloc([r]))
    _expect(balib, balib.BA_EINVAL, lambda: balib.pose_batch_noalloc(reqs))


def test_pose_batch_noalloc_rejects_oversize_batch(balib):
    """A batch whose staging exceeds the fixed array fails with BA_ENOMEM before any
    device work (160 bytes per request and 32 per correspondence)."""
    base = make_config4_requests(1, seed=1004)[0]
    n = balib.POSE_MAX_CORR
    per_req = 160 + 32 * n
    k = balib.POSE_NOALLOC_MAX_BYTES // per_req + 1
    X = np.tile(base.X[:1], (n, 1))
    uv = np.tile(base.uv[:1], (n, 1))
    big = []
    for _ in range(k):
        r = make_config4_requests(1, seed=1004)[0]
        r.X, r.uv = X, uv
        big.append(r)
    _expect(balib, balib.BA_ENOMEM, lambda: balib.pose_batch_noalloc(big))


def test_server_create_validation(balib):
    _expect(balib, balib.BA_EINVAL, lambda: balib.Server(1024, 4))
    _expect(balib, balib.BA_EINVAL, lambda: balib.Server(1 << 30, 0))
    _expect(balib, balib.BA_EINVAL, lambda: balib.Server(1 << 30, 4, precision=9))


def test_refine_validation(balib):
    """ba_refine checks its stage list before the problem handle, so every rule
    is visible without a device."""
    L = balib.lib()

    def call(stages, rounds, n=None):
        st = (balib.RefineStage * max(len(stages), 1))(*[balib.RefineStage(g[0], g[1], g[2] if len(g) > 2 else 0, 0)
                                                          for g in stages])
        rc = L.ba_refine(None, len(stages) if n is None else n, st, rounds, None)
        return rc, L.ba_last_error().decode()

    assert call([], 1)[1].startswith("n_stages")
    assert call([(1.0, 8.0)], 0)[1].startswith("rounds")
    for bad, needle in [((np.nan, 8.0), "huber_delta"), ((1.0, 0.0), "cull_px"),
                        ((1.0, -2.0), "cull_px"), ((0.0, np.inf), "cull_px")]:
        rc, msg = call([(1.0, 8.0), bad], 2)
        assert rc == balib.BA_EINVAL and "stage 1" in msg and needle in msg, msg
    rc, msg = call([(1.0, 8.0), (0.0, 3.0, 2)], 2)
    assert rc == balib.BA_EINVAL and "stage 1" in msg and "triangulation" in msg, msg
    rc, msg = call([(1.0, 8.0), (0.0, 3.0)], 2)
    assert rc == balib.BA_EINVAL and "NULL" in msg
    assert L.ba_get_active(None, None) == balib.BA_EINVAL


def test_pose_graph_validation(balib):
    """ba_pose_graph_create rejects bad graphs before touching the device."""
    from synth import make_pose_graph
    g = make_pose_graph(4, mode="rig")

    def expect(mutate, needle, **kw):
        gd = balib.pose_graph_desc(g)
        mutate(gd)
        h = ctypes.c_void_p()
        rc = balib.lib().ba_pose_graph_create(ctypes.byref(gd.desc), ctypes.byref(balib.options(**kw)), None,
                                              ctypes.byref(h))
        msg = balib.lib().ba_last_error().decode()
        assert rc == balib.BA_EINVAL and needle in msg, (needle, msg)

    def set_edge(k, field, value):
        def f(gd):
            gd.edges[field][k] = value
        return f

    expect(set_edge(3, "j", g.n_nodes), "out of range")
    expect(set_edge(3, "i", -1), "out of range")
    expect(set_edge(2, "j", int(g.edge_i[2])), "itself")
    expect(set_edge(1, "w_rot", -1.0), "weights")
    expect(set_edge(1, "w_trans", np.nan), "weights")

    def both_zero(gd):
        gd.edges["w_rot"][0] = 0.0
        gd.edges["w_trans"][0] = 0.0
    expect(both_zero, "weights")
    expect(set_edge(0, "q", [2.0, 0.0, 0.0, 0.0]), "quaternion")

    def duplicate(gd):  # the reverse of edge 0
        gd.edges["i"][1], gd.edges["j"][1] = gd.edges["j"][0], gd.edges["i"][0]
    expect(duplicate, "two edges")

    def all_fixed(gd):
        gd.fixed = np.ones(g.n_nodes, np.uint8)
        gd.desc.node_fixed = gd.fixed.ctypes.data_as(ctypes.c_void_p)
    expect(all_fixed, "fixed")
    expect(lambda gd: None, "robust loss", huber_delta=1.0)
    expect(lambda gd: None, "prior_seq", prior_seq=1.0)


def test_rig_validation(balib):
    """ba_rig_create rejects bad rig descriptions before touching the device."""
    from synth import make_rig_drive
    s = make_rig_drive(4, 60, seed=3)

    def expect(needle, mutate=None, pairs=((0, 1),), prior_ext=1.0, prior_rig=1.0, **kw):
        rd = balib.rig_desc(s, prior_ext, prior_rig, np.array(pairs))
        if mutate:
            mutate(rd)
        h = ctypes.c_void_p()
        rc = balib.lib().ba_rig_create(ctypes.byref(rd.desc), ctypes.byref(balib.options(**kw)), None,
                                       ctypes.byref(h))
        msg = balib.lib().ba_last_error().decode()
        assert rc == balib.BA_EINVAL and needle in msg, (needle, msg)

    def set_obs(field, value):
        def f(rd):
            rd.obs[field][0] = value
        return f

    expect("frame or rig camera", set_obs("frame", s.n_frames))
    expect("frame or rig camera", set_obs("cam", s.n_rig))
    expect("rig pair", pairs=((0, 0),))
    expect("rig pair", pairs=((0, 3),))
    expect("twice", pairs=((0, 1), (1, 0)))
    expect("prior_ext", prior_ext=-1.0)
    expect("prior_ext", prior_rig=float("nan"))
    expect("priors from the rig description", prior_abs=1.0)

    def bad_quat(rd):
        rd.ep[1, :4] = [2.0, 0.0, 0.0, 0.0]
    expect("quaternion", bad_quat)

    def too_many(rd):
        rd.desc.n_rig = 17
    expect("n_rig", too_many)


def test_triangulate_validation(balib):
    s = make_arc_scene(3, 20, seed=1)
    d = balib.scene_desc(s)
    L = balib.lib()
    X = np.zeros((s.n_pts, 3))
    ok = np.zeros(s.n_pts, np.uint8)

    def call(method=0, out=True):
        rc = L.ba_triangulate(ctypes.byref(d.desc), method, None, X.ctypes.data_as(ctypes.c_void_p) if out else None,
                              ok.ctypes.data_as(ctypes.c_void_p), None)
        return rc, L.ba_last_error().decode()

    rc, msg = call(method=5)
    assert rc == balib.BA_EINVAL and "method" in msg
    rc, msg = call(out=False)
    assert rc == balib.BA_EINVAL and "NULL" in msg
    d.obs["pt"][0] = s.n_pts
    rc, msg = call()
    assert rc == balib.BA_EINVAL and "out of range" in msg


# The binding's ctypes structs and numpy record dtypes, with the C struct each mirrors.
_MIRRORS = [("Intrinsics", "ba_intrinsics"), ("Pose", "ba_pose"), ("Options", "ba_options"),
            ("Report", "ba_report"), ("ProblemDesc", "ba_problem_desc"),
            ("PoseRequest", "ba_pose_request"), ("ProblemInfo", "ba_problem_info"),
            ("PoseEdge", "ba_pose_edge"), ("PoseGraphDesc", "ba_pose_graph_desc"),
            ("RigDesc", "ba_rig_desc"), ("RefineStage", "ba_refine_stage"),
            ("RefineRound", "ba_refine_round"), ("ServerStats", "ba_server_stats_t"),
            ("DebugIteration", "ba_debug_iteration")]
_DTYPES = [("OBS_DTYPE", "ba_obs"), ("RIG_OBS_DTYPE", "ba_rig_obs"), ("EDGE_DTYPE", "ba_pose_edge")]
_DTYPE_FIELDS = {"q": "meas.qw", "t": "meas.tx"}  # EDGE_DTYPE flattens the measured pose


def test_binding_layouts_and_constants_match_header(balib, tmp_path):
    """Every struct the binding mirrors has the C compiler's size and field offsets
    (a C program built against include/ba.h with gcc prints them), and the binding's
    flag and method constants equal the header's #defines."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines, expect = [], []
    for py, c in _MIRRORS:
        S = getattr(balib, py)
        lines.append(f'printf("%zu\\n", sizeof({c}));')
        expect.append(ctypes.sizeof(S))
        for name, _ in S._fields_:
            cname = "lambda" if name == "lambda_" else name
            lines.append(f'printf("%zu\\n", offsetof({c}, {cname}));')
            expect.append(getattr(S, name).offset)
    for py, c in _DTYPES:
        dt = getattr(balib, py)
        lines.append(f'printf("%zu\\n", sizeof({c}));')
        expect.append(dt.itemsize)
        for name in dt.names:
            lines.append(f'printf("%zu\\n", offsetof({c}, {_DTYPE_FIELDS.get(name, name)}));')
            expect.append(dt.fields[name][1])
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "ba.h"\nint main(void) {\n'
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == expect
    hdr = open(os.path.join(ROOT, "include", "ba.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"#define (BA_[A-Z0-9_]+) \(?(-?\d+)\)?", hdr)}
    assert balib.POSE_NOALLOC_MAX_BYTES == defs["BA_POSE_NOALLOC_MAX_BYTES"]
    for name in ("OK", "DAMPING", "NUMERICAL", "PCG_SYNC"):
        assert getattr(balib, "STATUS_" + name) == defs["BA_STATUS_" + name], name
    assert balib.POSE_MAX_CORR == defs["BA_POSE_MAX_CORR"]
    for name in ("NO_GRAPH", "PAIR_LISTS", "PCG_WIDE", "PCG_RESIDENT", "DENSE_SCHUR", "PCG_COOPERATIVE"):
        assert getattr(balib, "FLAG_" + name) == defs["BA_FLAG_" + name], name
    assert balib.TRI == {"midpoint": defs["BA_TRI_MIDPOINT"], "dlt": defs["BA_TRI_DLT"]}
    assert balib.PREC == {"f64": defs["BA_PREC_F64"], "f32": defs["BA_PREC_F32"],
                          "f16j": defs["BA_PREC_F16J"], "bf16j": defs["BA_PREC_BF16J"]}
