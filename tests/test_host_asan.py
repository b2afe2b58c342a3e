"""The library's host code (analysis, set-up, packing, server and validation) under
AddressSanitizer, CPU only: the host sources are compiled with ASan for the host side
alone (-Xarch_host), linked with the ordinary kernel object into a separate library, and
driven by tests/asan/host_driver.cpp through the C-ABI.  Without a device every call
stops after its host work (BA_EDEVICE), so the run covers the symbolic analysis in all
three Schur forms, the pose-graph and rig set-up, pose-request packing and every
validation path."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_15271_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SOURCES = ["ba_host.cpp", "ba_server.cpp", "ba_pose.cpp", "ba_noalloc.hip"]
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_host_code_under_address_sanitizer(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    kobj = os.path.join(ROOT, "paper_2510_15271_amd", "_build", "ba_kernels_hip.o")
    if not os.path.exists(kobj):
        from paper_2510_15271_amd import build_lib
        build_lib.build()
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = [kobj]
    for src in HOST_SOURCES:
        obj = str(tmp_path / (src.replace(".", "_") + ".o"))
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC"] + ASAN + DEVICE + inc +
             ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = str(tmp_path / "libba_asan.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared"] + ASAN + ["-o", lib] + objs + ["-lpthread"])
    exe = str(tmp_path / "host_driver")
    dobj = str(tmp_path / "host_driver.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC"] + ASAN + DEVICE + inc +
         ["-c", os.path.join(ROOT, "tests", "asan", "host_driver.cpp"), "-o", dobj])
    _run([HIPCC, "--offload-arch=gfx950"] + ASAN + [dobj, "-o", exe, "-L" + str(tmp_path), "-lba_asan",
                                                     "-Wl,-rpath," + str(tmp_path)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 unexpected statuses" in r.stdout
