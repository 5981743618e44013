"""The host runtime (parameter checks, planning, tiling, Maxwell solve) built with
AddressSanitizer and UndefinedBehaviorSanitizer on the host code only, driven by
tests/native/host_abi_check.cpp (no GPU needed): every check passes and the
sanitizers report nothing."""

import os
import shutil
import subprocess

import pytest

from conftest import ROOT

HIPCC = "/opt/rocm/bin/hipcc"
CSRC = os.path.join(ROOT, "paper_2008_01473_amd", "csrc")


LIB = os.path.join(ROOT, "paper_2008_01473_amd", "liblbm.so")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")
def test_host_abi_under_asan_and_ubsan(tmp_path):
    """The host runtime (api.cpp, maxwell.cpp) and the driver are built with the
    sanitizers; the kernels' launch wrappers and shape tables come from the built
    library (no kernel runs in these checks)."""
    from paper_2008_01473_amd import build as B
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    flags = [f for f in B.COMMON_FLAGS if f != "-O3"] + ["-O1", "--cuda-host-only"]
    objs, procs = [], []
    sources = [os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "maxwell.cpp"),
               os.path.join(ROOT, "tests", "native", "host_abi_check.cpp")]
    for src in sources:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC] + flags + san + ["-x", "hip", "-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-3000:]
    drv = str(tmp_path / "host_abi_check")
    cmd = [HIPCC, "-g"] + san + objs + [LIB, "-Wl,-rpath," + os.path.dirname(LIB), "-o", drv]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([drv], capture_output=True, text=True, timeout=300, env=env)
    print(res.stdout, res.stderr[-3000:])
    assert res.returncode == 0, res.stderr[-3000:]
    assert "host ABI checks passed" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
