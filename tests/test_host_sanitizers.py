"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU): the host sides of every translation unit are compiled
with the sanitizers (device code as usual), linked into a separate copy of
the library, and driven by tests/host_checks.cpp -- the request server's
arena allocator against a first-fit model, and the C ABI's argument
validation and plan arithmetic, including cc_workspace_bytes at extreme
sizes.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1612_01178_amd import build as hip_build  # noqa: E402

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN = "address,undefined"


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(hip_build.HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    objs, procs = [], []
    for src in hip_build.SOURCES:
        obj = str(tmp_path / (src.replace(".", "_") + ".o"))
        objs.append(obj)
        cmd = [hip_build.HIPCC, "-x", "hip", *hip_build.FLAGS,
               "-Xarch_host", "-fsanitize=" + SAN,
               "-Xarch_host", "-fno-sanitize-recover=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g",
               "-c", os.path.join(hip_build.CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, (src, out.decode(errors="replace")[-3000:])
    lib = str(tmp_path / "libhookcc_san.so")
    link = [CLANG, "-shared", "-fsanitize=" + SAN, *objs, "-o", lib,
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
            "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.check_call(link)
    exe = str(tmp_path / "host_checks")
    drv = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=" + SAN,
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "host_checks.cpp"), "-o", exe,
           "-L" + str(tmp_path), "-lhookcc_san", "-Wl,-rpath," + str(tmp_path),
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.check_call(drv)
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit: leak reports are not ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout + r.stderr
    assert "runtime error" not in report, report[-4000:]
    assert "AddressSanitizer" not in report, report[-4000:]
    assert r.returncode == 0 and "host checks ok" in r.stdout, report[-4000:]
