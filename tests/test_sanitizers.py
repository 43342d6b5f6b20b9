"""The graph builder and the serving scheduler (mock mode, no device calls)
built with AddressSanitizer + UndefinedBehaviorSanitizer and with
ThreadSanitizer on the host, driven by tests/sanitize/host_driver.cpp.  Any
sanitizer report makes the driver exit non-zero.  Only the host parts are
instrumented: the HIP translation unit of the scheduler is compiled with the
sanitizer flags for its host pass only (no GPU code is built with them)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_11402_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = [pytest.mark.slow, pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                                                   reason="ROCm toolchain not installed")]


def _build(tmp, kind):
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-pthread", "-I" + INCLUDE, "-I" + CSRC]
    san = ["address", "undefined"] if kind == "asan" else ["thread"]
    host_flags = ["-fsanitize=" + s for s in san]
    objs = []
    for src in ("graph.cpp", "graph_io.cpp", "status.cpp"):
        obj = os.path.join(tmp, src + ".o")
        subprocess.run([CLANG, "-c", os.path.join(CSRC, src), "-o", obj, "-ffp-contract=off"] + common + host_flags,
                       check=True)
        objs.append(obj)
    obj = os.path.join(tmp, "driver.o")
    subprocess.run([CLANG, "-c", DRIVER, "-o", obj] + common + host_flags, check=True)
    objs.append(obj)
    # the scheduler's translation unit: sanitizer flags on its host pass only
    obj = os.path.join(tmp, "serve.o")
    hip_host = []
    for s in san:
        hip_host += ["-Xarch_host", "-fsanitize=" + s]
    subprocess.run([HIPCC, "-c", os.path.join(CSRC, "serve.hip"), "-o", obj, "--offload-arch=gfx950"] + common +
                   hip_host, check=True)
    objs.append(obj)
    exe = os.path.join(tmp, "driver_" + kind)
    link = []
    for s in san:
        link += ["-Xarch_host", "-fsanitize=" + s]
    subprocess.run([HIPCC, "-o", exe, "--offload-arch=gfx950"] + objs + ["-pthread"] + link, check=True)
    return exe


@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_parts_under_sanitizers(tmp_path, kind):
    exe = _build(str(tmp_path), kind)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    proc = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(proc.stdout[-4000:])
    assert proc.returncode == 0, proc.stdout[-4000:]
    assert "host driver ok" in proc.stdout
    assert "runtime error" not in proc.stdout          # UBSan reports without halting on some checks
