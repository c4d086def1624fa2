"""The library's host code (model objects, workspaces, graph capture and
replay, tuner and tuner cache, the serving scheduler) under AddressSanitizer
with UndefinedBehaviorSanitizer and under ThreadSanitizer, on the CPU.

fgl_host.cpp, fgl_serve.cpp and fgl_plan.cpp are compiled with g++ as they
are, against a CPU stand-in of the HIP runtime (streams as in-order worker
threads, host functions on them, events, stream capture and graph replay)
and of the kernel launchers (tests/native/).  The driver,
tests/native/host_sched_test.cpp, checks the likelihood launch's channel
chunk plans and block map over many shapes, predicts every row's result
exactly and runs synchronous, device-pointer and gradient calls, eight threads on shared
models, and the serving scheduler with 16 client threads, with and without
shared launches and an HBM budget that forces eviction, and its cancellation
and queue wait limit.  The stand-ins
report reads of evicted model buffers and shared-launch plans that do not fit
their grids; after teardown no device or pinned allocation may be live.
"""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_13196_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SOURCES = [os.path.join(CSRC, f) for f in ("fgl_host.cpp", "fgl_serve.cpp", "fgl_plan.cpp")] + \
          [os.path.join(NATIVE, f) for f in ("hip_stub.cpp", "launch_stub.cpp",
                                              "host_sched_test.cpp")]
HIP_INCLUDE = "/opt/rocm/include"
SANITIZERS = {
    "asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "tsan": ["-fsanitize=thread"],
}

pytestmark = pytest.mark.skipif(
    shutil.which("g++") is None or not os.path.isdir(os.path.join(HIP_INCLUDE, "hip")),
    reason="needs g++ and the HIP headers")


@pytest.fixture(scope="module")
def binaries():
    out = tempfile.mkdtemp(prefix="fgl_san_")

    def build(name):
        exe = os.path.join(out, name)
        cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INCLUDE, "-g", "-O1",
               "-fno-omit-frame-pointer", *SANITIZERS[name], *SOURCES, "-o", exe, "-lpthread"]
        p = subprocess.run(cmd, capture_output=True, text=True)
        assert p.returncode == 0, p.stderr[-4000:]
        return name, exe

    with ThreadPoolExecutor(max_workers=2) as ex:
        exes = dict(ex.map(build, SANITIZERS))
    yield exes
    shutil.rmtree(out, ignore_errors=True)


def _run(exe, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    for k in ("FGL_TUNE", "FGL_NO_GRAPH", "FGL_DEVICE_GRAPHS", "FGL_SERVE_SHARE",
              "FGL_SERVE_FAIL_TICKET", "FGL_TUNE_CACHE", "FGL_HBM_BUDGET_MB", "LD_PRELOAD"):
        env.pop(k, None)
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    return p.returncode, p.stdout, p.stderr


def test_host_code_under_address_and_undefined_sanitizers(binaries):
    rc, out, err = _run(binaries["asan"], {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                                           "UBSAN_OPTIONS": "print_stacktrace=1"})
    print(out[-3000:])
    assert rc == 0, (out[-3000:], err[-6000:])
    assert "checks failed: 0, stand-in reports: 0" in out
    assert "shared" in out and "launches" in out


def test_host_code_under_thread_sanitizer(binaries):
    rc, out, err = _run(binaries["tsan"], {"TSAN_OPTIONS": "halt_on_error=0:exitcode=66"})
    print(out[-3000:])
    assert "WARNING: ThreadSanitizer" not in err, err[-8000:]
    assert rc == 0, (out[-3000:], err[-6000:])
    assert "checks failed: 0, stand-in reports: 0" in out
