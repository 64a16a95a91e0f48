"""The library's host code (pcv_problem.cpp, pcv_capi.cpp, pcv_server.cpp,
pcv_tune.cpp) built with g++ under AddressSanitizer and UBSan against a CPU
stand-in of the HIP runtime and of the kernel launchers
(tests/host_harness/hip_stub.cpp), driven through the C ABI
(tests/host_harness/driver.cpp):

  sequence  graph capture and replay across evaluations, batched and grid
            evaluations, factorisation, prediction (both entry points),
            local factors, GLS, a server toggling the served mode twice,
            eager / profiled / forced-fallback / busy-device variants, three
            times on fresh problems;
  oom       a memory cap below the problem's need: PCV_ERR_OOM with nothing
            left behind; a device allocation failing at each point of a
            multi-theta call: the workspace or plan that did not fit is
            given up and the theta values go one at a time; the same at
            each allocation of a server's creation (PCV_ERR_OOM, the problem
            back on its own stream, nothing left behind);
  tune      the autotuner on three problems of two shapes in both
            precisions: timing, the cache file (written, then reused for the
            identical problem), evaluations, batches and a server after
            tuning, tuning refused while served and repeated after.

The stand-in stops the process on a dead handle, a device pointer outside
every live allocation (also when a captured graph is replayed), a call the
capture mode forbids, or resources left alive after every problem is gone.
No GPU is used."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_13132_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host_harness")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
FLAGS = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
         "-I" + os.path.join(ROOT, "include")] + SAN


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++") or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("g++ or the HIP headers are missing")
    out = tmp_path_factory.mktemp("host_harness")
    srcs = [os.path.join(CSRC, f) for f in ("pcv_problem.cpp", "pcv_capi.cpp", "pcv_server.cpp", "pcv_tune.cpp")]
    srcs += [os.path.join(HARNESS, "hip_stub.cpp"), os.path.join(HARNESS, "driver.cpp")]
    objs = [str(out / (os.path.basename(s) + ".o")) for s in srcs]

    def cc(args):
        src, obj = args
        r = subprocess.run(["g++"] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]

    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        list(ex.map(cc, zip(srcs, objs)))
    exe = str(out / "driver")
    r = subprocess.run(["g++"] + SAN + ["-o", exe] + objs + ["-pthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe, out


def _run(driver, *args):
    exe, out = driver
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe] + list(args), capture_output=True, text=True, env=env, cwd=str(out), timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    return r.stdout


def test_call_sequences_clean_under_sanitizers(driver):
    out = _run(driver, "sequence")
    assert "live device allocations 0, pinned 0, streams 0, events 0" in out


def test_memory_cap_rejects_without_side_effects(driver):
    out = _run(driver, "oom")
    assert "nothing left behind" in out
    # a device allocation failing at every point of a multi-theta call
    # (the single evaluations need no new device memory here, so every call
    # completes; early failures give the workspace up, late ones keep it)
    m = re.search(r"oom_batch: (\d+) calls ok, (\d+) out of memory, (\d+) gave the workspace up", out)
    assert m and int(m.group(1)) == 60 and 0 < int(m.group(3)) < 60, out[-2000:]
    m = re.search(r"oom_server: (\d+) created, (\d+) out of memory", out)
    assert m and int(m.group(1)) > 0 and int(m.group(2)) > 0, out[-2000:]
    m = re.search(r"oom_tune: (\d+) tuned, (\d+) out of memory", out)
    assert m and int(m.group(1)) > 0 and int(m.group(2)) > 0, out[-2000:]
    m = re.search(r"launch_fail: (\d+) completed, (\d+) failed", out)
    assert m and int(m.group(1)) > 0 and int(m.group(2)) > 0, out[-2000:]


def test_tuner_cycle_clean_under_sanitizers(driver):
    cache = str(driver[1] / "tune_cache.txt")
    out = _run(driver, "tune", cache)
    assert "from_cache 1" in out
    lines = open(cache).read().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == 4  # two shapes x two precisions
