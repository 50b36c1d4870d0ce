"""Host code under the sanitizers (no GPU):

* the serving scheduler (paper_1603_02655_amd/csrc/tc_sched.cpp) driven by a
  fake round executor with injected faults (tests/native/sched_check.cpp):
  a failed launch, a build error, a round that never finishes (watchdog), a
  round held while its graph must stay busy, stop with work in flight and
  queued, admission by footprint in arrival order;
* the CPU oracle and the multicore CPU census against the oracle's brute force
  (tests/native/oracle_check.c).

Each runs built plainly, with AddressSanitizer + UndefinedBehaviorSanitizer
(g++/gcc) and with ThreadSanitizer.  The ThreadSanitizer builds use ROCm's
clang: the libtsan of this image's g++ does not intercept
pthread_cond_clockwait (what std::condition_variable::wait_for calls), so it
reports every timed wait as a double lock.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1603_02655_amd", "csrc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
CLANG_C = "/opt/rocm/lib/llvm/bin/clang"

VARIANTS = {
    "plain": ("g++", "gcc", ["-O2"]),
    "asan-ubsan": ("g++", "gcc", ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                  "-fno-sanitize-recover=undefined"]),
    "tsan": (CLANG, CLANG_C, ["-O1", "-g", "-fsanitize=thread"]),
}


def _need(tool):
    if not (shutil.which(tool) or os.path.exists(tool)):
        pytest.skip(f"{tool} not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_scheduler_with_fake_executor(tmp_path, variant):
    cxx, _, flags = VARIANTS[variant]
    _need(cxx)
    exe = str(tmp_path / "sched_check")
    _run([cxx, "-std=c++17", "-Wall", "-Wextra", *flags, "-pthread", "-I", CSRC,
          os.path.join(NATIVE, "sched_check.cpp"), os.path.join(CSRC, "tc_sched.cpp"), "-o", exe])
    r = _run([exe], timeout=300, env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1"))
    assert "all scheduler scenarios passed" in r.stdout
    assert "ThreadSanitizer" not in r.stderr and "ERROR" not in r.stderr, r.stderr[-4000:]


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_oracle_and_cpu_census(tmp_path, variant):
    cxx, cc, flags = VARIANTS[variant]
    _need(cxx)
    _need(cc)
    objs = []
    for src, comp, std in ((os.path.join(ROOT, "oracle", "oracle.c"), cc, "-std=gnu11"),
                           (os.path.join(NATIVE, "oracle_check.c"), cc, "-std=gnu11"),
                           (os.path.join(ROOT, "paper_1603_02655_amd", "cpu", "tc_cpu.cpp"), cxx, "-std=c++17")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([comp, std, *flags, "-pthread", "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "oracle_check")
    _run([cxx, *flags, "-pthread", *objs, "-o", exe])
    r = _run([exe], timeout=600, env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert "agree" in r.stdout
    assert "ThreadSanitizer" not in r.stderr and "ERROR" not in r.stderr, r.stderr[-4000:]
