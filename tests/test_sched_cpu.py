"""Threading of the host scheduling code, on the CPU, under sanitizers.

The library's Batcher, buffer release with its fenced graveyard, launch
profiler, batch_run and request server (csrc/sched.hip, csrc/server.hip)
are built with g++ against a CPU stand-in of the HIP host calls
(tests/sched/fakehip) and driven by tests/sched/sched_test.cpp: 16 batch
workers and a 6-slot server with three submitting threads, cancellations,
pipelined products through the Batcher whose scratch grows while earlier
products may still use it, and a thread reading the profiler while solves
record launches.  Every product is checked against its input, every
allocation must come back exactly once, the allocator must never be entered
by two threads at once, and ThreadSanitizer and AddressSanitizer /
UndefinedBehaviorSanitizer must report nothing.

Two planted mistakes, each in a copy of sched.hip built for the CPU, show
that the checks can fail: the profiler's fold without its lock (a data
race ThreadSanitizer reports) and buffers returned to the allocator without
waiting for the streams that still use them (a use-after-free
AddressSanitizer reports).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_17133_amd", "csrc")
TESTS = os.path.join(ROOT, "tests", "sched")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def build(tmp_path, name, sanitize=None, sched=None):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer",
           "-I", os.path.join(TESTS, "fakehip"), "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if sanitize:
        cmd.append("-fsanitize=" + sanitize)
    cmd += ["-x", "c++", sched or os.path.join(CSRC, "sched.hip"), os.path.join(CSRC, "server.hip"),
            "-x", "none", os.path.join(TESTS, "sched_test.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def run(exe, rounds=3):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, str(rounds)], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.parametrize("sanitize", [None, "thread", "address,undefined"])
def test_scheduling_threads_are_clean(tmp_path, sanitize):
    r = run(build(tmp_path, "sched_%s" % (sanitize or "plain").replace(",", "_"), sanitize))
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "SCHED_OK" in r.stdout
    assert "Sanitizer" not in out and "runtime error" not in out


def _planted(tmp_path, old, new):
    src = open(os.path.join(CSRC, "sched.hip")).read()
    assert old in src
    path = tmp_path / "sched_planted.hip"
    path.write_text(src.replace(old, new))
    return str(path)


def test_planted_profiler_race_is_reported(tmp_path):
    planted = _planted(tmp_path, "void Profiler::resolve() {\n  std::lock_guard<std::mutex> g(mu);",
                       "void Profiler::resolve() {")
    r = run(build(tmp_path, "sched_race", "thread", planted), rounds=2)
    assert "ThreadSanitizer" in r.stdout + r.stderr


def test_planted_early_release_is_reported(tmp_path):
    planted = _planted(tmp_path, "      park = ctx->defer_free > 0;", "      park = false;")
    r = run(build(tmp_path, "sched_uaf", "address", planted), rounds=2)
    assert "heap-use-after-free" in r.stdout + r.stderr
