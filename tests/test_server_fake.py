"""The serving runtime and the batched C-ABI path on the CPU, under
AddressSanitizer (+ UndefinedBehaviorSanitizer) and ThreadSanitizer.

The product's host runtime (paper_2404_10631_amd/csrc/knnf_api.cpp and
knnf_server.cpp, unchanged) is compiled with g++ against a fake HIP runtime
(tests/fakehip: streams as worker threads, events, copies) whose "device"
executes every filtering launch with the CPU oracle, reading the work table
when the launch runs as a kernel would.  tests/fakehip/test_server_fake.cpp
then checks: a mixed stream sliced into small steps equals each frame
filtered alone and runs every tile exactly once; first-in-first-out
admission by pool memory (no overtaking); KNNF_EAGAIN for a full queue,
KNNF_ENOMEM for a frame larger than the pool, KNNF_ESTATE before a frame is
done; the plain mode's one-at-a-time order; non-finite host inputs rejected;
concurrent submitters; batch tables passed as a kernel argument and through
the pinned staging, with the input check; and an injected copy failure that
fails the server and its context for good.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = os.path.join(ROOT, "tests", "fakehip")
CSRC = os.path.join(ROOT, "paper_2404_10631_amd", "csrc")
SOURCES = [os.path.join(CSRC, "knnf_api.cpp"), os.path.join(CSRC, "knnf_server.cpp"),
           os.path.join(FAKE, "fake_runtime.cpp"), os.path.join(FAKE, "fake_device.cpp"),
           os.path.join(FAKE, "test_server_fake.cpp")]


@pytest.fixture(scope="module")
def oracle_obj(tmp_path_factory):
    """The C oracle as an optimised object without instrumentation (it is the
    reference here, not the code under test, and it is slow when sanitised)."""
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("g++/gcc not available")
    d = tmp_path_factory.mktemp("fakehip")
    obj = str(d / "oracle.o")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-c",
                    os.path.join(ROOT, "oracle", "knn_oracle.c"), "-o", obj], check=True)
    return d, obj


def build_and_run(d, obj, name, flags, env=None):
    exe = str(d / name)
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
            "-Wall", "-I", FAKE, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
           + flags + SOURCES + [obj, "-lpthread", "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
        pytest.skip(f"sanitizer not supported: {r.stderr[:200]}")
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, **(env or {})))
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "FAIL" not in run.stdout
    assert run.stdout.count("\nok ") + run.stdout.startswith("ok ") == 11, run.stdout
    return out


def test_serving_runtime_under_address_sanitizer(oracle_obj):
    d, obj = oracle_obj
    build_and_run(d, obj, "t_asan", ["-fsanitize=address,undefined"],
                  env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                       "UBSAN_OPTIONS": "halt_on_error=1"})


def test_serving_runtime_under_thread_sanitizer(oracle_obj):
    d, obj = oracle_obj
    out = build_and_run(d, obj, "t_tsan",
                        ["-fsanitize=thread", "-include", os.path.join(FAKE, "tsan_cond.h")],
                        env={"TSAN_OPTIONS": "halt_on_error=1"})
    assert "ThreadSanitizer" not in out
