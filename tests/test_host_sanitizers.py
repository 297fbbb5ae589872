"""Host code under sanitizers, on the CPU (no GPU): the serving scheduler driven by a fake
backend (tests/sched_fake.cpp, virtual clock, scripted launch failures, budgeted images,
client threads) and the FP64 oracle's C code (tests/oracle_sanitize.c).  Each program is
built with g++/gcc plain, with AddressSanitizer + UndefinedBehaviorSanitizer, and with
ThreadSanitizer, and every run must be clean."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_08735_amd", "csrc")
ORACLE = os.path.join(ROOT, "oracle")
ORACLE_SOURCES = ["quad.c", "geodesic.c", "tables.c", "emission.c", "render.c", "animate.c",
                  "march.c", "bloom.c", "tonemap.c", "area.c", "spectrum.c"]

SCENARIOS = ["fifo_order", "continuous_batching", "admission_by_budget",
             "eagain_when_queue_full", "launch_failure_is_contained", "cancel_on_stop",
             "one_table_set_per_launch", "pool_gives_back_for_other_sizes", "threads"]

FLAVOURS = {
    "plain": ["-O2"],
    "asan_ubsan": ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                   "-fno-omit-frame-pointer"],
    "tsan": ["-O1", "-g", "-fsanitize=thread"],
}


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_sanitizers")
    out = {}
    for name, flags in FLAVOURS.items():
        exe = str(d / ("sched_fake_" + name))
        subprocess.run(["g++", "-std=c++17", "-Wall", "-Wextra", "-I", CSRC] + flags +
                       [os.path.join(ROOT, "tests", "sched_fake.cpp"), "-o", exe, "-lpthread"],
                       check=True)
        out[("sched", name)] = exe
        if name != "plain":
            exe = str(d / ("oracle_" + name))
            subprocess.run(["gcc", "-std=gnu11", "-I", ORACLE] + flags +
                           [os.path.join(ROOT, "tests", "oracle_sanitize.c")] +
                           [os.path.join(ORACLE, s) for s in ORACLE_SOURCES] +
                           ["-o", exe, "-lm", "-lpthread"], check=True)
            out[("oracle", name)] = exe
    return out


def _run_clean(cmd):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               TSAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.parametrize("flavour", list(FLAVOURS))
@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_with_fake_backend(builds, scenario, flavour):
    out = _run_clean([builds[("sched", flavour)], scenario])
    assert scenario + " ok" in out


@pytest.mark.parametrize("flavour", ["asan_ubsan", "tsan"])
def test_oracle_under_sanitizers(builds, flavour):
    assert "ok" in _run_clean([builds[("oracle", flavour)]])
