"""Host-only tests of the server's scheduling core (no GPU).

tests/host/sched_test.cpp drives fsa_sched.hpp with a scripted backend and
a virtual clock: arrival-order admission under the HBM budget, continuous
admission as completions free resources, rejection of requests that can
never fit, cancellation, LRU tensor-cache eviction, failure isolation,
slot limits and latency percentiles.  Built with AddressSanitizer and
UndefinedBehaviorSanitizer.

tests/host/server_tsan.cpp runs the scheduler with its threads (Runner:
submitting threads that admit and launch, one waiter thread per device
queue) against a fake device, under ThreadSanitizer: concurrent submits,
polls, waits with and without timeouts, cancellations, evictions under a
tight budget, and a shutdown with work in flight.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_core(tmp_path):
    exe = tmp_path / "sched_test"
    src = os.path.join(ROOT, "tests", "host", "sched_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", src, "-o",
                    str(exe), "-lpthread"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK (0 failures)" in r.stdout


def test_server_threads_under_thread_sanitizer(tmp_path):
    exe = tmp_path / "server_tsan"
    src = os.path.join(ROOT, "tests", "host", "server_tsan.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", src, "-o", str(exe),
                    "-lpthread"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK (0 failures)" in r.stdout
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
