"""Host-only tests of the server's scheduling core (no GPU).

tests/host/sched_test.cpp drives fsa_sched.hpp with a scripted backend and
a virtual clock: arrival-order admission under the HBM budget, continuous
admission as completions free resources, rejection of requests that can
never fit, cancellation, LRU tensor-cache eviction, failure isolation,
slot limits and latency percentiles.  Built with AddressSanitizer and
UndefinedBehaviorSanitizer.
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
