"""The served form's host side (request queue, admission by scratch budget, worker loop:
csrc/serve_core.h) on the CPU, with a stand-in for the query, built with the thread sanitizer
and with the address sanitizer: every request completes with its own result, the scratch the
workers keep never exceeds the budget (idle workers give theirs back when a request fits nowhere
else), and the loop ends."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_serve_core_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "harness")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-pthread", "-I",
                    os.path.join(os.path.dirname(HERE), "include"), "-o", exe,
                    os.path.join(HERE, "serve_core_harness.cpp")], check=True)
    for slots, n in ((1, 300), (3, 2000), (8, 4000)):
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([exe, str(slots), str(n)], capture_output=True, text=True, timeout=120, env=env)
        assert r.returncode == 0, (slots, r.stdout, r.stderr[-3000:])
        assert "over_budget 0 bad 0" in r.stdout, r.stdout
