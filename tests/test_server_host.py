"""Host-only test of the request server's threads (admission, two compute lanes, pool, poll
queue): server.hip is compiled with g++ and ThreadSanitizer against a stub of the HIP
runtime calls it makes and a stub of the batched count (tests/server_host/), and a driver
runs a burst through a small pool, one-request launches, failing requests (too large for
the pool, invalid, a failed copy) and a served arrival mix, under a stall watchdog.  No GPU
is used.  ROCm's clang builds it: GCC 11's ThreadSanitizer does not intercept the
pthread_cond_clockwait that its libstdc++ uses for timed waits and reports false races."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "server_host")


def test_server_threads_on_host(tmp_path):
    cxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(cxx):
        pytest.skip("no ROCm clang++")
    # the server source is copied to a .cpp so that the host compiler builds it as C++
    server_cpp = tmp_path / "server_host.cpp"
    with open(os.path.join(ROOT, "paper_1608_05138_amd", "csrc", "server.hip")) as f:
        server_cpp.write_text(f.read())
    exe = tmp_path / "server_host"
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-I", SRC, "-I", os.path.join(ROOT, "paper_1608_05138_amd", "csrc"),
           "-include", os.path.join(SRC, "hip", "hip_runtime.h"),
           str(server_cpp), os.path.join(SRC, "stub_runtime.cpp"), os.path.join(SRC, "driver.cpp"),
           "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env=env)
    print(p.stdout)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "WARNING: ThreadSanitizer" not in p.stderr, p.stderr
