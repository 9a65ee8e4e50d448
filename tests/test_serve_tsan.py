"""The serving loop's scheduler under ThreadSanitizer, on the CPU.

tests/serve_tsan_driver.cpp drives la_serve.cpp (compiled into the driver
with -fsanitize=thread; the rest of the library is linked uninstrumented)
from several client threads at once on the fake executor: submissions,
polls, releases, admission pauses, early and late injected failures,
summary reuse and shutdown with work queued.  The run must end cleanly with
no sanitizer report.  LLVM's sanitizer runtime is used (ROCm's clang): the
one of the system gcc does not intercept the clock-based condition-variable
wait of the scheduler's idle loop and reports lock/unlock pairs it cannot
see as races.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
LIBDIR = os.path.join(ROOT, "paper_2604_16590_amd")


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not installed")
def test_scheduler_is_race_free_under_thread_sanitizer(tmp_path):
    exe = str(tmp_path / "serve_tsan")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "serve_tsan_driver.cpp"),
           os.path.join(LIBDIR, "csrc", "la_serve.cpp"),
           "-o", exe, "-L" + LIBDIR, "-llinattn", "-llagen", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + LIBDIR, "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert r.returncode == 0 and "serve tsan driver: ok" in r.stdout
