"""The serving loop's host-side bookkeeping (csrc/jobboard.hpp: the device-pool arena and the
job board shared by client threads and the scheduler) built on the CPU under the host
sanitizers and driven by the stress programs in tests/host/: ThreadSanitizer for the job board
(submitters, scheduler, pollers and a canceller racing), AddressSanitizer with UBSan for both.
The same headers are what the server compiles."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
# clang's sanitizer runtimes (GCC 11's ThreadSanitizer reports false races on this glibc)
CXX = next((c for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")) if c and os.path.exists(c)), None)

CASES = [
    ("arena_stress", "address,undefined"),
    ("jobboard_stress", "address,undefined"),
    ("jobboard_stress", "thread"),
]


@pytest.mark.skipif(CXX is None, reason="no clang++ with sanitizer runtimes")
@pytest.mark.parametrize("prog,san", CASES, ids=[f"{p}-{s.split(',')[0]}" for p, s in CASES])
def test_host_bookkeeping_under_sanitizer(tmp_path, prog, san):
    exe = str(tmp_path / f"{prog}_{san.split(',')[0]}")
    build = subprocess.run([CXX, "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-sanitize-recover=all",
                            os.path.join(HERE, "host", prog + ".cpp"), "-o", exe, "-lpthread"],
                           capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert "ok" in run.stdout
    assert "WARNING" not in run.stderr and "runtime error" not in run.stderr, run.stderr[-6000:]
