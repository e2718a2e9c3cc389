"""The CPU code built with AddressSanitizer and UBSan: the oracle through every C entry point
(tests/native/oracle_asan.cpp), and the library's host-side plan logic with the kernel's schedule
arithmetic (tests/native/sched_replay.cpp, driven by test_schedule_replay.py)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["g++", "-std=gnu++17", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "tests", "native", "oracle_asan.cpp"),
                    os.path.join(ROOT, "oracle", "shgo_oracle.cpp"), "-o", exe, "-lquadmath"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout + r.stderr)[-3000:]
