"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's planner and parameter validation (csrc/plan.cpp, plain C++)
and the FP64 oracle (oracle/oracle.c), each driven by a randomised fuzzer
under tests/sanitize/ and built here with g++ / gcc.  Any sanitizer report
aborts the fuzzer (-fno-sanitize-recover=all), so a clean exit is the check."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(tool):
    return shutil.which(tool) is not None


@pytest.mark.skipif(not _have("g++"), reason="no g++")
def test_planner_and_validation_under_sanitizers(tmp_path):
    exe = tmp_path / "host_fuzz"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_1609_03782_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sanitize", "host_fuzz.cpp"),
                           os.path.join(ROOT, "paper_1609_03782_amd", "csrc", "plan.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    for seed in (1, 2, 3):
        r = subprocess.run([str(exe), str(seed), "1500"], capture_output=True, text=True, env=env, timeout=300)
        print(r.stdout.strip())
        assert r.returncode == 0, r.stderr[-4000:]


@pytest.mark.skipif(not _have("gcc"), reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_fuzz"
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-ffp-contract=off",
                           os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    for seed in (1, 2):
        r = subprocess.run([str(exe), str(seed), "400"], capture_output=True, text=True, env=env, timeout=300)
        print(r.stdout.strip())
        assert r.returncode == 0, r.stderr[-4000:]
