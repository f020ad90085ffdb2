"""The CPU oracle built with AddressSanitizer + UndefinedBehaviorSanitizer and
with ThreadSanitizer (host code only; gcc), driven by
tests/oracle_sanitize_driver.c through every entry point: pre-pass, iteration
matrix, alias tables, walks with 1 and 8 threads, FP32 mode, top-k, M filter,
per-row chains, pilot variance, features, apply. Any sanitizer report fails."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(HERE, "..", "oracle", "mcmi_oracle.c")
DRIVER_C = os.path.join(HERE, "oracle_sanitize_driver.c")


@pytest.mark.parametrize("san", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                 ["-fsanitize=thread"]], ids=["asan_ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, san):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "driver")
    cmd = [gcc, "-O1", "-g", "-std=gnu11", "-pthread", "-ffp-contract=off", "-fno-omit-frame-pointer",
           *san, "-o", exe, DRIVER_C, ORACLE_C, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               TSAN_OPTIONS="halt_on_error=1:exitcode=25")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle sanitize driver ok" in r.stdout
