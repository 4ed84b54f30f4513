"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): tests/fzo_sanitize.c drives round trips of every rank and bound
mode, fp64 input, the field-global predictor, escapes up to and past the
per-chunk cap, the error statuses, and decompression of truncated and
corrupted streams; any out-of-bounds access, leak or undefined operation in
oracle/fzo.c aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "fzo_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-I" + os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "fzo_sanitize.c"),
           os.path.join(ROOT, "oracle", "fzo.c"), "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ok: 0 failures" in r.stdout
