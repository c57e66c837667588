"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
every evaluator, on small square, rectangular, transposed and padded
shapes with one and several threads, must run clean and agree."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_address_and_ub_sanitizers():
    cc = shutil.which(os.environ.get("CC", "gcc"))
    if cc is None:
        pytest.skip("no host C compiler")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "driver")
    cmd = [cc, "-O1", "-g", "-std=gnu11", "-pthread", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in (r.stderr or ""):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert run.returncode == 0, (run.stdout[-1000:], run.stderr[-3000:])
    assert "all evaluators agree" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    shutil.rmtree(d, ignore_errors=True)
