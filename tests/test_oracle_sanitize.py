"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a host
program (tests/oracle_sanitize_driver.c, which includes the oracle source)
is built with gcc and -fsanitize=address,undefined and runs every oracle
entry point on small seeded inputs; any invalid access, leak-free or not,
or undefined behaviour fails the run.  Host code only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        src = os.path.join(HERE, "oracle_sanitize_driver.c")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
               "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", src, "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
        assert "oracle sanitize run ok" in r.stdout
