"""Host AddressSanitizer / UndefinedBehaviorSanitizer build of the C oracle.

oracle/sanitize_check.c runs every oracle routine on small inputs held in
exactly sized heap buffers and checks the tiers against each other; here it is
compiled with gcc together with oracle/jk_oracle.c under
-fsanitize=address,undefined (host code only, serial: no OpenMP) and run.  An
out-of-bounds access, a use after free, a leak or undefined behaviour aborts
it; a disagreement between the tiers makes it exit non-zero.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-std=c11", "-Wall",
           os.path.join(ROOT, "oracle", "jk_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_check.c"),
           "-lm", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("another preloaded library comes before the sanitizer runtime")
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok"), run.stdout
