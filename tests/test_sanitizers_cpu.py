"""The FP64 oracle under the host AddressSanitizer and UndefinedBehaviorSanitizer.

`sanitize_oracle_driver.c` calls every oracle entry point (partition,
negatives, evaluation negatives, walks, epochs of all five force models with
and without the bf16 emulation, walk mode, batch slices with injected
negatives, the loss) on graphs with an isolated vertex, self-loops and
duplicate entries, a star, n = 1 and dead ends, with b = 1, b > n and s = 0.
Built with gcc, -fsanitize=address,undefined and no recovery, any invalid
access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-fast-math", "-ffp-contract=off",
           "-o", exe, os.path.join(HERE, "sanitize_oracle_driver.c"), os.path.join(ROOT, "oracle", "f2v_oracle.c"),
           "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
