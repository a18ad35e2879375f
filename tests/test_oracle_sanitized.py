"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A standalone driver (sanitize_oracle.c) runs every oracle routine on random
small graphs, with the equalities the three selection algorithms must meet;
built here with gcc, host code only. Skipped when gcc cannot link the
sanitizer runtimes.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_is_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "sanitize_oracle"
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize_oracle.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "mlp.c"),
           "-o", str(exe), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and ("cannot find" in build.stderr or "libasan" in build.stderr):
        pytest.skip("sanitizer runtimes not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert run.stdout.strip().endswith("ok")
