"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a driver (oracle/sanitize_driver.c) runs
every step of the oracle on a small scene, built in both precisions with the sanitizers and -fno-sanitize-recover,
so any out-of-bounds access, use after free, leak or undefined operation ends it with a report; it also checks
that the tiled compositor equals the brute-force one bit for bit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.mark.parametrize("real", ["float", "double"])
def test_oracle_runs_clean_under_sanitizers(tmp_path, real):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / f"orc_san_{real}")
    cmd = [cc, "-O1", "-g", *SAN, "-ffp-contract=off", f"-DREAL={real}",
           os.path.join(ROOT, "oracle", "lodge_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c"),
           "-lm", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr + b.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok:"), (r.returncode, r.stdout, r.stderr[-2000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
