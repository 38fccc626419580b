"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc), driven from
C over 40 seeded random grids (tests/oracle_sanitized.c): no memory error, undefined behaviour
or leak, and every FMM result equals brute-force Jacobi and satisfies eq. (2)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-w",
           os.path.join(ROOT, "tests", "oracle_sanitized.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-lm", "-o", exe]
    built = subprocess.run(cmd, capture_output=True, text=True)
    if built.returncode != 0 and "asan" in (built.stderr or "").lower():
        pytest.skip("the sanitizer runtimes are not installed")
    assert built.returncode == 0, built.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 bad cases" in out.stdout
