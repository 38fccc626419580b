"""The queue protocol of the solve without rounds, as a CPU model under ThreadSanitizer
(tests/ring_protocol_model.cpp): the protocol as built passes (no race report, no lost tag, no
double ownership, termination with all work done), and each planted mistake is caught -- relaxed
ordering of the cell word by the sanitizer, a tag dropped for a running cell by the model's own
checks.  Section 5 of the paper counts active cells and decrements the count only after the
propagation of a cell's changes, so that no worker quits early; the model checks the GPU
restatement of that rule."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "ring_protocol_model.cpp")


def build_and_run(tmp_path, define=None):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path / ("model" + (define or "")))
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-o", exe, SRC, "-lpthread"]
    if define:
        cmd.insert(1, f"-D{define}")
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return out.returncode, out.stdout + out.stderr


def test_protocol_as_built_is_race_free_and_loses_nothing(tmp_path):
    rc, out = build_and_run(tmp_path)
    print(out[-400:])
    assert rc == 0, out[-2000:]
    assert "WARNING: ThreadSanitizer" not in out
    assert " 0 violations" in out


def test_relaxed_cell_word_is_reported_as_a_race(tmp_path):
    rc, out = build_and_run(tmp_path, "PLANT_RELAXED")
    assert rc != 0 and "WARNING: ThreadSanitizer: data race" in out


def test_a_lost_tag_is_detected(tmp_path):
    rc, out = build_and_run(tmp_path, "PLANT_LOST_TAG")
    assert rc != 0
    line = [l for l in out.splitlines() if l.startswith("protocol model:")][-1]
    assert int(line.split()[-2]) > 0
