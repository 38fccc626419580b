"""A C99 program (tests/c_abi_gpu.c) drives GPU solves through the C ABI with no Python and no
torch in its process: eik_solve, eik_solve_ex in the mixed mode, eik_solve_batch and a server.
It checks what eq. (2) fixes for a constant-speed point source (axis values q + d h bit for bit,
the two- and three-term roots next to the exit, a vanishing residual everywhere).

The HIP runtime grants cooperative launches to one process per device at a time: once a
process has launched the solver, another process's launches fail (EIK_EHIP) until it exits.
The program therefore runs before any other GPU test of the session (this file sorts first
among them), while the test process itself has launched nothing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build_c_caller(out_dir):
    """Compile and link tests/c_abi_gpu.c with gcc against libeik.so and the HIP runtime."""
    from paper_1306_4743_amd import eik
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    libdir = os.path.dirname(eik.LIB_PATH)
    assert os.path.exists(eik.LIB_PATH)
    exe = os.path.join(str(out_dir), "c_abi_gpu")
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "c_abi_gpu.c"), f"-L{libdir}", "-leik",
           "-L/opt/rocm/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,{libdir}",
           "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    subprocess.run(cmd, check=True)
    return exe


def test_c_caller_builds(tmp_path):
    """The program compiles as C99 without warnings and links (no GPU needed)."""
    assert os.path.exists(build_c_caller(tmp_path))


@pytest.mark.gpu
def test_c_caller_solves_on_gpu(tmp_path):
    exe = build_c_caller(tmp_path)
    print(f"running {exe}", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=100)
    print(out.stdout, out.stderr, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
    assert out.stdout.count("0 failed checks") == 7
