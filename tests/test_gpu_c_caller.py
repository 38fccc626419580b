"""A C99 program (tests/c_abi_gpu.c) drives GPU solves through the C ABI with no Python and no
torch in its process: eik_solve, eik_solve_ex in the mixed mode, eik_solve_batch and a server.
It checks what eq. (2) fixes for a constant-speed point source (axis values q + d h bit for bit,
the two- and three-term roots next to the exit, a vanishing residual everywhere).

The HIP runtime grants cooperative launches to one process per device at a time.  The test
process solves first (so it holds the device's cooperative launch while the program runs): the
program's solves are then refused the cooperative launch and take the host-driven round loop
(EIK_SCHED_AUTO), and must still pass every check."""
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
    import numpy as np
    import torch
    from paper_1306_4743_amd import eik
    exe = build_c_caller(tmp_path)
    # A solve in this process first, whatever ran before.
    eik.load()
    F = torch.ones((17, 17, 17), dtype=torch.float32, device="cuda:0")
    eik.solve(F, 1 / 16, np.array([[8, 8, 8]]), np.zeros(1), cell=8)
    assert eik.status()[0] == 0
    print(f"running {exe}", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=100)
    print(out.stdout, out.stderr, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
    assert out.stdout.count("0 failed checks") == 7
