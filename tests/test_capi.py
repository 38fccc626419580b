"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol that
include/eik.h declares, and rejects invalid arguments synchronously before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1306_4743_amd import eik

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "eik.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eik_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    assert _declared_symbols() == sorted(eik.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = eik.load()
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {eik.LIB_PATH}").read()
    for name in _declared_symbols():
        assert re.search(rf"\bT {name}\b", out), name


def test_min_store_build_exports_the_same_abi():
    """libeik_minstore.so (the race-check build: write-backs through an atomic minimum) exports
    every declared symbol, and the binding can route its calls there and back."""
    out = os.popen(f"nm -D --defined-only {eik.MINSTORE_LIB_PATH}").read()
    for name in _declared_symbols():
        assert re.search(rf"\bT {name}\b", out), name
    base = eik.load()
    with eik.library(eik.MINSTORE_LIB_PATH) as other:
        assert eik.load() is other and other is not base
        assert eik.strerror(0) == "EIK_OK"
    assert eik.load() is base


def test_strerror_and_version():
    assert eik.strerror(0) == "EIK_OK"
    for code in (-1, -2, -3, -4, -5):
        assert eik.strerror(code).startswith("EIK_E")
    assert "gfx950" in eik.version()


def test_query_workspace_sizes():
    b8 = eik.query_workspace((513, 513, 513), 8, eik.EIK_F32)
    ncell = 65 ** 3
    # values + FP32 speeds + six face layers, at least
    assert b8 >= ncell * 512 * (8 + 4) + ncell * 384 * 8
    assert b8 < ncell * 512 * 30
    b4 = eik.query_workspace((65, 65, 65), 4, eik.EIK_F64)
    assert b4 > 0
    with pytest.raises(eik.EikError):
        eik.query_workspace((65, 65, 65), 5, eik.EIK_F64)
    with pytest.raises(eik.EikError):
        eik.query_workspace((1, 65, 65), 8, eik.EIK_F64)


def _call(dims, h=0.1, F=1, f_dtype=0, n=1, idx=None, q=None, u=1, cell=8, tol=0.0):
    lib = eik.load()
    idx = np.array([[0, 0, 0]] * max(n, 1), dtype=np.int64) if idx is None else idx
    q = np.zeros(max(n, 1)) if q is None else q
    src = eik.Sources(n, idx.ctypes.data, q.ctypes.data, 0)
    d = (ctypes.c_int64 * 3)(*dims)
    return lib.eik_solve(ctypes.cast(d, ctypes.c_void_p), h, ctypes.c_void_p(F), f_dtype,
                         ctypes.byref(src), ctypes.c_void_p(u), cell, tol, None)


@pytest.mark.parametrize("kw", [
    dict(dims=(1, 8, 8)), dict(dims=(8, 8, 8), h=0.0), dict(dims=(8, 8, 8), h=float("nan")),
    dict(dims=(8, 8, 8), F=0), dict(dims=(8, 8, 8), u=0), dict(dims=(8, 8, 8), f_dtype=7),
    dict(dims=(8, 8, 8), cell=5), dict(dims=(8, 8, 8), cell=2), dict(dims=(8, 8, 8), tol=-1.0),
    dict(dims=(8, 8, 8), n=-1),
    dict(dims=(8, 8, 8), idx=np.array([[8, 0, 0]], dtype=np.int64)),
    dict(dims=(8, 8, 8), idx=np.array([[0, -1, 0]], dtype=np.int64)),
    dict(dims=(8, 8, 8), q=np.array([-1.0])), dict(dims=(8, 8, 8), q=np.array([np.inf])),
    dict(dims=(8, 8, 8), q=np.array([np.nan])),
    dict(dims=(2048, 2048, 1024)),
])
def test_invalid_arguments_rejected_synchronously(kw):
    """Each of these is refused with EIK_EINVAL before any device work (F and u_out are fake
    non-null pointers that are never dereferenced)."""
    assert _call(**kw) == eik.EIK_EINVAL


def test_stream_status_without_solve():
    lib = eik.load()
    st = eik.Stats()
    # a stream handle that never had a solve: no workspace -> EIK_EINVAL, no device access
    assert lib.eik_stream_status(ctypes.c_void_p(0x1234), ctypes.byref(st)) in (eik.EIK_EINVAL,
                                                                                  eik.EIK_EHIP)


def test_strerror_busy():
    assert eik.strerror(eik.EIK_EBUSY).startswith("EIK_EBUSY")


def test_problem_bytes():
    """A grid's pool footprint: cell-blocked values (8 B), speeds (F dtype) and six face layers
    per cell, each array rounded up to 256 B; it is the grid part of the workspace size."""
    ncell = 9 ** 3  # 65 nodes per axis -> 9 cells of 8
    want = sum(-(-b // 256) * 256 for b in (ncell * 512 * 8, ncell * 512 * 4, ncell * 384 * 8))
    assert eik.problem_bytes((65, 65, 65), 8, eik.EIK_F32) == want
    assert eik.query_workspace((65, 65, 65), 8, eik.EIK_F32) > want
    with pytest.raises(eik.EikError):
        eik.problem_bytes((65, 65, 65), 6, eik.EIK_F32)
    with pytest.raises(eik.EikError):
        eik.problem_bytes((65, 65, 65), 8, 3)


def test_problem_bytes_cell_16():
    """Cells of 16: 65 nodes per axis -> 5 cells (the last holds one node layer), 4096 nodes and
    six faces of 256 per cell."""
    ncell = 5 ** 3
    want = sum(-(-b // 256) * 256 for b in (ncell * 4096 * 8, ncell * 4096 * 4, ncell * 1536 * 8))
    assert eik.problem_bytes((65, 65, 65), 16, eik.EIK_F32) == want
    # the node limit applies to the grid rounded up to whole cells: 1280 = 80 * 16 fits, 1290
    # rounds up to 1296^3 > 2^31
    assert eik.query_workspace((1280, 1280, 1280), 16, eik.EIK_F32) > 0
    with pytest.raises(eik.EikError):
        eik.query_workspace((1290, 1290, 1290), 16, eik.EIK_F32)


def test_two_sweep_streams_refused_at_cell_16():
    """EIK_INNER_DUAL needs both streams' planes in one wave, which holds up to r = 8 only: a
    solve, a batch and a server asking for it at r = 16 are refused before any device work."""
    lib = eik.load()
    d = (ctypes.c_int64 * 3)(17, 17, 17)
    idx = np.zeros((1, 3), dtype=np.int64)
    q = np.zeros(1)
    src = eik.Sources(1, idx.ctypes.data, q.ctypes.data, 0)
    opts = eik._options(inner=eik.EIK_INNER_DUAL)
    assert lib.eik_solve_ex(ctypes.cast(d, ctypes.c_void_p), 0.1, ctypes.c_void_p(1), 0,
                            ctypes.byref(src), ctypes.c_void_p(1), 16, 0.0, None,
                            ctypes.byref(opts)) == eik.EIK_EINVAL
    good, keep = _problem()
    arr = (eik.Problem * 1)(good)
    assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 16, None, ctypes.byref(opts)) == eik.EIK_EINVAL
    srv = ctypes.c_void_p()
    assert lib.eik_server_create(ctypes.byref(srv), 1 << 20, 1000, 4, 16, eik.EIK_F32, None,
                                 ctypes.byref(opts)) == eik.EIK_EINVAL


def _problem(dims=(8, 8, 8), h=0.1, F=1, u=1, n=1, idx=None, q=None, tol=0.0):
    idx = np.array([[0, 0, 0]] * max(n, 1), dtype=np.int64) if idx is None else idx
    q = np.zeros(max(n, 1)) if q is None else q
    src = eik.Sources(n, idx.ctypes.data, q.ctypes.data, 0)
    pb = eik.Problem((ctypes.c_int64 * 3)(*dims), h, F, src, u, tol)
    return pb, (idx, q)


@pytest.mark.parametrize("bad", [
    dict(dims=(1, 8, 8)), dict(h=-1.0), dict(F=0), dict(u=0), dict(tol=float("inf")),
    dict(idx=np.array([[0, 0, 9]], dtype=np.int64)), dict(q=np.array([np.nan])),
])
def test_batch_with_one_invalid_problem_rejected(bad):
    """eik_solve_batch validates every problem first: one invalid problem refuses the batch."""
    lib = eik.load()
    good, k1 = _problem()
    badp, k2 = _problem(**bad)
    arr = (eik.Problem * 3)(good, badp, good)
    opts = eik._options()
    assert lib.eik_solve_batch(3, arr, eik.EIK_F32, 8, None, ctypes.byref(opts)) == eik.EIK_EINVAL


def test_problem_struct_layout():
    """The binding's eik_problem matches the C layout: u_approx follows tol at offset 88."""
    assert eik.Problem.u_approx.offset == 88 and ctypes.sizeof(eik.Problem) == 96


def test_options_struct_layout():
    """The binding's eik_options matches the C layout (88 bytes, schedule at 72, jitter last at
    80; the C side is checked in tests/c_abi_smoke.c)."""
    assert eik.Options.schedule.offset == 72 and eik.Options.jitter.offset == 80
    assert ctypes.sizeof(eik.Options) == 88


def test_schedule_option_checked():
    lib = eik.load()
    pb, keep = _problem()
    arr = (eik.Problem * 1)(pb)
    for bad in (-1, 4):
        opts = eik._options(schedule=bad)
        assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 8, None,
                                   ctypes.byref(opts)) == eik.EIK_EINVAL


def test_polish_not_allowed_with_mixed_mode():
    """A problem carrying an approximation cannot use EIK_MODE_MIXED (refused before any
    device work)."""
    lib = eik.load()
    pb, keep = _problem()
    pb.u_approx = 0x1000
    arr = (eik.Problem * 1)(pb)
    opts = eik._options(mode=eik.EIK_MODE_MIXED)
    assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 8, None, ctypes.byref(opts)) == eik.EIK_EINVAL


def test_batch_argument_checks():
    lib = eik.load()
    good, keep = _problem()
    arr = (eik.Problem * 1)(good)
    assert lib.eik_solve_batch(0, arr, eik.EIK_F32, 8, None, None) == eik.EIK_EINVAL
    assert lib.eik_solve_batch(-2, arr, eik.EIK_F32, 8, None, None) == eik.EIK_EINVAL
    assert lib.eik_solve_batch(1, None, eik.EIK_F32, 8, None, None) == eik.EIK_EINVAL
    assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 6, None, None) == eik.EIK_EINVAL
    assert lib.eik_solve_batch(1, arr, 9, 8, None, None) == eik.EIK_EINVAL
    bad_opt = eik._options(inner=9)
    assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 8, None, ctypes.byref(bad_opt)) == eik.EIK_EINVAL
    assert lib.eik_batch_status(ctypes.c_void_p(0x4321), 1,
                                np.zeros(1, np.int32).ctypes.data) in (eik.EIK_EINVAL, eik.EIK_EHIP)


@pytest.mark.parametrize("args", [
    (0, 100, 4, 8, eik.EIK_F32), (1 << 20, 0, 4, 8, eik.EIK_F32),
    (1 << 20, 100, 0, 8, eik.EIK_F32), (1 << 20, 100, 4, 5, eik.EIK_F32),
    (1 << 20, 100, 4, 8, 4), (1 << 20, 1 << 31, 4, 8, eik.EIK_F32),
])
def test_server_create_rejects_invalid(args):
    lib = eik.load()
    h = ctypes.c_void_p(None)
    rc = lib.eik_server_create(ctypes.byref(h), args[0], args[1], args[2], args[3], args[4], None,
                               None)
    assert rc == eik.EIK_EINVAL and not h.value


def test_server_calls_reject_null_server():
    lib = eik.load()
    t = ctypes.c_int64(0)
    fin = ctypes.c_int(0)
    pb, keep = _problem()
    n = ctypes.c_int(0)
    assert lib.eik_server_submit(None, ctypes.byref(pb), ctypes.byref(t)) == eik.EIK_EINVAL
    assert lib.eik_server_step(None, 4, ctypes.byref(fin)) == eik.EIK_EINVAL
    assert lib.eik_server_poll(None, 0, None, None, ctypes.byref(n)) == eik.EIK_EINVAL
    assert lib.eik_server_load(None, None, None, None) == eik.EIK_EINVAL
    assert lib.eik_server_destroy(None) == eik.EIK_EINVAL


def test_autotune_rejects_invalid():
    lib = eik.load()
    idx = np.zeros((1, 3), dtype=np.int64)
    q = np.zeros(1)
    src = eik.Sources(1, idx.ctypes.data, q.ctypes.data, 0)
    best = eik.TuneEntry()
    n = ctypes.c_int(0)
    table = (eik.TuneEntry * 4)()
    d = (ctypes.c_int64 * 3)(8, 8, 8)
    dp = ctypes.cast(d, ctypes.c_void_p)
    call = lambda **k: lib.eik_autotune(
        k.get("dims", dp), k.get("h", 0.1), ctypes.c_void_p(k.get("F", 1)), 0, ctypes.byref(src),
        ctypes.c_void_p(1), 0.0, None, k.get("reps", 1), k.get("table", table), k.get("cap", 4),
        ctypes.byref(n), k.get("best", ctypes.byref(best)))
    assert call(reps=0) == eik.EIK_EINVAL
    assert call(reps=101) == eik.EIK_EINVAL
    assert call(best=None) == eik.EIK_EINVAL
    assert call(table=None, cap=3) == eik.EIK_EINVAL
    assert call(h=-1.0) == eik.EIK_EINVAL
    assert call(F=0) == eik.EIK_EINVAL
    assert call(dims=None) == eik.EIK_EINVAL


def test_mode_sizes_and_server_mode():
    """FP32 mode halves the value and face arrays; mixed keeps both; servers take one precision."""
    d = (65, 65, 65)
    b64 = eik.problem_bytes(d, 8, eik.EIK_F32, eik.EIK_MODE_FP64)
    b32 = eik.problem_bytes(d, 8, eik.EIK_F32, eik.EIK_MODE_FP32)
    bmx = eik.problem_bytes(d, 8, eik.EIK_F32, eik.EIK_MODE_MIXED)
    ncell = 9 ** 3
    assert b64 - b32 == ncell * (512 + 384) * 4
    assert bmx - b64 == ncell * (512 + 384) * 4
    with pytest.raises(eik.EikError):
        eik.problem_bytes(d, 8, eik.EIK_F32, 3)
    lib = eik.load()
    h = ctypes.c_void_p(None)
    opts = eik._options(mode=eik.EIK_MODE_MIXED)
    assert lib.eik_server_create(ctypes.byref(h), 1 << 20, 100, 4, 8, eik.EIK_F32, None,
                                 ctypes.byref(opts)) == eik.EIK_EINVAL


def test_cell_value_option_checked():
    lib = eik.load()
    pb, keep = _problem()
    arr = (eik.Problem * 1)(pb)
    bad = eik._options(cell_value=2)
    assert lib.eik_solve_batch(1, arr, eik.EIK_F32, 8, None, ctypes.byref(bad)) == eik.EIK_EINVAL


def test_size_limits():
    """Grids are limited to fewer than 2^31 nodes, also after rounding up to whole cells
    (32-bit node and cell-node indices); the limit is checked before any allocation."""
    assert eik.query_workspace((1280, 1280, 1280), 8, eik.EIK_F32) > 0       # 160^3 cells
    with pytest.raises(eik.EikError):                                      # 2.1467e9 nodes, but
        eik.query_workspace((1290, 1290, 1290), 8, eik.EIK_F32)            # 162^3 cells of 512
    with pytest.raises(eik.EikError):
        eik.query_workspace((1291, 1291, 1291), 8, eik.EIK_F32)            # >= 2^31 nodes
    with pytest.raises(eik.EikError):
        eik.query_workspace((1 << 16, 1 << 16, 2), 8, eik.EIK_F32)
    # two nodes per side is the smallest grid
    assert eik.query_workspace((2, 2, 2), 4, eik.EIK_F64) > 0


def test_probe_library_exports():
    """libeik_probe.so (bandwidth probes) exports what include/eik_probe.h declares and rejects
    invalid arguments before touching a device."""
    from paper_1306_4743_amd import probes
    lib = probes.load()
    hdr = open(os.path.join(ROOT, "include", "eik_probe.h")).read()
    declared = set(re.findall(r"^int (eikp_\w+)\(", hdr, re.M))
    assert declared == set(probes.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)
    ms, nb = ctypes.c_float(0), ctypes.c_double(0)
    assert lib.eikp_copy(None, None, 16, 1, None, ctypes.byref(ms)) == -1
    assert lib.eikp_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1008), 16, 1, None,
                         ctypes.byref(ms)) == -1  # overlap / misaligned
    assert lib.eikp_lds(0, 8, 0, 1, ctypes.c_void_p(0x1000), None, ctypes.byref(ms),
                        ctypes.byref(nb)) == -1
    assert lib.eikp_lds(1, 8, 2, 1, ctypes.c_void_p(0x1000), None, ctypes.byref(ms),
                        ctypes.byref(nb)) == -1


def test_headers_are_a_c_abi(tmp_path):
    """include/eik.h and include/eik_probe.h compile as C99 (gcc, not a C++ compiler) and a C
    program links against both libraries and calls their host-side entry points."""
    import shutil
    import subprocess
    from paper_1306_4743_amd import probes
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    libdir = os.path.dirname(eik.LIB_PATH)
    assert os.path.exists(eik.LIB_PATH) and os.path.exists(probes.LIB_PATH)
    exe = tmp_path / "c_abi_smoke"
    cmd = [gcc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "c_abi_smoke.c"), f"-L{libdir}", "-leik", "-leik_probe",
           f"-Wl,-rpath,{libdir}", "-o", str(exe)]
    subprocess.run(cmd, check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libeik.so the binding raises on load and on every solve: there is no CPU
    fallback that could stand in for the HIP path."""
    import numpy as np
    monkeypatch.setattr(eik, "LIB_PATH", str(tmp_path / "libeik.so"))
    monkeypatch.setattr(eik, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        eik.load()
    import torch
    F = torch.ones((4, 4, 4), dtype=torch.float64)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        eik.solve(F, 0.25, np.zeros((1, 3), np.int64), np.zeros(1), cell=8)


def test_noalloc_limits_checked_on_the_host():
    """eik_solve_noalloc refuses, before any device call, a problem whose workspace exceeds the
    static scratch (EIK_ETOOBIG), more host-side exits than a kernel argument carries, and
    timing (which would create events)."""
    lib = eik.load()
    idx = np.array([[1, 2, 3]], dtype=np.int64)
    q = np.zeros(1)
    src = eik.Sources(1, idx.ctypes.data, q.ctypes.data, 0)
    dims = (ctypes.c_int64 * 3)(300, 300, 300)
    opts = eik._options()
    assert lib.eik_solve_noalloc(ctypes.cast(dims, ctypes.c_void_p), 1 / 299, ctypes.c_void_p(16),
                                 eik.EIK_F32, ctypes.byref(src), ctypes.c_void_p(16), 8, 0.0, None,
                                 ctypes.byref(opts)) == eik.EIK_ETOOBIG
    dims = (ctypes.c_int64 * 3)(40, 40, 40)
    many = np.array([[i, i, i] for i in range(33)], dtype=np.int64)
    qs = np.zeros(33)
    src33 = eik.Sources(33, many.ctypes.data, qs.ctypes.data, 0)
    assert lib.eik_solve_noalloc(ctypes.cast(dims, ctypes.c_void_p), 1 / 39, ctypes.c_void_p(16),
                                 eik.EIK_F32, ctypes.byref(src33), ctypes.c_void_p(16), 8, 0.0,
                                 None, ctypes.byref(opts)) == eik.EIK_EINVAL
    timed = eik._options(timing=True)
    assert lib.eik_solve_noalloc(ctypes.cast(dims, ctypes.c_void_p), 1 / 39, ctypes.c_void_p(16),
                                 eik.EIK_F32, ctypes.byref(src), ctypes.c_void_p(16), 8, 0.0, None,
                                 ctypes.byref(timed)) == eik.EIK_EINVAL
    assert "384 MiB" in eik.strerror(eik.EIK_ETOOBIG)

