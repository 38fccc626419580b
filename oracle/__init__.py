"""Serial FP64 reference for the discrete Eikonal system -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It wraps ``liboracle.so`` (plain C built from ``oracle.c`` with gcc) and adds the
numpy checks that pin it.  It shares no code with the GPU solver in ``paper_1306_4743_amd``.

What it computes (Chacon & Vladimirsky, "A parallel Heap-Cell Method for Eikonal equations"):

* ``fmm``       -- Fast Marching Method (Section 2, FMM paragraph), the exact solution of the
                   first-order upwind system, eq. (2) of Section 1.1, up to rounding.
* ``jacobi``    -- brute-force Jacobi iteration of the same system to an exact fixed point
                   (Section 1.1: iterate temporary labels until they stop changing).
* ``residual``  -- eq. (2) written out per node (C, for large grids); ``residual_numpy`` is the
                   same definition vectorised in numpy and pins the C version.
* ``gamma``     -- the per-node solve of eq. (2) given the three upwind axis values.

Every function here is pinned by ``tests/test_oracle_pins.py`` against closed forms, the
1D reduction, brute force and invariants (see that file's docstrings for the passages).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (plain IEEE doubles, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, dbl, p = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_fmm.argtypes = [i64, i64, i64, dbl, p, i64, p, p, p]
    lib.oracle_fmm.restype = ctypes.c_int
    lib.oracle_fmm_progress.argtypes = [i64, i64, i64, dbl, p, i64, p, p, p, i64]
    lib.oracle_fmm_progress.restype = ctypes.c_int
    lib.oracle_fmm_planted.argtypes = [i64, i64, i64, dbl, p, i64, p, p, p, ctypes.c_int]
    lib.oracle_fmm_planted.restype = ctypes.c_int
    lib.oracle_jacobi.argtypes = [i64, i64, i64, dbl, p, i64, p, p, i64, p]
    lib.oracle_jacobi.restype = i64
    lib.oracle_residual.argtypes = [i64, i64, i64, dbl, p, i64, p, p, dbl,
                                    ctypes.POINTER(i64)]
    lib.oracle_residual.restype = dbl
    lib.oracle_gamma.argtypes = [dbl, dbl, dbl, dbl]
    lib.oracle_gamma.restype = dbl
    _lib = lib
    return lib


def _prep(F, idx3, q):
    F = np.ascontiguousarray(F, dtype=np.float64)  # FP32 speeds widen exactly
    if F.ndim != 3:
        raise ValueError("F must be a 3-D array indexed [k][j][i] (z, y, x)")
    idx3 = np.ascontiguousarray(np.asarray(idx3, dtype=np.int64).reshape(-1, 3))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
    if q.shape[0] != idx3.shape[0]:
        raise ValueError("one q value per source node")
    nz, ny, nx = F.shape
    return F, idx3, q, nx, ny, nz


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def fmm(F, h, idx3, q, progress: int = 0) -> np.ndarray:
    """Serial FP64 FMM; returns U with the shape of F ([nz][ny][nx]).  With progress > 0 a line
    goes to stderr after every `progress` accepted nodes (same arithmetic)."""
    lib = _load()
    F, idx3, q, nx, ny, nz = _prep(F, idx3, q)
    u = np.empty_like(F)
    if progress > 0:
        rc = lib.oracle_fmm_progress(nx, ny, nz, float(h), _ptr(F), idx3.shape[0], _ptr(idx3),
                                     _ptr(q), _ptr(u), int(progress))
    else:
        rc = lib.oracle_fmm(nx, ny, nz, float(h), _ptr(F), idx3.shape[0], _ptr(idx3), _ptr(q),
                            _ptr(u))
    if rc != 0:
        raise ValueError(f"oracle_fmm rejected the input (code {rc})")
    return u


def fmm_planted(F, h, idx3, q, variant: int) -> np.ndarray:
    """FMM with a deliberately wrong local solve (tests of the pins only)."""
    lib = _load()
    F, idx3, q, nx, ny, nz = _prep(F, idx3, q)
    u = np.empty_like(F)
    rc = lib.oracle_fmm_planted(nx, ny, nz, float(h), _ptr(F), idx3.shape[0], _ptr(idx3),
                                _ptr(q), _ptr(u), int(variant))
    if rc != 0:
        raise ValueError(f"oracle_fmm_planted rejected the input (code {rc})")
    return u


def jacobi(F, h, idx3, q, max_sweeps: int = 100000):
    """Brute-force Jacobi to an exact fixed point; returns (V, sweeps)."""
    lib = _load()
    F, idx3, q, nx, ny, nz = _prep(F, idx3, q)
    v = np.empty_like(F)
    n = lib.oracle_jacobi(nx, ny, nz, float(h), _ptr(F), idx3.shape[0], _ptr(idx3), _ptr(q),
                          int(max_sweeps), _ptr(v))
    if n < 0:
        raise ValueError(f"oracle_jacobi failed (code {n})")
    return v, int(n)


def residual(F, h, idx3, q_unused, U, bad_tol: float = 1e-12):
    """Max scaled residual of eq. (2) over non-source nodes (C); returns (rho_max, n_bad)."""
    lib = _load()
    F, idx3, _, nx, ny, nz = _prep(F, idx3, np.zeros(len(np.asarray(idx3).reshape(-1, 3))))
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.shape != F.shape:
        raise ValueError("U and F must have the same shape")
    nbad = ctypes.c_int64(0)
    r = lib.oracle_residual(nx, ny, nz, float(h), _ptr(F), idx3.shape[0], _ptr(idx3), _ptr(U),
                            float(bad_tol), ctypes.byref(nbad))
    return float(r), int(nbad.value)


def gamma(m0: float, m1: float, m2: float, s: float) -> float:
    """Per-node solve of eq. (2): smallest U with sum_k max(U - m_k, 0)^2 = s^2."""
    return float(_load().oracle_gamma(float(m0), float(m1), float(m2), float(s)))


def upwind_minima(U: np.ndarray):
    """The smaller axis neighbour along x, y, z at every node (+inf beyond the grid)."""
    out = []
    for axis in (2, 1, 0):  # x, y, z in [k][j][i] storage
        lo = np.full_like(U, np.inf)
        hi = np.full_like(U, np.inf)
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[axis] = slice(1, None)
        sl_src[axis] = slice(None, -1)
        lo[tuple(sl_dst)] = U[tuple(sl_src)]
        sl_dst[axis] = slice(None, -1)
        sl_src[axis] = slice(1, None)
        hi[tuple(sl_dst)] = U[tuple(sl_src)]
        out.append(np.minimum(lo, hi))
    return out


def residual_numpy(F, h, idx3, U):
    """Eq. (2) per node, vectorised: rho = |sum_k max(U-m_k,0)^2 - s^2| / (s * max(U, s)).

    Returns an array of rho with sources set to 0 (their values are checked against q
    separately).  Nodes with U=+inf get rho=+inf unless every neighbour is +inf."""
    U = np.asarray(U, dtype=np.float64)
    s = h / np.asarray(F, dtype=np.float64)
    ms = upwind_minima(U)
    finite = np.isfinite(U)
    with np.errstate(invalid="ignore"):
        tot = np.zeros_like(U)
        for m in ms:
            d = U - m
            tot += np.where(finite & (d > 0), d * d, 0.0)
        rho = np.abs(tot - s * s) / (s * np.maximum(np.where(finite, U, 0.0), s))
    isolated = np.isinf(ms[0]) & np.isinf(ms[1]) & np.isinf(ms[2])
    rho = np.where(finite, rho, np.where(isolated, 0.0, np.inf))
    idx3 = np.asarray(idx3, dtype=np.int64).reshape(-1, 3)
    rho[idx3[:, 2], idx3[:, 1], idx3[:, 0]] = 0.0
    return rho
