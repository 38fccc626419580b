"""Python binding of libeik (include/eik.h): argument marshalling only.

Every step of the solve runs in the HIP kernels of ``libeik.so``; this module converts torch
device tensors and numpy source lists into the C ABI's plain pointers and sizes.  It never
computes values itself and has no CPU fallback: if the library is missing it raises.
"""
from __future__ import annotations

import atexit
import contextlib
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeik.so")
# The same solver with every write-back through an atomic minimum (a race check, see library()).
MINSTORE_LIB_PATH = os.path.join(_HERE, "libeik_minstore.so")

EIK_OK, EIK_EINVAL, EIK_ENOMEM, EIK_EHIP, EIK_ENOCONV, EIK_ECANCELLED = 0, -1, -2, -3, -4, -5
EIK_EBUSY = -6
EIK_ETOOBIG = -7
EIK_F64, EIK_F32 = 0, 1
EIK_MODE_FP64, EIK_MODE_FP32, EIK_MODE_MIXED = 0, 1, 2
EIK_INNER_SWEEP, EIK_INNER_LIST, EIK_INNER_DUAL, EIK_INNER_PAIR = 1, 2, 3, 4
EIK_CELL_VALUE_NEW, EIK_CELL_VALUE_OLD = 0, 1
EIK_SCHED_AUTO, EIK_SCHED_COOPERATIVE, EIK_SCHED_HOST_LOOP, EIK_SCHED_ASYNC = 0, 1, 2, 3


class EikError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}{strerror(code)} ({code})")


class Sources(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("idx3", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("on_device", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("delta", ctypes.c_double),
                ("max_rounds", ctypes.c_int64), ("max_sweeps", ctypes.c_int),
                ("workers", ctypes.c_int), ("shuffle", ctypes.c_uint64), ("timing", ctypes.c_int),
                ("round_log", ctypes.c_void_p), ("round_log_len", ctypes.c_int64),
                ("inner", ctypes.c_int), ("cell_value", ctypes.c_int), ("schedule", ctypes.c_int),
                ("jitter", ctypes.c_uint64)]


class Problem(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 3), ("h", ctypes.c_double), ("F", ctypes.c_void_p),
                ("sources", Sources), ("u_out", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("u_approx", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int), ("inner", ctypes.c_int), ("workers", ctypes.c_int),
                ("delta", ctypes.c_double), ("ms", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("rounds", "visits", "sweeps", "updates", "deferred", "requeued", "cells",
                 "status", "workers", "cycles_pop", "cycles_stage", "cycles_sweep",
                 "cycles_write", "cycles_wait")] + [
                ("sweep_hist", ctypes.c_int64 * 32), ("visit_cycles_log2_hist", ctypes.c_int64 * 32),
                ("polish_redone", ctypes.c_int64)]

    def as_dict(self):
        d = {n: int(getattr(self, n)) for n, t in self._fields_ if t is ctypes.c_int64}
        d["sweep_hist"] = [int(v) for v in self.sweep_hist]
        d["visit_cycles_log2_hist"] = [int(v) for v in self.visit_cycles_log2_hist]
        return d


_lib = None

# Every symbol declared in include/eik.h.
EXPORTS = ("eik_solve", "eik_solve_ex", "eik_solve_noalloc", "eik_cancel", "eik_query_workspace", "eik_problem_bytes",
           "eik_stream_status", "eik_kernel_times", "eik_solve_batch", "eik_batch_status",
           "eik_server_create", "eik_server_submit", "eik_server_step", "eik_server_poll",
           "eik_server_load", "eik_server_destroy", "eik_server_polish_redone", "eik_autotune",
           "eik_strerror", "eik_release", "eik_version")


def load():
    """Load libeik.so (built in-tree by __graft_entry__.build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    _lib = _open(LIB_PATH)
    atexit.register(_shutdown)
    return _lib


@contextlib.contextmanager
def library(path: str):
    """Inside the block, every call of this module goes to another build of the same ABI at
    `path` (e.g. MINSTORE_LIB_PATH); the block waits for the device and releases that build's
    workspaces at its end.  Not for use while servers of the default build are running."""
    global _lib
    saved = load()
    other = _open(path)
    _lib = other
    try:
        yield other
    finally:
        try:
            import torch
            if torch.cuda.is_initialized():  # no device work can be pending otherwise
                torch.cuda.synchronize()
        finally:
            other.eik_release()
            _lib = saved


def _open(path: str):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.eik_solve.argtypes = [vp, dbl, vp, i32, ctypes.POINTER(Sources), vp, i32, dbl, vp]
    lib.eik_solve.restype = i32
    lib.eik_solve_ex.argtypes = [vp, dbl, vp, i32, ctypes.POINTER(Sources), vp, i32, dbl, vp,
                                 ctypes.POINTER(Options)]
    lib.eik_solve_ex.restype = i32
    lib.eik_solve_noalloc.argtypes = [vp, dbl, vp, i32, ctypes.POINTER(Sources), vp, i32, dbl,
                                      vp, ctypes.POINTER(Options)]
    lib.eik_solve_noalloc.restype = i32
    lib.eik_query_workspace.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.eik_query_workspace.restype = i32
    lib.eik_stream_status.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.eik_stream_status.restype = i32
    lib.eik_cancel.argtypes = [vp]
    lib.eik_cancel.restype = i32
    lib.eik_kernel_times.argtypes = [vp, i32, vp, vp]
    lib.eik_kernel_times.restype = i32
    lib.eik_strerror.argtypes = [i32]
    lib.eik_strerror.restype = ctypes.c_char_p
    lib.eik_release.argtypes = []
    lib.eik_release.restype = None
    lib.eik_version.argtypes = []
    lib.eik_version.restype = ctypes.c_char_p
    lib.eik_problem_bytes.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.eik_problem_bytes.restype = i32
    lib.eik_solve_batch.argtypes = [i32, ctypes.POINTER(Problem), i32, i32, vp,
                                    ctypes.POINTER(Options)]
    lib.eik_solve_batch.restype = i32
    lib.eik_batch_status.argtypes = [vp, i32, vp]
    lib.eik_batch_status.restype = i32
    lib.eik_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, i64, i32, i32, i32, vp,
                                      ctypes.POINTER(Options)]
    lib.eik_server_create.restype = i32
    lib.eik_server_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(i64)]
    lib.eik_server_submit.restype = i32
    lib.eik_server_step.argtypes = [vp, i64, ctypes.POINTER(i32)]
    lib.eik_server_step.restype = i32
    lib.eik_server_poll.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i32)]
    lib.eik_server_poll.restype = i32
    lib.eik_server_load.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.eik_server_load.restype = i32
    lib.eik_autotune.argtypes = [vp, dbl, vp, i32, ctypes.POINTER(Sources), vp, dbl, vp, i32,
                                 ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32),
                                 ctypes.POINTER(TuneEntry)]
    lib.eik_autotune.restype = i32
    lib.eik_server_destroy.argtypes = [vp]
    lib.eik_server_destroy.restype = i32
    lib.eik_server_polish_redone.argtypes = [vp]
    lib.eik_server_polish_redone.restype = i64
    return lib


# Servers not yet closed; at interpreter exit they are closed and every workspace released
# while the HIP runtime is still fully up, so that no library state (device memory, pinned
# buffers, events) outlives the process's own teardown.
_live_servers = weakref.WeakSet()


def _shutdown():
    if _lib is None:
        return
    for s in list(_live_servers):
        try:
            s.close()
        except Exception:
            pass
    try:
        _lib.eik_release()
    except Exception:
        pass


def strerror(code: int) -> str:
    try:
        return load().eik_strerror(int(code)).decode()
    except RuntimeError:
        return f"code {code}"


def version() -> str:
    return load().eik_version().decode()


def _dims_array(dims):
    return (ctypes.c_int64 * 3)(*[int(d) for d in dims])


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def query_workspace(dims, cell: int = 8, f_dtype: int = EIK_F64, mode: int = EIK_MODE_FP64) -> int:
    out = ctypes.c_size_t(0)
    rc = load().eik_query_workspace(ctypes.cast(_dims_array(dims), ctypes.c_void_p), int(cell),
                                    int(f_dtype), int(mode), ctypes.byref(out))
    if rc != EIK_OK:
        raise EikError(rc, "eik_query_workspace: ")
    return int(out.value)


class _HostSources:
    """Keeps host copies alive for the duration of the (synchronous) staging in eik_solve."""

    def __init__(self, idx3, q):
        self.idx3 = np.ascontiguousarray(np.asarray(idx3, dtype=np.int64).reshape(-1, 3))
        self.q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
        if self.q.shape[0] != self.idx3.shape[0]:
            raise ValueError("one q value per source node")
        self.struct = Sources(self.idx3.shape[0],
                              self.idx3.ctypes.data if self.idx3.size else None,
                              self.q.ctypes.data if self.q.size else None, 0)


def _f_dtype(F):
    import torch
    if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dim() == 3 and F.is_contiguous()):
        raise ValueError("F must be a contiguous 3-D CUDA tensor [nz, ny, nx]")
    if F.dtype == torch.float32:
        return EIK_F32
    if F.dtype == torch.float64:
        return EIK_F64
    raise ValueError("F must be float32 or float64")


def _out_tensor(F, u_out):
    import torch
    if u_out is None:
        return torch.empty(F.shape, dtype=torch.float64, device=F.device)
    if not (u_out.is_cuda and u_out.dtype == torch.float64 and u_out.shape == F.shape
            and u_out.is_contiguous()):
        raise ValueError("u_out must be a contiguous float64 CUDA tensor shaped like F")
    return u_out


def _sources(F, idx3, q, stream):
    """(ctypes Sources, objects to keep alive while the library may read them)."""
    import torch
    if isinstance(idx3, torch.Tensor) and idx3.is_cuda:
        idx3_t = idx3.to(torch.int64).contiguous()
        q_t = torch.as_tensor(q, dtype=torch.float64, device=F.device).contiguous()
        if stream is not None:
            idx3_t.record_stream(stream)
            q_t.record_stream(stream)
        return Sources(idx3_t.shape[0], idx3_t.data_ptr(), q_t.data_ptr(), 1), (idx3_t, q_t)
    keep = _HostSources(idx3, q)
    return keep.struct, keep


def _options(delta=0.0, max_rounds=0, max_sweeps=0, workers=0, shuffle=0, timing=False,
             round_log=None, inner=0, mode=EIK_MODE_FP64, cell_value=EIK_CELL_VALUE_NEW,
             schedule=EIK_SCHED_AUTO, jitter=0):
    rl_ptr, rl_len = None, 0
    if round_log is not None:
        import torch
        if not (round_log.is_cuda and round_log.dtype == torch.int64 and round_log.is_contiguous()):
            raise ValueError("round_log must be a contiguous int64 CUDA tensor")
        rl_ptr, rl_len = round_log.data_ptr(), round_log.numel() // 2
    return Options(int(mode), float(delta), int(max_rounds), int(max_sweeps), int(workers),
                   int(shuffle), int(bool(timing)), rl_ptr, rl_len, int(inner),
                   int(cell_value), int(schedule), int(jitter))


def _approx(F, u_approx):
    """Device address of an approximation to polish (0 for none), checked against F."""
    import torch
    if u_approx is None:
        return 0
    if not (u_approx.is_cuda and u_approx.dtype == torch.float64 and u_approx.shape == F.shape
            and u_approx.is_contiguous()):
        raise ValueError("u_approx must be a contiguous float64 CUDA tensor shaped like F")
    return u_approx.data_ptr()


def _problem(F, h, idx3, q, tol, u_out, stream, u_approx=None):
    """(ctypes Problem, u_out tensor, keep-alive objects) of one grid."""
    _f_dtype(F)
    u_out = _out_tensor(F, u_out)
    src, keep = _sources(F, idx3, q, stream)
    nz, ny, nx = F.shape
    pb = Problem((ctypes.c_int64 * 3)(nx, ny, nz), float(h), F.data_ptr(), src,
                 u_out.data_ptr(), float(tol), _approx(F, u_approx))
    return pb, u_out, (keep, u_approx)


def solve(F, h: float, idx3, q, cell: int = 8, tol: float = 0.0, u_out=None, stream=None,
          delta: float = 0.0, max_rounds: int = 0, max_sweeps: int = 0, workers: int = 0,
          shuffle: int = 0, timing: bool = False, round_log=None, inner: int = 0,
          mode: int = EIK_MODE_FP64, cell_value: int = EIK_CELL_VALUE_NEW,
          check: bool = True, u_approx=None, schedule: int = EIK_SCHED_AUTO, jitter: int = 0):
    """Enqueue one solve of eq. (2) on ``stream`` (torch stream; default: current stream).

    F: torch CUDA tensor [nz, ny, nx] of float32 or float64 speeds (contiguous).
    idx3, q: host arrays of exit nodes (i, j, k) and their values, or torch CUDA tensors
    (int64 [n, 3] and float64 [n]).  Returns u_out (allocated if None), a float64 CUDA tensor
    of F's shape.  The call returns after enqueueing; use ``status()`` to wait and read the
    device-side status and counters.  u_approx (float64 CUDA tensor shaped like F, may be
    u_out): a single-precision-accurate solution to polish to the FP64 one (a one-problem
    ``eik_solve_batch`` with the problem's ``u_approx`` set).
    """
    if u_approx is not None:
        outs = solve_batch([dict(F=F, h=h, src=idx3, q=q, tol=tol, u_out=u_out,
                                 u_approx=u_approx)], cell=cell, stream=stream, check=check,
                           delta=delta, max_rounds=max_rounds, max_sweeps=max_sweeps,
                           workers=workers, shuffle=shuffle, timing=timing, round_log=round_log,
                           inner=inner, mode=mode, cell_value=cell_value, schedule=schedule,
                           jitter=jitter)
        return outs[0]
    lib = load()
    f_dtype = _f_dtype(F)
    u_out = _out_tensor(F, u_out)
    src, keep = _sources(F, idx3, q, stream)
    opts = _options(delta, max_rounds, max_sweeps, workers, shuffle, timing, round_log, inner,
                    mode, cell_value, schedule, jitter)
    nz, ny, nx = F.shape
    dims = _dims_array((nx, ny, nz))
    rc = lib.eik_solve_ex(ctypes.cast(dims, ctypes.c_void_p), float(h),
                          ctypes.c_void_p(F.data_ptr()), f_dtype, ctypes.byref(src),
                          ctypes.c_void_p(u_out.data_ptr()), int(cell), float(tol),
                          _stream_handle(stream), ctypes.byref(opts))
    del keep
    if rc != EIK_OK and check:
        raise EikError(rc, "eik_solve: ")
    return u_out


def solve_noalloc(F, h: float, idx3, q, cell: int = 8, tol: float = 0.0, u_out=None,
                  stream=None, check: bool = True, **opt):
    """Enqueue one solve through eik_solve_noalloc (the entry point that allocates nothing; its
    workspace is the library's static device scratch).  Arguments as in ``solve``; u_out must be
    given (the library allocates nothing, and neither does this wrapper).  Returns the C status
    (raises on a negative one if ``check``)."""
    lib = load()
    f_dtype = _f_dtype(F)
    if u_out is None:
        raise ValueError("u_out is required: eik_solve_noalloc allocates nothing")
    u_out = _out_tensor(F, u_out)
    src, keep = _sources(F, idx3, q, stream)
    opts = _options(**opt)
    nz, ny, nx = F.shape
    dims = _dims_array((nx, ny, nz))
    rc = lib.eik_solve_noalloc(ctypes.cast(dims, ctypes.c_void_p), float(h),
                               ctypes.c_void_p(F.data_ptr()), f_dtype, ctypes.byref(src),
                               ctypes.c_void_p(u_out.data_ptr()), int(cell), float(tol),
                               _stream_handle(stream), ctypes.byref(opts))
    del keep
    if rc != EIK_OK and check:
        raise EikError(rc, "eik_solve_noalloc: ")
    return rc


def autotune(F, h: float, idx3, q, tol: float = 0.0, reps: int = 2, u_out=None, stream=None):
    """Time every solver configuration on this problem (eik_autotune); returns (best, table)
    as dicts with keys cell, inner, workers, delta, ms, status.  Blocks until done."""
    lib = load()
    f_dtype = _f_dtype(F)
    u_out = _out_tensor(F, u_out)
    src, keep = _sources(F, idx3, q, stream)
    nz, ny, nx = F.shape
    dims = _dims_array((nx, ny, nz))
    table = (TuneEntry * 32)()
    n = ctypes.c_int(0)
    best = TuneEntry()
    rc = lib.eik_autotune(ctypes.cast(dims, ctypes.c_void_p), float(h),
                          ctypes.c_void_p(F.data_ptr()), f_dtype, ctypes.byref(src),
                          ctypes.c_void_p(u_out.data_ptr()), float(tol), _stream_handle(stream),
                          int(reps), table, 32, ctypes.byref(n), ctypes.byref(best))
    del keep
    if rc != EIK_OK:
        raise EikError(rc, "eik_autotune: ")
    return best.as_dict(), [table[i].as_dict() for i in range(n.value)]


def problem_bytes(dims, cell: int = 8, f_dtype: int = EIK_F32, mode: int = EIK_MODE_FP64) -> int:
    """Device bytes of one grid's arrays inside a server pool (dims = (nx, ny, nz))."""
    out = ctypes.c_size_t(0)
    rc = load().eik_problem_bytes(ctypes.cast(_dims_array(dims), ctypes.c_void_p), int(cell),
                                  int(f_dtype), int(mode), ctypes.byref(out))
    if rc != EIK_OK:
        raise EikError(rc, "eik_problem_bytes: ")
    return int(out.value)


def solve_batch(problems, cell: int = 8, stream=None, check: bool = True, **opt):
    """Enqueue one batched solve of independent grids on ``stream``.

    problems: sequence of dicts with keys F, h, src (idx3), q and optional tol, u_out,
    u_approx (an approximation to polish); every F of one dtype.  Returns the list of u_out tensors; ``batch_status(len(problems))`` waits and
    returns the per-problem status.
    """
    lib = load()
    if not problems:
        raise ValueError("empty batch")
    f_dtype = _f_dtype(problems[0]["F"])
    arr = (Problem * len(problems))()
    outs, keep = [], []
    for i, p in enumerate(problems):
        if _f_dtype(p["F"]) != f_dtype:
            raise ValueError("every F of a batch has the same dtype")
        pb, u, k = _problem(p["F"], p["h"], p["src"], p["q"], p.get("tol", 0.0),
                            p.get("u_out"), stream, p.get("u_approx"))
        arr[i] = pb
        outs.append(u)
        keep.append(k)
    opts = _options(**opt)
    rc = lib.eik_solve_batch(len(problems), arr, f_dtype, int(cell), _stream_handle(stream),
                             ctypes.byref(opts))
    del keep
    if rc != EIK_OK and check:
        raise EikError(rc, "eik_solve_batch: ")
    return outs


def batch_status(n: int, stream=None):
    """Wait for ``stream``; the device status of each problem of its last batch (numpy int32)."""
    st = np.zeros(max(n, 0), dtype=np.int32)
    got = load().eik_batch_status(_stream_handle(stream), int(n), st.ctypes.data)
    if got < 0:
        raise EikError(got, "eik_batch_status: ")
    return st[:got]


class Server:
    """Continuous-batching server over the eik_server_* calls (one thread per server).

    submit() admits a grid or returns None when it does not fit now (EIK_EBUSY); step() runs
    one step and returns {ticket: (status, u_out)} for the grids retired in it.
    """

    def __init__(self, pool_bytes: int, max_cells: int, max_problems: int, cell: int = 8,
                 f_dtype: int = EIK_F32, stream=None, **opt):
        self._lib = load()
        self._stream = stream
        self._h = ctypes.c_void_p(None)
        opts = _options(**opt)
        rc = self._lib.eik_server_create(ctypes.byref(self._h), int(pool_bytes), int(max_cells),
                                         int(max_problems), int(cell), int(f_dtype),
                                         _stream_handle(stream), ctypes.byref(opts))
        if rc != EIK_OK:
            self._h = None
            raise EikError(rc, "eik_server_create: ")
        self._pending = {}   # ticket -> (u_out, keep-alive)
        self._staged = []    # keep-alive of problems whose inputs the next step reads
        _live_servers.add(self)

    def submit(self, F, h, idx3, q, tol=0.0, u_out=None, u_approx=None):
        pb, u, keep = _problem(F, h, idx3, q, tol, u_out, None, u_approx)
        t = ctypes.c_int64(-1)
        rc = self._lib.eik_server_submit(self._h, ctypes.byref(pb), ctypes.byref(t))
        if rc == EIK_EBUSY:
            return None
        if rc != EIK_OK:
            raise EikError(rc, "eik_server_submit: ")
        self._pending[int(t.value)] = (u, F)
        self._staged.append(keep)
        return int(t.value)

    def step(self, rounds: int):
        fin = ctypes.c_int(0)
        rc = self._lib.eik_server_step(self._h, int(rounds), ctypes.byref(fin))
        self._staged.clear()
        if rc not in (EIK_OK, EIK_ECANCELLED):
            raise EikError(rc, "eik_server_step: ")
        out = {}
        n = max(fin.value, 0)
        while True:
            m = max(n, 16)
            tickets = np.zeros(m, dtype=np.int64)
            st = np.zeros(m, dtype=np.int32)
            got = ctypes.c_int(0)
            prc = self._lib.eik_server_poll(self._h, m, tickets.ctypes.data, st.ctypes.data,
                                            ctypes.byref(got))
            if prc != EIK_OK:
                raise EikError(prc, "eik_server_poll: ")
            for t, s in zip(tickets[:got.value], st[:got.value]):
                u, _ = self._pending.pop(int(t))
                out[int(t)] = (int(s), u)
            if got.value < m:
                break
        return out

    def load(self):
        np_, nc, pb = ctypes.c_int(0), ctypes.c_int64(0), ctypes.c_size_t(0)
        rc = self._lib.eik_server_load(self._h, ctypes.byref(np_), ctypes.byref(nc),
                                       ctypes.byref(pb))
        if rc != EIK_OK:
            raise EikError(rc, "eik_server_load: ")
        return {"problems": np_.value, "cells": nc.value, "pool_bytes": pb.value}

    def polish_redone(self) -> int:
        """Problems restarted from +inf after their polished result failed the eq. (2) check."""
        return int(self._lib.eik_server_polish_redone(self._h))

    def close(self):
        if self._h:
            self._lib.eik_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status(stream=None):
    """Wait for ``stream`` and return (status code, counters dict) of its last solve."""
    st = Stats()
    rc = load().eik_stream_status(_stream_handle(stream), ctypes.byref(st))
    return rc, st.as_dict()


def kernel_times(n: int, stream=None):
    """(solve_kernel_ms, whole_call_ms) arrays of the last n solves enqueued with timing=True."""
    a = np.zeros(max(n, 0), dtype=np.float64)
    b = np.zeros(max(n, 0), dtype=np.float64)
    got = load().eik_kernel_times(_stream_handle(stream), int(n), a.ctypes.data, b.ctypes.data)
    if got < 0:
        raise EikError(got, "eik_kernel_times: ")
    return a[:got], b[:got]


def cancel(stream=None) -> int:
    """Ask every solve enqueued on ``stream`` so far to stop (eik_cancel); does not wait."""
    return int(load().eik_cancel(_stream_handle(stream)))


def release():
    load().eik_release()
