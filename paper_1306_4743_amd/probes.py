"""Python binding of the bandwidth probes (include/eik_probe.h, libeik_probe.so): the HBM copy
and LDS read / write rates plain kernels reach on the device, reported beside the solver's
roofline fractions."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libeik_probe.so")
EXPORTS = ("eikp_copy", "eikp_lds")
_lib = None


def load():
    """Load libeik_probe.so (built in-tree with the solver); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    lib.eikp_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, vp, ctypes.POINTER(ctypes.c_float)]
    lib.eikp_copy.restype = i32
    lib.eikp_lds.argtypes = [i32, i32, i32, i32, vp, vp, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_double)]
    lib.eikp_lds.restype = i32
    _lib = lib
    return lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def copy(src, dst, reps: int = 10) -> float:
    """Mean ms of one copy src -> dst (contiguous CUDA tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    ms = ctypes.c_float(0)
    rc = load().eikp_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                          nbytes, int(reps), _stream(), ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"eikp_copy failed ({rc})")
    return float(ms.value)


def lds(out, blocks: int, iters: int, write: bool, reps: int = 10):
    """(mean ms of one launch, LDS bytes it moves); out: int32 CUDA tensor of blocks * 256."""
    if out.numel() < blocks * 256:
        raise ValueError("out is too small")
    ms, nb = ctypes.c_float(0), ctypes.c_double(0)
    rc = load().eikp_lds(int(blocks), int(iters), int(bool(write)), int(reps),
                         ctypes.c_void_p(out.data_ptr()), _stream(), ctypes.byref(ms),
                         ctypes.byref(nb))
    if rc != 0:
        raise RuntimeError(f"eikp_lds failed ({rc})")
    return float(ms.value), float(nb.value)


def measure(device, copy_bytes: int = 4 << 30, lds_iters: int = 4096):
    """Achievable HBM copy rate (GB/s, read + write) over a copy_bytes buffer and LDS read and
    write rates (GB/s) with four 32 KiB workgroups per CU."""
    import torch
    props = torch.cuda.get_device_properties(device)
    a = torch.empty(copy_bytes // 8, dtype=torch.float64, device=device).fill_(1.0)
    b = torch.empty_like(a)
    ms = copy(a, b, reps=10)
    hbm = 2.0 * copy_bytes / (ms / 1000.0) / 1e9
    del a, b
    blocks = 4 * props.multi_processor_count
    out = torch.empty(blocks * 256, dtype=torch.int32, device=device)
    r_ms, r_b = lds(out, blocks, lds_iters, False)
    w_ms, w_b = lds(out, blocks, lds_iters, True)
    return {"hbm_copy_gbs": hbm, "copy_bytes": copy_bytes, "copy_ms": ms,
            "lds_read_gbs": r_b / (r_ms / 1000.0) / 1e9,
            "lds_write_gbs": w_b / (w_ms / 1000.0) / 1e9,
            "lds_workgroups": blocks, "lds_iters": lds_iters,
            "cus": props.multi_processor_count}
