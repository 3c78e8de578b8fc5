"""ctypes binding of librowbench.so (include/rowbench.h): streaming reads for
the achievable HBM bandwidth, and row-pair intersections with the four
intersection variants.  Argument marshalling only; raises if the library
is missing."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librowbench.so")

RB_BINARY, RB_GALLOP, RB_MERGEPATH, RB_LDS = 0, 1, 2, 3
VARIANTS = {"binary": RB_BINARY, "gallop": RB_GALLOP, "mergepath": RB_MERGEPATH, "lds": RB_LDS}
EXPORTS = ["rb_stream_read", "rb_flush", "rb_intersect", "rb_last_error"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.rb_stream_read.argtypes = [vp, i64, i32, vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_uint64), vp]
        L.rb_flush.argtypes = [vp, i64, vp]
        L.rb_intersect.argtypes = [i32, vp, vp, vp, vp, i64, vp, i32, ctypes.POINTER(ctypes.c_double), vp]
        L.rb_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"rowbench error {rc}: {lib().rb_last_error().decode()}")


def stream_read(buf, reps: int = 5, stream=None) -> tuple[float, int]:
    """(ms per pass, checksum) of reading the int32 device tensor buf."""
    import torch
    acc = torch.zeros(1, dtype=torch.int64, device=buf.device)
    ms, ck = ctypes.c_double(), ctypes.c_uint64()
    _check(lib().rb_stream_read(ctypes.c_void_p(buf.data_ptr()), buf.numel(), reps, ctypes.c_void_p(acc.data_ptr()),
                                ctypes.byref(ms), ctypes.byref(ck), _s(stream)))
    return ms.value, ck.value


def flush(buf, stream=None):
    _check(lib().rb_flush(ctypes.c_void_p(buf.data_ptr()), buf.numel(), _s(stream)))


def intersect(variant: int, rp, col, pu, pv, out, grid: int = 0, stream=None) -> float:
    """out[i] = |row(pu[i]) & row(pv[i])| (device tensors); returns kernel ms."""
    n = pu.numel()
    assert pv.numel() == n and out.numel() >= n and n > 0
    ms = ctypes.c_double()
    _check(lib().rb_intersect(variant, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                              ctypes.c_void_p(pu.data_ptr()), ctypes.c_void_p(pv.data_ptr()), n,
                              ctypes.c_void_p(out.data_ptr()), grid, ctypes.byref(ms), _s(stream)))
    return ms.value


def _s(stream):
    return None if stream is None else ctypes.c_void_p(stream.cuda_stream)
