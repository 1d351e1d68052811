"""pospopcnt on AMD MI355X: thin Python binding of the C-ABI in include/ppc.h.

Every function here only marshals arguments (torch tensors -> device
pointers, torch streams -> hipStream_t) and calls ``libppc.so``; all counting
runs in the library's HIP kernels.  There is no fallback: if the library is
not built, every call raises.

Names follow the C-ABI: ``ppc_pospopcnt8/16/32/64(counts, buf, nbytes,
stream)``.  ``counts`` is a device tensor of w 64-bit integers (int64 or
uint64 storage, reinterpreted as uint64), ``buf`` any device tensor (its
data pointer is the byte pointer; slice it for unaligned starts).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppc.so")

PPC_OK, PPC_EINVAL, PPC_ENOMEM, PPC_EDEVICE, PPC_EBUSY = 0, 1, 2, 3, 4
WIDTHS = (8, 16, 32, 64)


class PpcError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s" % (what, lib().ppc_status_string(status).decode()))


_lib = None

_c_size = ctypes.c_size_t
_c_ptr = ctypes.c_void_p
_c_uint = ctypes.c_uint


def _declare(lib):
    sig = {
        "ppc_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "ppc_version": ([], ctypes.c_int),
        "ppc_pospopcnt": ([_c_uint, _c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt8": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt16": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt32": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt64": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_set_plain_geometry": ([_c_uint, _c_uint], ctypes.c_int),
        "ppc_get_plain_geometry": ([ctypes.POINTER(_c_uint), ctypes.POINTER(_c_uint)], ctypes.c_int),
        "ppc_read_roofline": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def lib():
    """The loaded ``libppc.so``.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libppc.so is not built (expected at %s); run "
                "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


# ------------------------------------------------------------ marshalling
def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("expected a device tensor, got one on %s" % x.device)
        if not x.is_contiguous():
            raise ValueError("expected a contiguous tensor")
        return x.data_ptr()
    raise TypeError("expected a device tensor or an integer address")


def _nbytes(buf, nbytes):
    if nbytes is not None:
        return int(nbytes)
    if hasattr(buf, "numel"):
        return buf.numel() * buf.element_size()
    raise ValueError("nbytes is required for a raw address")


def _stream(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc: int, what: str):
    if rc != PPC_OK:
        raise PpcError(rc, what)


def _counts_ptr(counts, w):
    if hasattr(counts, "numel"):
        if counts.numel() != w or counts.element_size() != 8:
            raise ValueError("counts must hold exactly %d 64-bit integers" % w)
    return _ptr(counts)


# ------------------------------------------------------------ C-ABI mirrors
def ppc_pospopcnt(width, counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt(int(width), _counts_ptr(counts, width), _ptr(buf),
                               _nbytes(buf, nbytes), _stream(stream)), "ppc_pospopcnt")


def ppc_pospopcnt8(counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt8(_counts_ptr(counts, 8), _ptr(buf), _nbytes(buf, nbytes),
                                _stream(stream)), "ppc_pospopcnt8")


def ppc_pospopcnt16(counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt16(_counts_ptr(counts, 16), _ptr(buf), _nbytes(buf, nbytes),
                                 _stream(stream)), "ppc_pospopcnt16")


def ppc_pospopcnt32(counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt32(_counts_ptr(counts, 32), _ptr(buf), _nbytes(buf, nbytes),
                                 _stream(stream)), "ppc_pospopcnt32")


def ppc_pospopcnt64(counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt64(_counts_ptr(counts, 64), _ptr(buf), _nbytes(buf, nbytes),
                                 _stream(stream)), "ppc_pospopcnt64")


def ppc_set_plain_geometry(waves: int, waves_per_block: int):
    _check(lib().ppc_set_plain_geometry(int(waves), int(waves_per_block)), "ppc_set_plain_geometry")


def ppc_get_plain_geometry() -> tuple[int, int]:
    w, b = _c_uint(0), _c_uint(0)
    _check(lib().ppc_get_plain_geometry(ctypes.byref(w), ctypes.byref(b)), "ppc_get_plain_geometry")
    return w.value, b.value


def ppc_read_roofline(sink, buf, nbytes=None, stream=None):
    _check(lib().ppc_read_roofline(_ptr(sink), _ptr(buf), _nbytes(buf, nbytes), _stream(stream)),
           "ppc_read_roofline")


# ------------------------------------------------------------ convenience
def pospopcnt(buf, width: int, counts=None, stream=None):
    """Allocate (or add into) a device counter tensor and count ``buf``.
    Returns the int64 device tensor holding the uint64 counts."""
    import torch

    if counts is None:
        counts = torch.zeros(width, dtype=torch.int64, device=buf.device)
    ppc_pospopcnt(width, counts, buf, None, stream)
    return counts


def counts_to_numpy(counts):
    """Device counter tensor -> host numpy uint64 array."""
    import numpy as np

    return counts.detach().cpu().numpy().view(np.uint64).copy()
