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

PPC_OK, PPC_EINVAL, PPC_ENOMEM, PPC_EDEVICE, PPC_EBUSY, PPC_ETIMEDOUT = 0, 1, 2, 3, 4, 5
WIDTHS = (8, 16, 32, 64)


class PpcError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s" % (what, lib().ppc_status_string(status).decode()))


_lib = None


class ppc_desc(ctypes.Structure):
    _fields_ = [("buf", ctypes.c_void_p), ("nbytes", ctypes.c_uint64), ("counts", ctypes.c_void_p),
                ("width", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ppc_plan_opts(ctypes.Structure):
    _fields_ = [("tiles_per_item", ctypes.c_uint32), ("waves", ctypes.c_uint32),
                ("autotune", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ppc_plan_info(ctypes.Structure):
    _fields_ = [("n_arrays", ctypes.c_uint64), ("n_items", ctypes.c_uint64),
                ("total_bytes", ctypes.c_uint64), ("tiles_per_item", ctypes.c_uint32),
                ("waves", ctypes.c_uint32), ("tuned", ctypes.c_uint32), ("graph", ctypes.c_uint32)]


class ppc_server_cfg(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("tiles_per_item", ctypes.c_uint32),
                ("inflight_bytes", ctypes.c_uint64), ("waves", ctypes.c_uint32),
                ("batch_timeout_us", ctypes.c_uint32)]


class ppc_request(ctypes.Structure):
    _fields_ = [("column", ctypes.c_uint32), ("width", ctypes.c_uint32), ("offset", ctypes.c_uint64),
                ("nbytes", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class ppc_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("width", ctypes.c_uint32), ("status", ctypes.c_uint32),
                ("t_submit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("counts", ctypes.c_uint64 * 64)]


class ppc_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("inflight", "pending", "inflight_bytes", "batches",
                                                "batched_requests", "max_batch_seen",
                                                "host_dispatch_ns", "host_retire_ns")]


class ppc_trace_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("n_requests", "total_bytes", "makespan_ns", "p50_ns",
                                                "p99_ns", "max_ns", "mean_ns", "batches",
                                                "busy_rejections", "host_dispatch_ns",
                                                "host_retire_ns")] + \
               [("mean_batch", ctypes.c_double), ("gbps", ctypes.c_double)]


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
        "ppc_pospopcnt_at": ([_c_uint, _c_ptr, _c_ptr, _c_size, ctypes.c_uint64, _c_ptr], ctypes.c_int),
        "ppc_popcount": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt_timed": ([_c_uint, _c_ptr, _c_ptr, _c_size, _c_ptr, _c_ptr, _c_ptr], ctypes.c_int),
        "ppc_read_roofline_timed": ([_c_ptr, _c_ptr, _c_size, _c_ptr, _c_ptr, _c_ptr], ctypes.c_int),
        "ppc_pospopcnt_variant": ([_c_uint, _c_uint, _c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_set_plain_geometry": ([_c_uint, _c_uint], ctypes.c_int),
        "ppc_get_plain_geometry": ([ctypes.POINTER(_c_uint), ctypes.POINTER(_c_uint)], ctypes.c_int),
        "ppc_read_roofline": ([_c_ptr, _c_ptr, _c_size, _c_ptr], ctypes.c_int),
        "ppc_plan_create": ([ctypes.POINTER(_c_ptr), ctypes.POINTER(ppc_desc), _c_size,
                             ctypes.POINTER(ppc_plan_opts), _c_ptr], ctypes.c_int),
        "ppc_plan_run": ([_c_ptr, _c_ptr], ctypes.c_int),
        "ppc_plan_get_info": ([_c_ptr, ctypes.POINTER(ppc_plan_info)], ctypes.c_int),
        "ppc_plan_destroy": ([_c_ptr], ctypes.c_int),
        "ppc_batch_noalloc": ([_c_ptr, ctypes.c_uint32, _c_ptr, _c_ptr], ctypes.c_int),
        "ppc_server_create": ([ctypes.POINTER(_c_ptr), _c_ptr, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.POINTER(ppc_server_cfg)], ctypes.c_int),
        "ppc_server_submit": ([_c_ptr, ctypes.POINTER(ppc_request)], ctypes.c_int),
        "ppc_server_poll": ([_c_ptr, ctypes.POINTER(ppc_result), _c_size, ctypes.POINTER(_c_size)],
                            ctypes.c_int),
        "ppc_server_get_stats": ([_c_ptr, ctypes.POINTER(ppc_server_stats)], ctypes.c_int),
        "ppc_server_run_trace": ([_c_ptr, ctypes.POINTER(ppc_request), ctypes.POINTER(ctypes.c_uint64),
                                  _c_size, ctypes.POINTER(ppc_result), ctypes.POINTER(ppc_trace_stats)],
                                 ctypes.c_int),
        "ppc_server_destroy": ([_c_ptr], ctypes.c_int),
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
        # torch ships its own HIP runtime under the same soname.  Loaded
        # first, it is the runtime libppc.so binds to; loaded after
        # libppc.so, it would come in as a second runtime whose streams and
        # allocations the library's runtime does not know (launches on
        # torch's streams then fail).
        import torch  # noqa: F401

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
    size = buf.numel() * buf.element_size() if hasattr(buf, "numel") else None
    if nbytes is not None:
        nbytes = int(nbytes)
        if nbytes < 0 or (size is not None and nbytes > size):
            raise ValueError("nbytes=%d outside the %s-byte tensor" % (nbytes, size))
        return nbytes
    if size is not None:
        return size
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


def ppc_pospopcnt_at(width, counts, buf, nbytes=None, stream_offset=0, stream=None):
    _check(lib().ppc_pospopcnt_at(int(width), _counts_ptr(counts, width), _ptr(buf), _nbytes(buf, nbytes),
                                  int(stream_offset), _stream(stream)), "ppc_pospopcnt_at")


def ppc_popcount(total, buf, nbytes=None, stream=None):
    _check(lib().ppc_popcount(_counts_ptr(total, 1), _ptr(buf), _nbytes(buf, nbytes), _stream(stream)),
           "ppc_popcount")


def ppc_pospopcnt_variant(variant, width, counts, buf, nbytes=None, stream=None):
    _check(lib().ppc_pospopcnt_variant(int(variant), int(width), _counts_ptr(counts, width), _ptr(buf),
                                       _nbytes(buf, nbytes), _stream(stream)), "ppc_pospopcnt_variant")


_hip = None


def _hiprt():
    """The HIP runtime libppc.so itself uses (loaded by soname, so it is the
    process's one runtime, torch's when torch is loaded)."""
    global _hip
    if _hip is None:
        lib()
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        h.hipEventCreate.restype = ctypes.c_int
        h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        h.hipEventElapsedTime.restype = ctypes.c_int
        h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        h.hipEventDestroy.restype = ctypes.c_int
        _hip = h
    return _hip


class HipEvent:
    """A timing hipEvent_t for the *_timed calls, which record it from the
    kernel dispatch itself."""

    def __init__(self):
        self.handle = ctypes.c_void_p()
        if _hiprt().hipEventCreate(ctypes.byref(self.handle)) != 0:
            raise RuntimeError("hipEventCreate failed")

    def elapsed_ms(self, end: "HipEvent") -> float:
        """Milliseconds from this event to `end`; both must have completed."""
        ms = ctypes.c_float()
        rc = _hiprt().hipEventElapsedTime(ctypes.byref(ms), self.handle, end.handle)
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed (%d)" % rc)
        return ms.value

    def __del__(self):
        if self.handle and _hip is not None:
            _hip.hipEventDestroy(self.handle)
            self.handle = ctypes.c_void_p()


def _event(e):
    if e is None:
        return None
    if isinstance(e, int):
        return e
    if isinstance(e, HipEvent):
        return e.handle.value
    raise TypeError("expected a HipEvent or a raw hipEvent_t address")


def ppc_pospopcnt_timed(width, counts, buf, nbytes=None, stream=None, start_event=None, stop_event=None):
    """Plain call whose kernel dispatch records the given HipEvent pair at
    its start and end."""
    _check(lib().ppc_pospopcnt_timed(int(width), _counts_ptr(counts, width), _ptr(buf), _nbytes(buf, nbytes),
                                     _stream(stream), _event(start_event), _event(stop_event)),
           "ppc_pospopcnt_timed")


def ppc_read_roofline_timed(sink, buf, nbytes=None, stream=None, start_event=None, stop_event=None):
    _check(lib().ppc_read_roofline_timed(_ptr(sink), _ptr(buf), _nbytes(buf, nbytes), _stream(stream),
                                         _event(start_event), _event(stop_event)), "ppc_read_roofline_timed")


def ppc_set_plain_geometry(waves: int, waves_per_block: int):
    _check(lib().ppc_set_plain_geometry(int(waves), int(waves_per_block)), "ppc_set_plain_geometry")


def ppc_get_plain_geometry() -> tuple[int, int]:
    w, b = _c_uint(0), _c_uint(0)
    _check(lib().ppc_get_plain_geometry(ctypes.byref(w), ctypes.byref(b)), "ppc_get_plain_geometry")
    return w.value, b.value


def ppc_read_roofline(sink, buf, nbytes=None, stream=None):
    _check(lib().ppc_read_roofline(_ptr(sink), _ptr(buf), _nbytes(buf, nbytes), _stream(stream)),
           "ppc_read_roofline")


def make_descs(bufs, nbytes, counts, widths):
    """ctypes array of ppc_desc from parallel sequences of device addresses
    (ints), byte lengths, counter addresses and widths."""
    n = len(nbytes)
    arr = (ppc_desc * n)()
    for i in range(n):
        arr[i].buf = int(bufs[i]) if bufs[i] is not None else None
        arr[i].nbytes = int(nbytes[i])
        arr[i].counts = int(counts[i])
        arr[i].width = int(widths[i])
        arr[i].reserved = 0
    return arr


def ppc_plan_create(descs, n=None, opts=None, stream=None):
    """Returns an opaque plan handle (int).  ``descs`` is a ctypes array of
    ppc_desc (see make_descs); ``opts`` a ppc_plan_opts or None."""
    handle = _c_ptr()
    n = len(descs) if n is None else n
    rc = lib().ppc_plan_create(ctypes.byref(handle), descs, n,
                               ctypes.byref(opts) if opts is not None else None, _stream(stream))
    _check(rc, "ppc_plan_create")
    return handle.value


def ppc_plan_run(plan, stream=None):
    _check(lib().ppc_plan_run(plan, _stream(stream)), "ppc_plan_run")


def ppc_plan_get_info(plan) -> dict:
    info = ppc_plan_info()
    _check(lib().ppc_plan_get_info(plan, ctypes.byref(info)), "ppc_plan_get_info")
    return {k: getattr(info, k) for k, _ in ppc_plan_info._fields_}


def ppc_plan_destroy(plan):
    _check(lib().ppc_plan_destroy(plan), "ppc_plan_destroy")


def descs_bytes(descs) -> bytes:
    """The raw bytes of a ctypes ppc_desc array (the C layout), to be placed
    in device memory for :func:`ppc_batch_noalloc`."""
    return ctypes.string_at(ctypes.addressof(descs), ctypes.sizeof(descs)) if len(descs) else b""


def ppc_batch_noalloc(descs_dev, n, n_invalid=None, stream=None):
    """``descs_dev``: device tensor (or address) holding ``n`` ppc_desc in
    the C layout (see descs_bytes); ``n_invalid``: optional device tensor
    of one 32-bit integer that receives the number of invalid descriptors."""
    _check(lib().ppc_batch_noalloc(_ptr(descs_dev), int(n), _ptr(n_invalid), _stream(stream)),
           "ppc_batch_noalloc")


def ppc_server_create(pool, pool_bytes=None, column_bytes=None, cfg=None):
    """Returns an opaque server handle over a device pool tensor (or address)."""
    handle = _c_ptr()
    rc = lib().ppc_server_create(ctypes.byref(handle), _ptr(pool), _nbytes(pool, pool_bytes),
                                 int(column_bytes), ctypes.byref(cfg) if cfg is not None else None)
    _check(rc, "ppc_server_create")
    return handle.value


def ppc_server_submit(server, column, width, offset, nbytes, tag=0) -> int:
    """Returns PPC_OK or PPC_EBUSY; raises on other errors."""
    req = ppc_request(int(column), int(width), int(offset), int(nbytes), int(tag))
    rc = lib().ppc_server_submit(server, ctypes.byref(req))
    if rc not in (PPC_OK, PPC_EBUSY):
        raise PpcError(rc, "ppc_server_submit")
    return rc


def ppc_server_poll(server, cap=1024) -> list:
    out = (ppc_result * cap)()
    n = _c_size(0)
    _check(lib().ppc_server_poll(server, out, cap, ctypes.byref(n)), "ppc_server_poll")
    return [out[i] for i in range(n.value)]


def ppc_server_get_stats(server) -> dict:
    st = ppc_server_stats()
    _check(lib().ppc_server_get_stats(server, ctypes.byref(st)), "ppc_server_get_stats")
    return {k: getattr(st, k) for k, _ in ppc_server_stats._fields_}


def ppc_server_run_trace(server, column, width, offset, nbytes, arrival_ns):
    """Open-loop trace through the server.  Returns (results ctypes array,
    stats dict)."""
    n = len(nbytes)
    reqs = (ppc_request * n)()
    for i in range(n):
        reqs[i].column, reqs[i].width = int(column[i]), int(width[i])
        reqs[i].offset, reqs[i].nbytes, reqs[i].tag = int(offset[i]), int(nbytes[i]), i
    arr = (ctypes.c_uint64 * n)(*[int(a) for a in arrival_ns])
    results = (ppc_result * n)()
    st = ppc_trace_stats()
    _check(lib().ppc_server_run_trace(server, reqs, arr, n, results, ctypes.byref(st)),
           "ppc_server_run_trace")
    return results, {k: getattr(st, k) for k, _ in ppc_trace_stats._fields_}


def ppc_server_destroy(server):
    _check(lib().ppc_server_destroy(server), "ppc_server_destroy")


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
