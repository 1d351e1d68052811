"""The oracle: a plain, slow, obviously correct CPU model of pospopcnt.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with ``paper_2412_16370_amd`` and never imports it.

Two independent statements of the operation live here:

* :func:`pospopcnt` -- the word loop of Fig. 2 (Section 1), in plain C
  (``ppc_oracle.c``), with little-endian words, a zero-padded trailing word and
  bit positions counted from the caller's pointer.
* :func:`pospopcnt_streams` -- the "w interleaved bit streams" statement of
  Section 1 in pure Python: the input is one long bit string (byte 0 first,
  least significant bit first) and counter j sums the bits at j, j+w, j+2w, ...

They are pinned against each other and against the invariants and closed
forms in ``tests/test_oracle_*.py``.  Every function cites the passage it
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppc_oracle.c")
_LIB = os.path.join(_HERE, "libppc_oracle.so")

WIDTHS = (8, 16, 32, 64)

_lib = None


def build(force: bool = True) -> str:
    """Compile ``ppc_oracle.c`` into ``libppc_oracle.so`` with the host gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
             "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.ppc_oracle_pospopcnt.argtypes = [
            ctypes.c_uint, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p,
            ctypes.c_size_t]
        lib.ppc_oracle_pospopcnt.restype = ctypes.c_int
        lib.ppc_oracle_pospopcnt_mt.argtypes = [
            ctypes.c_uint, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p,
            ctypes.c_size_t, ctypes.c_int]
        lib.ppc_oracle_pospopcnt_mt.restype = ctypes.c_int
        lib.ppc_oracle_sweep.argtypes = [
            ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_size_t,
            ctypes.POINTER(ctypes.c_uint64)]
        lib.ppc_oracle_sweep.restype = ctypes.c_int
        lib.ppc_oracle_popcount.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
        lib.ppc_oracle_popcount.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _as_u8(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    arr = np.ascontiguousarray(data)
    return arr.view(np.uint8).reshape(-1)


def pospopcnt(data, w: int, counts: np.ndarray | None = None) -> np.ndarray:
    """counts[j] += bit j of every little-endian w-bit word of ``data``.

    Fig. 2 (Section 1) word loop; counters accumulate (Section 4, step 1,
    footnote).  Returns the (possibly new) uint64 counter array of length w.
    """
    if w not in WIDTHS:
        raise ValueError("width must be one of 8, 16, 32, 64")
    buf = _as_u8(data)
    out = np.zeros(w, dtype=np.uint64) if counts is None else counts
    if out.dtype != np.uint64 or out.shape != (w,) or not out.flags.c_contiguous:
        raise ValueError("counts must be a contiguous uint64 array of length w")
    rc = _load().ppc_oracle_pospopcnt(
        w, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        buf.ctypes.data if buf.size else None, buf.size)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def pospopcnt_mt(data, w: int, nthreads: int) -> np.ndarray:
    """Same result as :func:`pospopcnt`, split over threads at word
    boundaries and summed (the streamed-accumulation use of Section 4)."""
    if w not in WIDTHS:
        raise ValueError("width must be one of 8, 16, 32, 64")
    buf = _as_u8(data)
    out = np.zeros(w, dtype=np.uint64)
    rc = _load().ppc_oracle_pospopcnt_mt(
        w, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        buf.ctypes.data if buf.size else None, buf.size, int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def host_threads() -> int:
    """Host cores this process may run on (its CPU affinity set)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def pospopcnt_ranges(data, starts, lengths, widths, threads: int | None = None) -> list:
    """:func:`pospopcnt` of many ranges data[start:start+length] at their
    own widths, each range counted by the Fig. 2 word loop on its own (the
    same call as :func:`pospopcnt`), spread over host threads.  Returns the
    list of uint64 counter arrays in input order."""
    from concurrent.futures import ThreadPoolExecutor

    buf = _as_u8(data)
    jobs = [(int(s), int(n), int(w)) for s, n, w in zip(starts, lengths, widths)]
    for s, n, w in jobs:
        if w not in WIDTHS or s < 0 or n < 0 or s + n > buf.size:
            raise ValueError("range or width out of bounds: %r" % ((s, n, w),))
    # the C loop runs without the interpreter lock, so threads run in parallel
    with ThreadPoolExecutor(max_workers=threads or host_threads()) as ex:
        return list(ex.map(lambda j: pospopcnt(buf[j[0]:j[0] + j[1]], j[2]), jobs))


def sweep(data, w: int, max_len: int, n_offsets: int) -> np.ndarray:
    """pospopcnt of every window data[o:o+n], o < n_offsets, n <= max_len.
    Returns an array of shape (n_offsets, max_len + 1, w)."""
    buf = _as_u8(data)
    if buf.size < n_offsets - 1 + max_len:
        raise ValueError("buffer too short for the sweep")
    out = np.zeros((n_offsets, max_len + 1, w), dtype=np.uint64)
    rc = _load().ppc_oracle_sweep(w, buf.ctypes.data, max_len, n_offsets,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def popcount(data) -> int:
    """Total number of set bits (the conventional population count that the
    Harley-Seal scheme of Section 3.3 computes), one bit at a time in C."""
    buf = _as_u8(data)
    return int(_load().ppc_oracle_popcount(
        buf.ctypes.data if buf.size else None, buf.size))


def pospopcnt_streams(data, w: int) -> list[int]:
    """Section 1's second statement of the operation, in pure Python.

    The input is read as one stream of 8*L bits (byte 0 first, least
    significant bit first within a byte).  Counter j is the number of set
    bits among stream positions j, j+w, j+2w, ...  Only for small inputs.
    """
    if w not in WIDTHS:
        raise ValueError("width must be one of 8, 16, 32, 64")
    raw = bytes(_as_u8(data))
    x = int.from_bytes(raw, "little")
    bits = bin(x)[2:][::-1].ljust(8 * len(raw), "0")
    return [bits[j::w].count("1") for j in range(w)]


def full_adder(a: int, b: int, c: int) -> tuple[int, int]:
    """Bit-parallel full adder of Section 3.1, from its arithmetic meaning.

    For every bit column i the three input bits are added as integers;
    the sum bit is the low bit of that total and the carry bit the high one.
    Returns (carry, sum) as ints.
    """
    carry = total = 0
    i = 0
    while (a >> i) or (b >> i) or (c >> i):
        n = ((a >> i) & 1) + ((b >> i) & 1) + ((c >> i) & 1)
        total |= (n & 1) << i
        carry |= (n >> 1) << i
        i += 1
    return carry, total

