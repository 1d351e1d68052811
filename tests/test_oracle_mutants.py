"""Plausible mistakes planted in a copy of the oracle's C source must be caught.

Each mutant is compiled on the CPU from ppc_oracle.c with one edit, and the
pins used in test_oracle_definition.py (the stream statement of Section 1,
the single-bit closed form, the ragged tail) must reject it.  This shows the
pins are strong enough to catch a wrong byte order, a reversed bit index, a
dropped trailing word, a skipped last bit or a cleared (not accumulated)
counter array.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "ppc_oracle.c")

MUTANTS = {
    "big_endian": ("word |= byte << (8 * b);", "word |= byte << (8 * (s - 1 - b));"),
    "reversed_bits": ("counts[j] += (word >> j) & 1u;", "counts[j] += (word >> (w - 1 - j)) & 1u;"),
    "drop_partial_word": ("size_t nwords = (nbytes + s - 1) / s;\n    for (size_t i",
                          "size_t nwords = nbytes / s;\n    for (size_t i"),
    "skip_last_bit": ("for (unsigned j = 0; j < w; j++)\n            counts[j] +=",
                      "for (unsigned j = 0; j + 1 < w; j++)\n            counts[j] +="),
    "clears_counts": ("        for (unsigned j = 0; j < w; j++)\n            counts[j] += (word >> j) & 1u;",
                      "        for (unsigned j = 0; j < w; j++)\n            counts[j] = (word >> j) & 1u;"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new, 1)
    c_path = os.path.join(tmpdir, name + ".c")
    so_path = os.path.join(tmpdir, name + ".so")
    with open(c_path, "w") as f:
        f.write(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", so_path, c_path])
    lib = ctypes.CDLL(so_path)
    lib.ppc_oracle_pospopcnt.argtypes = [ctypes.c_uint, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.c_void_p, ctypes.c_size_t]
    return lib


def _call(lib, data, w):
    buf = np.frombuffer(bytes(data), dtype=np.uint8)
    out = np.zeros(w, dtype=np.uint64)
    lib.ppc_oracle_pospopcnt(w, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             buf.ctypes.data if buf.size else None, buf.size)
    return out


def _pins_pass(lib) -> bool:
    rng = np.random.default_rng(0)
    for w in (8, 16, 32, 64):
        for n in range(0, 40):
            data = bytes(rng.integers(0, 256, size=n, dtype=np.uint8))
            if _call(lib, data, w).tolist() != oracle.pospopcnt_streams(data, w):
                return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(name, d)
        if name == "clears_counts":
            # the accumulate pin: a pre-loaded counter must be added to
            acc = np.full(8, 5, dtype=np.uint64)
            buf = np.frombuffer(b"\x01\x01", dtype=np.uint8)
            lib.ppc_oracle_pospopcnt(8, acc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     buf.ctypes.data, 2)
            assert acc[0] != 7
        else:
            assert not _pins_pass(lib)


def test_unmutated_copy_passes_the_same_pins():
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "same.so")
        subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", so, SRC])
        lib = ctypes.CDLL(so)
        lib.ppc_oracle_pospopcnt.argtypes = [ctypes.c_uint, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.c_void_p, ctypes.c_size_t]
        assert _pins_pass(lib)
