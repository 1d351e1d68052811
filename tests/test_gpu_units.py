"""GPU unit tests of the device building blocks, each driven through a
test-only kernel (tests/csrc/unit_kernels.hip, which compiles the library's
device header) and checked against host arithmetic that shares nothing with
the device code:

* full adder (Section 3.1): sum + 2*carry = a + b + c in every bit column,
  and the worked example of Section 3.1;
* CSA_{16+4} (Sections 3.2, 4.2): the place-value identity
  a1' + 2a2' + 4a4' + 8a8' + 16a16 = a1 + 2a2 + 4a4 + 8a8 + sum(v), for all
  2^20 bit columns;
* the end-of-segment reduction (Section 4.5): lane L's result is the
  weighted number of set bits at address position L over all lanes and
  planes, for every number of planes in use;
* f_w: counts of address positions land in the counter of the byte slot
  the buffer's own bytes give them, for every width and pointer residue.
"""
import ctypes
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "libppc_unit.so")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def unit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(LIB):
        pytest.fail("tests/csrc/libppc_unit.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    p, u = ctypes.c_void_p, ctypes.c_uint32
    L.ppc_unit_full_add.argtypes = [p, p, p, p, p, u]
    L.ppc_unit_csa16.argtypes = [p, p, p, u]
    L.ppc_unit_wave_counts.argtypes = [p, u, p, u]
    L.ppc_unit_fold.argtypes = [p, u, u, p, u]
    for f in (L.ppc_unit_full_add, L.ppc_unit_csa16, L.ppc_unit_wave_counts, L.ppc_unit_fold):
        f.restype = ctypes.c_int
    L.ppc_unit_planes.restype = ctypes.c_int
    return L


def dev(a: np.ndarray):
    """Host array -> device tensor with the same bytes (unsigned types travel
    as their signed twins; the kernels read raw memory)."""
    a = np.ascontiguousarray(a)
    signed = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}.get(a.dtype)
    return torch.from_numpy(a.view(signed) if signed else a).to("cuda:0")


def host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def bits(a: np.ndarray) -> np.ndarray:
    """uint32 array -> its bits (LSB first) along a new last axis."""
    return np.unpackbits(a.astype("<u4").view(np.uint8).reshape(a.shape + (4,)), axis=-1,
                         bitorder="little").reshape(a.shape + (32,)).astype(np.int64)


def test_full_adder_bit_columns(unit):
    rng = np.random.default_rng(0)
    n = 4096
    a, b, c = (rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32) for _ in range(3))
    # the worked example of Section 3.1 in thread 0's first dword
    with open(os.path.join(GOLDEN, "full_adder_example.txt")) as f:
        row = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")][0]
    vals = dict(zip(("a", "b", "c", "C", "S"), row))
    a[0, 0], b[0, 0], c[0, 0] = (int(vals[k], 2) for k in ("a", "b", "c"))
    da, db, dc = dev(a), dev(b), dev(c)
    carry = torch.empty_like(da)
    s = torch.empty_like(da)
    assert unit.ppc_unit_full_add(da.data_ptr(), db.data_ptr(), dc.data_ptr(), carry.data_ptr(), s.data_ptr(), n) == 0
    torch.cuda.synchronize()
    C, S = host_u32(carry).reshape(n, 4), host_u32(s).reshape(n, 4)
    assert np.array_equal(bits(S) + 2 * bits(C), bits(a) + bits(b) + bits(c))
    assert (int(C[0, 0]) & 0xF, int(S[0, 0]) & 0xF) == (int(vals["C"], 2), int(vals["S"], 2))


def test_csa16_place_value_identity_all_columns(unit):
    # column k in [0, 2^20): bits 0..15 are the 16 inputs, bits 16..19 the
    # accumulator planes a1, a2, a4, a8; 128 columns per thread (one uint4)
    cols = np.arange(1 << 20, dtype=np.uint32).reshape(-1, 128)  # (8192, 128)
    n = cols.shape[0]

    def plane(bit):  # (n, 4) uint32: bit `bit` of every column, packed LSB first
        b = ((cols >> np.uint32(bit)) & np.uint32(1)).astype(np.uint8).reshape(n, 4, 32)
        return np.packbits(b, axis=-1, bitorder="little").view("<u4").reshape(n, 4)

    v = np.stack([plane(i) for i in range(16)], axis=1)        # (n, 16, 4)
    acc = np.stack([plane(16 + i) for i in range(4)], axis=1)  # (n, 4, 4)
    dacc, dv = dev(acc), dev(v)
    out = torch.empty((n, 5, 4), dtype=torch.int32, device="cuda:0")
    assert unit.ppc_unit_csa16(dacc.data_ptr(), dv.data_ptr(), out.data_ptr(), n) == 0
    torch.cuda.synchronize()
    o = host_u32(out).reshape(n, 5, 4)
    got = sum(bits(o[:, i, :]) << i for i in range(5))           # (n, 4, 32) weighted output
    k = cols.reshape(n, 4, 32).astype(np.int64)
    want = sum(((k >> i) & 1) for i in range(16)) + sum(((k >> (16 + i)) & 1) << i for i in range(4))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("e_used", list(range(0, 11)))
def test_wave_reduction_counts_every_position(unit, e_used):
    kp = unit.ppc_unit_planes()
    assert kp == 10
    rng = np.random.default_rng(100 + e_used)
    n_waves = 6
    planes = np.zeros((n_waves, 64, kp, 4), dtype=np.uint32)
    planes[:, :, :e_used, :] = rng.integers(0, 2**32, size=(n_waves, 64, e_used, 4), dtype=np.uint64)
    if e_used:
        planes[0, :, :e_used, :] = 0xFFFFFFFF  # the largest value every position can reach
    out = torch.empty(n_waves * 64, dtype=torch.int32, device="cuda:0")
    assert unit.ppc_unit_wave_counts(dev(planes).data_ptr(), e_used, out.data_ptr(), n_waves) == 0
    torch.cuda.synchronize()
    got = host_u32(out).reshape(n_waves, 64).astype(np.int64)
    b = bits(planes)                                   # (waves, lanes, planes, dword, bit)
    weight = (1 << np.arange(kp, dtype=np.int64))[None, None, :, None]
    lo = ((b[:, :, :, 0, :] + b[:, :, :, 2, :]) * weight).sum(axis=(1, 2))  # dwords x, z: positions 0..31
    hi = ((b[:, :, :, 1, :] + b[:, :, :, 3, :]) * weight).sum(axis=(1, 2))  # dwords y, w: positions 32..63
    want = np.concatenate([lo, hi], axis=1)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("width", [0, 8, 16, 32, 64])
def test_fold_sends_each_position_to_its_byte_slot(unit, width):
    s = max(width // 8, 1)
    rng = np.random.default_rng(width)
    n_waves = 8
    for m in range(s):
        v = rng.integers(0, 1 << 40, size=(n_waves, 64), dtype=np.uint64)
        counts = torch.zeros((n_waves, 64), dtype=torch.int64, device="cuda:0")
        assert unit.ppc_unit_fold(dev(v).data_ptr(), width, m, counts.data_ptr(), n_waves) == 0
        torch.cuda.synchronize()
        got = counts.cpu().numpy().view(np.uint64)
        want = np.zeros((n_waves, 64), dtype=np.uint64)
        if width == 0:
            want[:, 0] = v.sum(axis=1, dtype=np.uint64)
        else:
            # a buffer starting at address A with A mod s = m: its byte b sits at
            # address slot (A + b) mod 8 and feeds counters 8*(b mod s) + bit
            A = 8 * 1000 + m
            for a in range(8):
                b = next(x for x in range(8) if (A + x) % 8 == a)
                for k in range(8):
                    want[:, 8 * (b % s) + k] += v[:, 8 * a + k]
        assert np.array_equal(got, want), "width %d, m %d" % (width, m)
