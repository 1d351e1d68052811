"""Pins of the oracle's word loop (Fig. 2) against things other than itself.

* The "w interleaved streams" statement of Section 1, written independently
  in pure Python, exhaustively on every 1- and 2-byte input and on random
  ragged inputs up to 64 bytes at every width.
* Closed forms: all-zero, all-ones, a single set bit, periodic patterns.
* Argument handling and the accumulate (never clear) contract of Section 4.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

WIDTHS = (8, 16, 32, 64)


@pytest.mark.parametrize("w", WIDTHS)
def test_every_one_byte_input(w):
    for b in range(256):
        got = oracle.pospopcnt(bytes([b]), w).tolist()
        assert got == oracle.pospopcnt_streams(bytes([b]), w), (w, b)


@pytest.mark.parametrize("w", (8, 16, 32))
def test_every_two_byte_input(w):
    for b0, b1 in itertools.product(range(256), repeat=2):
        data = bytes([b0, b1])
        assert oracle.pospopcnt(data, w).tolist() == oracle.pospopcnt_streams(data, w)


def test_three_byte_inputs_w32_sampled():
    rng = np.random.default_rng(11)
    for _ in range(4000):
        data = bytes(rng.integers(0, 256, size=3, dtype=np.uint8))
        assert oracle.pospopcnt(data, 32).tolist() == oracle.pospopcnt_streams(data, 32)


@pytest.mark.parametrize("w", WIDTHS)
def test_random_ragged_lengths(w):
    rng = np.random.default_rng(100 + w)
    for n in range(0, 65):
        for _ in range(6):
            data = bytes(rng.integers(0, 256, size=n, dtype=np.uint8))
            assert oracle.pospopcnt(data, w).tolist() == oracle.pospopcnt_streams(data, w), (w, n)


@pytest.mark.parametrize("w", WIDTHS)
def test_all_zero_is_zero(w):
    assert not oracle.pospopcnt(bytes(1000), w).any()


@pytest.mark.parametrize("w", WIDTHS)
@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 63, 64, 65, 1000])
def test_all_ones_counts_bytes_per_slot(w, n):
    s = w // 8
    got = oracle.pospopcnt(b"\xff" * n, w)
    # N_j: number of byte indices b < n with b mod s == j // 8
    want = [sum(1 for b in range(n) if b % s == j // 8) for j in range(w)]
    assert got.tolist() == want


@pytest.mark.parametrize("w", WIDTHS)
def test_single_set_bit(w):
    s = w // 8
    for n in (1, 5, 16, 17):
        for b in range(n):
            for k in range(8):
                data = bytearray(n)
                data[b] = 1 << k
                got = oracle.pospopcnt(bytes(data), w)
                want = np.zeros(w, dtype=np.uint64)
                want[8 * (b % s) + k] = 1
                assert (got == want).all(), (w, n, b, k)


@pytest.mark.parametrize("w", WIDTHS)
def test_periodic_pattern(w):
    s = w // 8
    rng = np.random.default_rng(5 + w)
    word = bytes(rng.integers(0, 256, size=s, dtype=np.uint8))
    reps = 37
    got = oracle.pospopcnt(word * reps, w)
    x = int.from_bytes(word, "little")
    want = [reps * ((x >> j) & 1) for j in range(w)]
    assert got.tolist() == want


@pytest.mark.parametrize("w", WIDTHS)
def test_counts_accumulate_not_clear(w):
    data = synth.random_bytes(333, seed=9)
    start = np.arange(w, dtype=np.uint64) * np.uint64(1000003) + np.uint64(2**40)
    acc = start.copy()
    oracle.pospopcnt(data, w, counts=acc)
    assert (acc - start == oracle.pospopcnt(data, w)).all()


def test_counter_wraps_mod_2_64():
    acc = np.full(8, np.iinfo(np.uint64).max, dtype=np.uint64)
    oracle.pospopcnt(b"\x01", 8, counts=acc)
    assert acc[0] == 0 and acc[1] == np.iinfo(np.uint64).max


@pytest.mark.parametrize("w", WIDTHS)
def test_multithreaded_equals_single(w):
    data = synth.random_bytes(100_003, seed=3)
    one = oracle.pospopcnt(data, w)
    for t in (1, 2, 3, 7, 16):
        assert (oracle.pospopcnt_mt(data, w, t) == one).all()


def test_empty_and_bad_arguments():
    for w in WIDTHS:
        assert not oracle.pospopcnt(b"", w).any()
    for bad in (0, 1, 4, 12, 24, 128):
        with pytest.raises(ValueError):
            oracle.pospopcnt(b"\x01", bad)


def test_popcount_matches_unpackbits():
    data = synth.random_bytes(5000, seed=21)
    assert oracle.popcount(data) == int(np.unpackbits(data).sum())


@pytest.mark.parametrize("w", WIDTHS)
def test_window_sweep_matches_the_streams_statement(w):
    """oracle.sweep (every window data[o:o+n]) is what the GPU sweep tests
    compare against: each of its windows must equal the independent
    interleaved-streams statement of Section 1 on the same bytes, laid out
    as (offset, length, counter)."""
    data = synth.random_bytes(40 + 9, seed=w)
    got = oracle.sweep(data, w, 40, 9)
    assert got.shape == (9, 41, w) and got.dtype == np.uint64
    for o in range(9):
        for n in range(41):
            assert got[o, n].tolist() == oracle.pospopcnt_streams(bytes(data[o:o + n]), w), (o, n)
    with pytest.raises(ValueError):
        oracle.sweep(data[:40], w, 40, 9)  # the last window would run past the buffer


def test_ranges_equal_the_streams_statement_per_range():
    """The threaded per-range helper (used to check full-size GPU batches)
    gives, range by range and in input order, what the interleaved-streams
    statement gives for that range alone."""
    data = synth.random_bytes(4096, seed=17)
    rng = np.random.default_rng(18)
    starts = rng.integers(0, 4000, size=300)
    lengths = [int(rng.integers(0, 4096 - s + 1)) % 97 for s in starts]
    widths = rng.choice(np.array(WIDTHS), size=300)
    got = oracle.pospopcnt_ranges(data, starts, lengths, widths, threads=4)
    assert len(got) == 300
    for g, s, n, w in zip(got, starts, lengths, widths):
        assert g.tolist() == oracle.pospopcnt_streams(data[int(s):int(s) + int(n)], int(w))


def test_ranges_reject_out_of_bounds_and_bad_widths():
    data = bytes(64)
    for bad in (([60], [5], [8]), ([-1], [2], [8]), ([0], [8], [12])):
        with pytest.raises(ValueError):
            oracle.pospopcnt_ranges(data, *bad)
