"""CPU checks of the seeded input generators shared by the tests and the
bench: same seed, same bytes; the stated shapes, bounds and laws hold."""
import math

import numpy as np

import synth

MiB = 1 << 20


def test_random_bytes_and_bernoulli_are_seeded():
    assert np.array_equal(synth.random_bytes(1000, 3), synth.random_bytes(1000, 3))
    assert not np.array_equal(synth.random_bytes(1000, 3), synth.random_bytes(1000, 4))
    a = synth.bernoulli(1 << 16, 0.1, seed=5)
    assert np.array_equal(a, synth.bernoulli(1 << 16, 0.1, seed=5))
    assert a.dtype == np.uint8 and a.size == 1 << 16


def test_bernoulli_density_and_bit_order():
    for p in (0.01, 0.3, 0.99):
        bits = np.unpackbits(synth.bernoulli(1 << 18, p, seed=1), bitorder="little")
        assert abs(bits.mean() - p) < 5 * math.sqrt(p * (1 - p) / bits.size)
    # p = 0.5 is plain uniform random bytes
    assert np.array_equal(synth.bernoulli(4096, 0.5, seed=2), synth.random_bytes(4096, 2))


def test_onehot_columns_hold_one_bit_per_word():
    pool, cats = synth.onehot_u32_columns(3, 5000, seed=4)
    words = pool.view("<u4")
    assert words.size == 15000 and cats.size == 15000
    assert np.array_equal(words, (np.uint32(1) << cats.astype(np.uint32)))
    assert cats.max() < 32
    u8, c8 = synth.onehot_u8(20000, seed=1)
    assert np.array_equal(u8, (1 << c8).astype(np.uint8)) and c8.max() < 8
    # the Zipf law: category 0 is the most frequent, about P(1) of the words
    p = synth.zipf_probs(8, 1.1)
    assert abs(np.mean(c8 == 0) - p[0]) < 0.02 and abs(p.sum() - 1.0) < 1e-12


def test_batch_spec_bounds_and_layout():
    spec = synth.batch_spec(2000, seed=3, lo=16, hi=16 * MiB, align=256, start_jitter=64)
    off, ln, w = spec["offsets"], spec["lengths"], spec["widths"]
    assert set(np.unique(w)) <= {8, 16, 32, 64}
    assert np.all(ln % (w // 8) == 0) and np.all(ln >= w // 8) and np.all(ln <= 16 * MiB)
    assert np.all((off % 256) < 64)  # aligned start plus jitter
    assert np.all(off[1:] >= off[:-1] + ln[:-1])  # arrays do not overlap
    assert spec["pool_bytes"] >= int(off[-1] + ln[-1])
    assert np.all((spec["p"] >= 0) & (spec["p"] <= 1))
    again = synth.batch_spec(2000, seed=3, lo=16, hi=16 * MiB, align=256, start_jitter=64)
    assert all(np.array_equal(spec[k], again[k]) for k in ("offsets", "lengths", "widths", "p"))


def test_serve_trace_requests_stay_inside_their_columns():
    col = 64 * MiB
    t = synth.serve_trace(20000, seed=4, n_columns=16, column_bytes=col, rate_per_s=1e6, lo=64, hi=64 * MiB)
    assert np.all((t["column"] >= 0) & (t["column"] < 16))
    assert np.all((t["length"] >= 64) & (t["length"] <= col))
    assert np.all(t["offset"] >= 0) and np.all(t["offset"] + t["length"] <= col)
    assert set(np.unique(t["width"])) <= {8, 16, 32, 64}
    gaps = np.diff(t["arrival_ns"])
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() / 1e3 - 1.0) < 0.05  # Poisson arrivals at 1 per microsecond


def test_log_uniform_mean_matches_sampling():
    rng = np.random.default_rng(0)
    x = np.exp(rng.uniform(math.log(64), math.log(64 * MiB), size=400000))
    assert abs(x.mean() / synth.log_uniform_mean(64, 64 * MiB) - 1.0) < 0.02
