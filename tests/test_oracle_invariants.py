"""Invariants and applications that pin the oracle (exact, at any size).

* sum(counts) = total popcount (Section 1: pospopcnt generalises popcount).
* Complement: counts(~x) = N - counts(x).
* Additivity over concatenation with the word-slot rotation (the streamed
  accumulation of Section 4, step 1 footnote).
* Folding: counts_w[j] = counts_2w[j] + counts_2w[j+w] (one kernel, the width
  is only applied by the accumulation function, Section 5).
* One-hot columns: counts equal the category histogram (Section 1).
* The paper's worked examples in tests/golden/.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth

WIDTHS = (8, 16, 32, 64)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rotate_slots(counts: np.ndarray, q: int) -> np.ndarray:
    """Counts of a piece that starts q bytes into a word: byte slot a of the
    piece lands in slot (a + q) mod s of the whole."""
    w = counts.size
    s = w // 8
    out = np.zeros_like(counts)
    for a in range(s):
        for k in range(8):
            out[8 * ((a + q) % s) + k] = counts[8 * a + k]
    return out


@pytest.mark.parametrize("w", WIDTHS)
@pytest.mark.parametrize("n", [0, 1, 3, 64, 1001, 65536 + 5])
def test_sum_is_total_popcount(w, n):
    data = synth.random_bytes(n, seed=n)
    assert int(oracle.pospopcnt(data, w).sum()) == int(np.unpackbits(data).sum())


@pytest.mark.parametrize("w", WIDTHS)
@pytest.mark.parametrize("n", [1, 2, 7, 8, 100, 4099])
def test_complement(w, n):
    s = w // 8
    data = synth.bernoulli(n, 0.3, seed=n)
    n_j = np.array([len(range(j // 8, n, s)) for j in range(w)], dtype=np.uint64)
    assert (oracle.pospopcnt(~data, w) == n_j - oracle.pospopcnt(data, w)).all()


@pytest.mark.parametrize("w", WIDTHS)
def test_additivity_over_concatenation(w):
    rng = np.random.default_rng(w)
    for _ in range(40):
        a = synth.random_bytes(int(rng.integers(0, 80)), seed=int(rng.integers(1 << 30)))
        b = synth.random_bytes(int(rng.integers(0, 80)), seed=int(rng.integers(1 << 30)))
        whole = oracle.pospopcnt(np.concatenate([a, b]), w)
        parts = oracle.pospopcnt(a, w) + rotate_slots(oracle.pospopcnt(b, w), a.size % (w // 8))
        assert (whole == parts).all()


@pytest.mark.parametrize("w", (8, 16, 32))
def test_fold_to_half_width(w):
    for n in (0, 1, 5, 17, 1000, 4097):
        data = synth.random_bytes(n, seed=7 * n + w)
        wide = oracle.pospopcnt(data, 2 * w)
        assert (oracle.pospopcnt(data, w) == wide[:w] + wide[w:]).all()


@pytest.mark.parametrize("w", WIDTHS)
def test_misaligned_views_match_stream_definition(w):
    base = synth.random_bytes(300, seed=77)
    for off in range(0, 64):
        view = base[off:off + 131]
        assert oracle.pospopcnt(view, w).tolist() == oracle.pospopcnt_streams(view, w)


def test_onehot_counts_equal_histogram():
    data, cats = synth.onehot_u8(200_000, seed=2)
    hist = np.bincount(cats, minlength=8)
    assert (oracle.pospopcnt(data, 8) == hist).all()
    for w in (16, 32, 64):
        c = oracle.pospopcnt(data, w).reshape(w // 8, 8).sum(axis=0)
        assert (c == hist).all()


def test_onehot_u32_columns_histogram():
    pool, cats = synth.onehot_u32_columns(2, 5000, seed=4)
    assert (oracle.pospopcnt(pool, 32) == np.bincount(cats, minlength=32)).all()


# ---- the paper's worked examples ---------------------------------------
def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_full_adder_worked_example():
    for a, b, c, carry, total in _rows("full_adder_example.txt"):
        got = oracle.full_adder(int(a, 2), int(b, 2), int(c, 2))
        assert got == (int(carry, 2), int(total, 2))


def test_full_adder_truth_tables():
    tables = {r[0]: int(r[1], 16) for r in _rows("truth_tables.txt")}
    par = maj = mux = 0
    for a, b, c in itertools.product((0, 1), repeat=3):
        idx = 4 * a + 2 * b + c
        carry, total = oracle.full_adder(a, b, c)
        par |= total << idx
        maj |= carry << idx
        mux |= (b if a else c) << idx
    assert par == tables["parity"]
    assert maj == tables["majority"]
    assert mux == tables["mux"]


def test_mux_carry_form_equals_full_adder_carry():
    # Eq. mux: the carry is (a xor b) ? c : b; pinned against the arithmetic
    # definition on every 3-bit column of two random 16-bit vectors sets.
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c = (int(x) for x in rng.integers(0, 1 << 16, size=3))
        carry, total = oracle.full_adder(a, b, c)
        t = a ^ b
        assert carry == ((t & c) | (~t & b)) & 0xFFFF
        assert total == a ^ b ^ c


def test_carry_save_network_of_full_adders_keeps_place_values():
    # Sections 3.2-3.3: a 4-bit carry-save accumulator (planes of weight
    # 1, 2, 4, 8) takes 16 vectors through 15 full adders arranged as
    # pairs -> twos -> fours -> eights and emits a plane of weight 16.  For
    # every bit column, the weighted planes after the step must equal the
    # weighted planes before it plus the number of input vectors with that
    # bit set.  The column counts come from numpy's bit unpacking, not from
    # the full adder, so a wrong carry weight, a swapped carry/sum or a
    # dropped input fails here.
    rng = np.random.default_rng(3)
    nbits = 32
    for _ in range(50):
        vecs = [int(x) for x in rng.integers(0, 1 << nbits, size=16, dtype=np.uint64)]
        a1, a2, a4, a8 = (int(x) for x in rng.integers(0, 1 << nbits, size=4, dtype=np.uint64))
        before = [((a1 >> i) & 1) + 2 * ((a2 >> i) & 1) + 4 * ((a4 >> i) & 1) + 8 * ((a8 >> i) & 1)
                  for i in range(nbits)]
        fa = oracle.full_adder
        twos, fours, eights = [], [], []
        for k in range(0, 16, 2):
            c, a1 = fa(a1, vecs[k], vecs[k + 1])
            twos.append(c)
        for k in range(0, 8, 2):
            c, a2 = fa(a2, twos[k], twos[k + 1])
            fours.append(c)
        for k in range(0, 4, 2):
            c, a4 = fa(a4, fours[k], fours[k + 1])
            eights.append(c)
        a16, a8 = fa(a8, eights[0], eights[1])
        planes = np.array(vecs, dtype="<u4").view(np.uint8).reshape(16, 4)
        column = np.unpackbits(planes, axis=1, bitorder="little").sum(axis=0)
        for i in range(nbits):
            after = sum(((p >> i) & 1) << e for e, p in enumerate((a1, a2, a4, a8, a16)))
            assert after == before[i] + int(column[i]), "bit column %d" % i


def test_onehot_age_example():
    rows = _rows("onehot_age_example.txt")
    data = bytes(int(word, 2) for word, _ in rows)
    hist = np.bincount([int(cat) for _, cat in rows], minlength=8)
    assert (oracle.pospopcnt(data, 8) == hist).all()
