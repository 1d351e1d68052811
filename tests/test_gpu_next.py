"""GPU parity of the follow-on forms: streamed pieces, the total popcount
and every size of the paper's length sweep (Section 5.2: 2^i and 3*2^i
bytes), all bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDTHS = (8, 16, 32, 64)
HOST_THREADS = 16


@pytest.fixture(scope="module")
def ppc():
    import paper_2412_16370_amd as ppc

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ppc.lib()
    return ppc


def dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("w", WIDTHS)
def test_streamed_pieces_cut_anywhere_add_up(ppc, w):
    n = 10_000_019
    host = synth.bernoulli(n, 0.4, seed=50 + w)
    buf = torch.from_numpy(host).to(dev())
    rng = np.random.default_rng(w)
    cuts = np.unique(np.concatenate([[0, n], rng.integers(0, n, size=60), rng.integers(0, 64, size=5)]))
    pieces = list(zip(cuts[:-1], cuts[1:]))
    rng.shuffle(pieces)  # order does not matter
    counts = torch.zeros(w, dtype=torch.int64, device=dev())
    for a, b in pieces:
        ppc.ppc_pospopcnt_at(w, counts, buf[int(a):int(b)], stream_offset=int(a))
    torch.cuda.synchronize()
    assert np.array_equal(ppc.counts_to_numpy(counts), oracle.pospopcnt(host, w))


def test_stream_offset_rotates_slots(ppc):
    host = synth.random_bytes(4099, seed=51)
    buf = torch.from_numpy(host).to(dev())
    for w in WIDTHS:
        for off in range(0, 9):
            counts = torch.zeros(w, dtype=torch.int64, device=dev())
            ppc.ppc_pospopcnt_at(w, counts, buf[3:], stream_offset=off)
            torch.cuda.synchronize()
            # the same bytes preceded by `off` zero bytes, counted from the start
            want = oracle.pospopcnt(np.concatenate([np.zeros(off, np.uint8), host[3:]]), w)
            assert np.array_equal(ppc.counts_to_numpy(counts), want), (w, off)


@pytest.mark.parametrize("n,off", [(0, 0), (1, 0), (15, 1), (31, 7), (4096, 3), (1_000_003, 5),
                                   ((64 << 20) + 11, 0), (1 << 28, 0)])
def test_total_popcount(ppc, n, off):
    buf = synth.device_bernoulli(n + off, 0.3, seed=52, device=dev())
    total = torch.zeros(1, dtype=torch.int64, device=dev())
    ppc.ppc_popcount(total, buf[off:off + n])
    torch.cuda.synchronize()
    host = buf.cpu().numpy()[off:off + n]
    got = int(ppc.counts_to_numpy(total)[0])
    if n < (1 << 26):
        assert got == int(np.unpackbits(host).sum())
    else:  # sum of the 64 positional counts = total popcount
        assert got == int(oracle.pospopcnt_mt(host, 64, HOST_THREADS).sum())


def test_total_popcount_small_cases_against_oracle(ppc):
    host = synth.random_bytes(20_000, seed=53)
    buf = torch.from_numpy(host).to(dev())
    rng = np.random.default_rng(54)
    for _ in range(200):
        a = int(rng.integers(0, 10_000))
        b = a + int(rng.integers(0, 10_000))
        total = torch.zeros(1, dtype=torch.int64, device=dev())
        ppc.ppc_popcount(total, buf[a:b])
        torch.cuda.synchronize()
        assert int(ppc.counts_to_numpy(total)[0]) == oracle.popcount(host[a:b])


def sweep_sizes(limit):
    sizes = [1 << i for i in range(1, 31)] + [3 << i for i in range(0, 30)]
    return sorted(s for s in sizes if s <= limit)


def test_every_size_of_the_length_sweep(ppc):
    top = 3 << 29  # 1.5 GiB
    buf = synth.device_bernoulli(top + 64, 0.5, seed=55, device=dev())
    host = buf.cpu().numpy()
    for n in sweep_sizes(top):
        for w in WIDTHS:
            off = (n * 7 + w) % 64
            counts = torch.zeros(w, dtype=torch.int64, device=dev())
            ppc.ppc_pospopcnt(w, counts, buf[off:off + n])
            torch.cuda.synchronize()
            view = host[off:off + n]
            want = oracle.pospopcnt(view, w) if n < (1 << 22) else oracle.pospopcnt_mt(view, w, HOST_THREADS)
            assert np.array_equal(ppc.counts_to_numpy(counts), want), (n, w, off)
