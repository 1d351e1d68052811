"""GPU parity of the plain call (C-ABI ppc_pospopcnt*) against the oracle.

Tolerance is zero: the counts are integers and every case must be equal to
the oracle bit for bit.  Cases:
  * 2 MiB, w = 16, random bits, seed 0 (the single-call workload);
  * every length 0..4096 at every start offset 0..63 at all four widths,
    inside 0xFF guard bytes, plus the same sweep on the complemented buffer
    so that any byte read outside the window changes some count;
  * 256 MiB at every width and densities 0.01 / 0.5 / 0.99, in the launch
    geometry the benchmark times;
  * a 64 MiB one-hot column (counts equal the category histogram);
  * small grids that force many overflow segments per wave;
  * a buffer just over 4 GiB with a ragged tail;
  * an input over one launch's tile budget (16 GiB at a one-wave grid),
    split into two launches;
  * accumulation into non-zero counters, repeatability, side streams.
"""
import ctypes

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


@pytest.fixture
def geometry(ppc):
    saved = ppc.ppc_get_plain_geometry()
    ppc.ppc_set_plain_geometry(0, 8)
    yield ppc
    ppc.ppc_set_plain_geometry(0, saved[1])


def dev():
    return torch.device("cuda:0")


def run(ppc, w, buf, n=None):
    counts = torch.zeros(w, dtype=torch.int64, device=dev())
    ppc.ppc_pospopcnt(w, counts, buf, n)
    torch.cuda.synchronize()
    return ppc.counts_to_numpy(counts)


def test_single_call_2MiB_w16(geometry):
    ppc = geometry
    host = synth.random_bytes(1 << 21, seed=0)
    got = run(ppc, 16, torch.from_numpy(host).to(dev()))
    assert np.array_equal(got, oracle.pospopcnt(host, 16))


def test_width_entry_points_agree(geometry):
    ppc = geometry
    host = synth.random_bytes(123_457, seed=12)
    buf = torch.from_numpy(host).to(dev())
    fns = {8: ppc.ppc_pospopcnt8, 16: ppc.ppc_pospopcnt16, 32: ppc.ppc_pospopcnt32,
           64: ppc.ppc_pospopcnt64}
    for w, fn in fns.items():
        counts = torch.zeros(w, dtype=torch.int64, device=dev())
        fn(counts, buf[3:])
        torch.cuda.synchronize()
        assert np.array_equal(ppc.counts_to_numpy(counts), oracle.pospopcnt(host[3:], w))


GUARD_LO, GUARD_HI = 64, 128
MAX_LEN, N_OFF = 4096, 64


def _sweep(ppc, w, region):
    """Every window region[o:o+n] through the plain C entry point, each into
    its own counter row; returns (n_off, max_len+1, w) uint64."""
    host = np.concatenate([np.full(GUARD_LO, 0xFF, np.uint8), region,
                           np.full(GUARD_HI, 0xFF, np.uint8)])
    buf = torch.from_numpy(host).to(dev())
    rows = N_OFF * (MAX_LEN + 1)
    counts = torch.zeros((rows, w), dtype=torch.int64, device=dev())
    base = buf.data_ptr() + GUARD_LO
    cbase = counts.data_ptr()
    fn = ppc.lib().ppc_pospopcnt
    stream = torch.cuda.current_stream().cuda_stream
    row = 0
    for o in range(N_OFF):
        for n in range(MAX_LEN + 1):
            rc = fn(w, cbase + row * w * 8, base + o, n, stream)
            if rc != 0:
                raise AssertionError("status %d at w=%d o=%d n=%d" % (rc, w, o, n))
            row += 1
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), host)  # input untouched
    return ppc.counts_to_numpy(counts).reshape(N_OFF, MAX_LEN + 1, w)


@pytest.mark.parametrize("w", WIDTHS)
def test_every_short_length_and_offset(geometry, w):
    region = synth.random_bytes(MAX_LEN + N_OFF, seed=2)
    got = _sweep(geometry, w, region)
    want = oracle.sweep(region, w, MAX_LEN, N_OFF)
    bad = np.argwhere((got != want).any(axis=2))
    assert bad.size == 0, "first mismatches (offset, length): %s" % bad[:5].tolist()


def test_every_short_length_and_offset_complemented(geometry):
    region = ~synth.random_bytes(MAX_LEN + N_OFF, seed=2)
    got = _sweep(geometry, 16, region)
    assert np.array_equal(got, oracle.sweep(region, 16, MAX_LEN, N_OFF))


@pytest.mark.parametrize("w", WIDTHS)
@pytest.mark.parametrize("p", [0.01, 0.5, 0.99])
def test_256MiB_each_width_and_density(geometry, w, p):
    n = 1 << 28
    buf = synth.device_bernoulli(n, p, seed=1, device=dev())
    got = run(geometry, w, buf)
    host = buf.cpu().numpy()
    assert np.array_equal(got, oracle.pospopcnt_mt(host, w, HOST_THREADS))


def test_onehot_64MiB_equals_histogram(geometry):
    data, cats = synth.onehot_u8(1 << 26, seed=2)
    buf = torch.from_numpy(data).to(dev())
    hist = np.bincount(cats, minlength=8).astype(np.uint64)
    assert np.array_equal(run(geometry, 8, buf), hist)
    for w in (16, 32, 64):
        got = run(geometry, w, buf)
        assert np.array_equal(got.reshape(w // 8, 8).sum(axis=0), hist)


@pytest.mark.parametrize("waves,wpb", [(1, 2), (3, 4), (64, 8), (700, 2), (1000, 8), (4096, 4), (20000, 8)])
def test_small_grids_force_many_segments(geometry, waves, wpb):
    ppc = geometry
    ppc.ppc_set_plain_geometry(waves, wpb)
    host = synth.random_bytes((32 << 20) + 77, seed=waves)
    buf = torch.from_numpy(host).to(dev())
    for w, off in ((8, 0), (64, 9)):  # aligned and unaligned starts
        got = run(ppc, w, buf[off:])
        assert np.array_equal(got, oracle.pospopcnt_mt(host[off:], w, HOST_THREADS))


@pytest.mark.parametrize("waves,wpb", [(1, 2), (8, 8), (64, 4)])
def test_total_popcount_on_small_grids(geometry, waves, wpb):
    """The total popcount with each wave walking hundreds of tiles (several
    segment flushes of its per-lane totals), aligned and unaligned starts."""
    ppc = geometry
    ppc.ppc_set_plain_geometry(waves, wpb)
    host = synth.random_bytes((32 << 20) + 77, seed=100 + waves)
    buf = torch.from_numpy(host).to(dev())
    for off in (0, 9):
        total = torch.zeros(1, dtype=torch.int64, device=dev())
        ppc.ppc_popcount(total, buf[off:])
        torch.cuda.synchronize()
        assert int(ppc.counts_to_numpy(total)[0]) == int(np.unpackbits(host[off:]).sum()), (waves, wpb, off)


def test_just_over_4GiB_ragged(geometry):
    n = (4 << 30) + 4099
    buf = synth.device_bernoulli(n, 0.5, seed=7, device=dev())
    got = run(geometry, 64, buf[5:])
    host = buf.cpu().numpy()
    want = oracle.pospopcnt_mt(host[5:], 64, HOST_THREADS)
    del buf
    assert np.array_equal(got, want)


def test_input_split_into_several_launches(geometry):
    """A launch gives no wave more than 2^20 tiles of 16 KiB (its 32-bit
    counts stay below 2^31).  With the grid capped at one wave the budget is
    16 GiB per launch, so 16 GiB + 12,345 bytes from an unaligned start takes
    two launches with the same pointer residue."""
    ppc = geometry
    ppc.ppc_set_plain_geometry(1, 2)
    n = (16 << 30) + 12345 + 5
    buf = synth.device_bernoulli(n, 0.5, seed=17, device=dev())
    got = run(ppc, 32, buf[5:])
    host = buf.cpu().numpy()
    del buf
    torch.cuda.empty_cache()
    want = oracle.pospopcnt_mt(host[5:], 32, HOST_THREADS)
    assert np.array_equal(got, want)


def test_accumulates_into_existing_counts(geometry):
    ppc = geometry
    host = synth.random_bytes(1_000_003, seed=4)
    buf = torch.from_numpy(host).to(dev())
    start = (np.arange(32, dtype=np.uint64) * np.uint64(7919) + np.uint64(1 << 50))
    counts = torch.from_numpy(start.view(np.int64).copy()).to(dev())
    ppc.ppc_pospopcnt32(counts, buf[1:])
    ppc.ppc_pospopcnt32(counts, buf[1:])
    torch.cuda.synchronize()
    want = start + 2 * oracle.pospopcnt(host[1:], 32)
    assert np.array_equal(ppc.counts_to_numpy(counts), want)


def test_repeatable_and_on_a_side_stream(geometry):
    ppc = geometry
    host = synth.bernoulli(3_000_001, 0.2, seed=8)
    buf = torch.from_numpy(host).to(dev())
    s = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        counts = torch.zeros(16, dtype=torch.int64, device=dev())
        with torch.cuda.stream(s):
            ppc.ppc_pospopcnt16(counts, buf[7:])
        s.synchronize()
        outs.append(ppc.counts_to_numpy(counts))
    want = oracle.pospopcnt(host[7:], 16)
    for o in outs:
        assert np.array_equal(o, want)


def test_host_threads_on_their_own_streams(geometry):
    """Plain calls from four host threads at once (ctypes drops the GIL for
    the call), each thread on its own stream; every thread adds into its own
    counters and into one shared set (atomics commute), 25 calls each."""
    import threading

    ppc = geometry
    host = [synth.random_bytes((3 << 20) + 11 * k, seed=90 + k) for k in range(4)]
    bufs = [torch.from_numpy(h).to(dev()) for h in host]
    own = [torch.zeros(16, dtype=torch.int64, device=dev()) for _ in range(4)]
    shared = torch.zeros(16, dtype=torch.int64, device=dev())
    streams = [torch.cuda.Stream() for _ in range(4)]
    torch.cuda.synchronize()
    errors = []

    def work(k):
        try:
            for _ in range(25):
                ppc.ppc_pospopcnt16(own[k], bufs[k][k:], stream=streams[k])
                ppc.ppc_pospopcnt16(shared, bufs[k][k:], stream=streams[k])
        except Exception as e:  # reported below, in the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors
    want = [oracle.pospopcnt(h[k:], 16) for k, h in enumerate(host)]
    for k in range(4):
        assert np.array_equal(ppc.counts_to_numpy(own[k]), want[k] * np.uint64(25))
    assert np.array_equal(ppc.counts_to_numpy(shared), sum(want) * np.uint64(25))


def test_errors_reported_not_raised_on_device(geometry):
    ppc = geometry
    buf = torch.zeros(64, dtype=torch.uint8, device=dev())
    counts = torch.zeros(16, dtype=torch.int64, device=dev())
    lib = ppc.lib()
    st = torch.cuda.current_stream().cuda_stream
    assert lib.ppc_pospopcnt(24, counts.data_ptr(), buf.data_ptr(), 64, st) == ppc.PPC_EINVAL
    assert lib.ppc_pospopcnt(16, counts.data_ptr() + 4, buf.data_ptr(), 64, st) == ppc.PPC_EINVAL
    assert lib.ppc_pospopcnt(16, counts.data_ptr(), None, 64, st) == ppc.PPC_EINVAL
    assert lib.ppc_pospopcnt(16, counts.data_ptr(), None, 0, st) == ppc.PPC_OK
    with pytest.raises(ValueError):
        ppc.ppc_pospopcnt16(counts, torch.zeros(8, dtype=torch.uint8))  # host tensor
    torch.cuda.synchronize()
    assert not counts.any()


def test_read_roofline_sums_words(geometry):
    ppc = geometry
    n = 64 << 20
    host = synth.random_bytes(n, seed=5)
    buf = torch.from_numpy(host).to(dev())
    sink = torch.zeros(1, dtype=torch.int64, device=dev())
    ppc.ppc_read_roofline(sink, buf)
    torch.cuda.synchronize()
    want = int(host.view("<u8").sum(dtype=np.uint64))
    assert int(sink.cpu().numpy().view(np.uint64)[0]) == want


def test_timed_entry_points_record_the_kernel(geometry):
    ppc = geometry
    host = synth.random_bytes((48 << 20) + 9, seed=13)
    buf = torch.from_numpy(host).to(dev())
    for w in (8, 64):
        counts = torch.zeros(w, dtype=torch.int64, device=dev())
        a, b = ppc.HipEvent(), ppc.HipEvent()
        ppc.ppc_pospopcnt_timed(w, counts, buf[1:], start_event=a, stop_event=b)
        torch.cuda.synchronize()
        assert np.array_equal(ppc.counts_to_numpy(counts), oracle.pospopcnt_mt(host[1:], w, HOST_THREADS))
        assert 0.0 < a.elapsed_ms(b) < 1000.0
    sink = torch.zeros(1, dtype=torch.int64, device=dev())
    a, b = ppc.HipEvent(), ppc.HipEvent()
    ppc.ppc_read_roofline_timed(sink, buf[:48 << 20], start_event=a, stop_event=b)
    torch.cuda.synchronize()
    assert int(sink.cpu().numpy().view(np.uint64)[0]) == int(host[:48 << 20].view("<u8").sum(dtype=np.uint64))
    assert 0.0 < a.elapsed_ms(b) < 1000.0
    # no events at all, and nothing launched for an empty input
    counts = torch.zeros(16, dtype=torch.int64, device=dev())
    ppc.ppc_pospopcnt_timed(16, counts, buf[:0])
    ppc.ppc_pospopcnt_timed(16, counts, buf[:100])
    torch.cuda.synchronize()
    assert np.array_equal(ppc.counts_to_numpy(counts), oracle.pospopcnt(host[:100], 16))
