"""GPU parity of the batched form (ppc_plan_*) against the oracle and the plain call.

Every array of a batch must get exactly the counts the oracle gives for its
bytes and width (tolerance 0), and exactly what a plain call adds.  Arrays
sit in one pool filled with 0xFF between them, so a read outside any array
changes some count.
"""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(scope="module")
def ppc():
    import paper_2412_16370_amd as ppc

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ppc.lib()
    return ppc


def dev():
    return torch.device("cuda:0")


def make_pool(spec, seed):
    """Device pool with array i at spec offsets[i], Bernoulli(p_i) bits, 0xFF
    between arrays."""
    pool = torch.full((spec["pool_bytes"] + 128,), 0xFF, dtype=torch.uint8, device=dev())
    for i, (off, n, p) in enumerate(zip(spec["offsets"], spec["lengths"], spec["p"])):
        if n:
            synth.device_bernoulli(int(n), float(p), seed=seed * 1_000_003 + i, device=dev(),
                                   out=pool[int(off):int(off) + int(n)])
    torch.cuda.synchronize()
    return pool


def plan_for(ppc, pool, spec, counts, opts=None):
    n = len(spec["lengths"])
    base, cbase = pool.data_ptr(), counts.data_ptr()
    descs = ppc.make_descs([base + int(o) for o in spec["offsets"]], spec["lengths"],
                           [cbase + i * 64 * 8 for i in range(n)], spec["widths"])
    return ppc.ppc_plan_create(descs, n, opts)


def plain_counts(ppc, pool, spec):
    n = len(spec["lengths"])
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    lib = ppc.lib()
    st = torch.cuda.current_stream().cuda_stream
    base, cbase = pool.data_ptr(), counts.data_ptr()
    for i in range(n):
        rc = lib.ppc_pospopcnt(int(spec["widths"][i]), cbase + i * 512, base + int(spec["offsets"][i]),
                               int(spec["lengths"][i]), st)
        assert rc == 0
    torch.cuda.synchronize()
    return ppc.counts_to_numpy(counts)


def oracle_rows(host_pool, spec, idx):
    rows = {}
    for i in idx:
        o, n, w = int(spec["offsets"][i]), int(spec["lengths"][i]), int(spec["widths"][i])
        rows[i] = oracle.pospopcnt(host_pool[o:o + n], w)
    return rows


def check_rows(got, spec, want_rows, reps=1):
    for i, want in want_rows.items():
        w = int(spec["widths"][i])
        assert np.array_equal(got[i, :w], want * np.uint64(reps)), "array %d (w=%d, n=%d)" % (
            i, w, int(spec["lengths"][i]))
        assert not got[i, w:].any(), "array %d wrote past its %d counters" % (i, w)


def opts(ppc, tiles=0, waves=0, autotune=0, graph=1):
    return ppc.ppc_plan_opts(tiles, waves, autotune, graph, 0)


def test_mixed_batch_unaligned_starts(ppc):
    spec = synth.batch_spec(3000, seed=30, lo=16, hi=1 * MiB, start_jitter=64)
    pool = make_pool(spec, seed=30)
    counts = torch.zeros((3000, 64), dtype=torch.int64, device=dev())
    plan = plan_for(ppc, pool, spec, counts, opts(ppc, tiles=4))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
        info = ppc.ppc_plan_get_info(plan)
    finally:
        ppc.ppc_plan_destroy(plan)
    assert info["n_arrays"] == 3000 and info["tiles_per_item"] == 4 and info["graph"] == 1
    assert info["n_items"] > 3000  # large arrays were split
    got = ppc.counts_to_numpy(counts).reshape(3000, 64)
    check_rows(got, spec, oracle_rows(pool.cpu().numpy(), spec, range(3000)))
    assert np.array_equal(got, plain_counts(ppc, pool, spec))


def test_edge_only_and_empty_arrays(ppc):
    # every length 0..40 at every start offset 0..15, all widths
    offs, lens, widths = [], [], []
    pos = 0
    for w in (8, 16, 32, 64):
        for o in range(16):
            for n in range(41):
                offs.append(pos + o)
                lens.append(n)
                widths.append(w)
                pos += 128
    spec = dict(offsets=np.array(offs), lengths=np.array(lens), widths=np.array(widths),
                p=np.full(len(lens), 0.5), pool_bytes=pos + 128)
    pool = make_pool(spec, seed=31)
    n = len(lens)
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    plan = plan_for(ppc, pool, spec, counts, opts(ppc, graph=0))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
    finally:
        ppc.ppc_plan_destroy(plan)
    got = ppc.counts_to_numpy(counts).reshape(n, 64)
    check_rows(got, spec, oracle_rows(pool.cpu().numpy(), spec, range(n)))


def test_autotuned_plan_replays_and_cache(ppc, tmp_path, monkeypatch):
    monkeypatch.setenv("PPC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    spec = synth.batch_spec(800, seed=32, lo=16, hi=4 * MiB)
    assert spec["pool_bytes"] > 64 * MiB  # large enough to be tuned
    pool = make_pool(spec, seed=32)
    counts = torch.zeros((800, 64), dtype=torch.int64, device=dev())
    plan = plan_for(ppc, pool, spec, counts)  # default options: autotune + graph
    try:
        info = ppc.ppc_plan_get_info(plan)
        assert info["tuned"] == 1 and info["graph"] == 1
        # graph replays with eager work and synchronisations in between
        scratch = torch.zeros(1 << 20, device=dev())
        for r in range(3):
            ppc.ppc_plan_run(plan)
            scratch.add_(1.0)
            torch.cuda.synchronize()
            got = ppc.counts_to_numpy(counts).reshape(800, 64)
            if r == 0:
                want = oracle_rows(pool.cpu().numpy(), spec, range(800))
            check_rows(got, spec, want, reps=r + 1)
    finally:
        ppc.ppc_plan_destroy(plan)
    counts2 = torch.zeros((800, 64), dtype=torch.int64, device=dev())
    plan2 = plan_for(ppc, pool, spec, counts2)
    try:
        info2 = ppc.ppc_plan_get_info(plan2)
        assert info2["tuned"] == 2
        assert (info2["tiles_per_item"], info2["waves"]) == (info["tiles_per_item"], info["waves"])
    finally:
        ppc.ppc_plan_destroy(plan2)
    assert not counts2.any()  # tuning never touched the caller's counters


def test_ten_thousand_arrays_full_size(ppc, tmp_path, monkeypatch):
    """10,000 arrays, log-uniform 16 B .. 16 MiB, mixed widths, p ~ U[0,1]
    (11.95 GB): every array's counts equal the oracle on its bytes (threads
    over the host cores, one Fig. 2 loop per array) and what a plain call
    adds for it."""
    monkeypatch.setenv("PPC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    spec = synth.batch_spec(10_000, seed=3)
    pool = make_pool(spec, seed=3)
    counts = torch.zeros((10_000, 64), dtype=torch.int64, device=dev())
    plan = plan_for(ppc, pool, spec, counts)
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
    finally:
        ppc.ppc_plan_destroy(plan)
    got = ppc.counts_to_numpy(counts).reshape(10_000, 64)
    assert np.array_equal(got, plain_counts(ppc, pool, spec))
    host = pool.cpu().numpy()
    del pool
    torch.cuda.empty_cache()
    want = oracle.pospopcnt_ranges(host, spec["offsets"], spec["lengths"], spec["widths"])
    check_rows(got, spec, dict(enumerate(want)))


def test_empty_plan_and_bad_descriptors(ppc):
    plan = ppc.ppc_plan_create(ppc.make_descs([], [], [], []), 0, None)
    ppc.ppc_plan_run(plan)
    torch.cuda.synchronize()
    assert ppc.ppc_plan_get_info(plan)["n_items"] == 0
    ppc.ppc_plan_destroy(plan)
    buf = torch.zeros(64, dtype=torch.uint8, device=dev())
    counts = torch.zeros(64, dtype=torch.int64, device=dev())
    for bad in ([buf.data_ptr()], [64], [counts.data_ptr() + 4], [16]), \
               ([buf.data_ptr()], [64], [counts.data_ptr()], [7]), \
               ([None], [64], [counts.data_ptr()], [8]):
        with pytest.raises(ppc.PpcError) as e:
            ppc.ppc_plan_create(ppc.make_descs(*bad), 1, None)
        assert e.value.status == ppc.PPC_EINVAL
    torch.cuda.synchronize()
    assert not counts.any()


@pytest.mark.parametrize("w", (8, 16, 32, 64))
def test_every_short_length_and_offset_in_one_plan(ppc, w):
    """The short sweep of the plain-call tests -- every length 0..4096 at
    every start offset 0..63, between 0xFF guard bytes -- as ONE batched
    plan of 262,208 arrays, run twice (the replay adds the same counts
    again).  Covers the plan's small-array kernel on empty arrays,
    head/tail-only arrays, single-chunk arrays and partial tiles; the
    batched walk's own short paths are covered by
    test_walk_short_paths_on_last_items."""
    max_len, n_off, lo, hi = 4096, 64, 64, 128
    region = synth.random_bytes(max_len + n_off, seed=2)
    host = np.concatenate([np.full(lo, 0xFF, np.uint8), region, np.full(hi, 0xFF, np.uint8)])
    buf = torch.from_numpy(host).to(dev())
    rows = n_off * (max_len + 1)
    counts = torch.zeros((rows, w), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr() + lo, counts.data_ptr()
    addrs = [base + o for o in range(n_off) for _ in range(max_len + 1)]
    lens = [n for _ in range(n_off) for n in range(max_len + 1)]
    descs = ppc.make_descs(addrs, lens, [cbase + r * w * 8 for r in range(rows)], [w] * rows)
    plan = ppc.ppc_plan_create(descs, rows, ppc.ppc_plan_opts(16, 0, 0, 1, 0))
    try:
        want = oracle.sweep(region, w, max_len, n_off)
        for rep in (1, 2):
            ppc.ppc_plan_run(plan)
            torch.cuda.synchronize()
            got = ppc.counts_to_numpy(counts).reshape(n_off, max_len + 1, w)
            bad = np.argwhere((got != want * np.uint64(rep)).any(axis=2))
            assert bad.size == 0, "run %d, first mismatches (offset, length): %s" % (rep, bad[:5].tolist())
    finally:
        ppc.ppc_plan_destroy(plan)
    assert np.array_equal(buf.cpu().numpy(), host)  # input untouched


@pytest.mark.parametrize("w", (8, 16, 32, 64))
def test_partial_tiles_of_4_to_16_KiB(ppc, w):
    """Arrays of 4,080..16,392 bytes (every 8th length) at start offsets 0, 3,
    16 and 63: at most one tile, 4..16 chunks per lane, counted by one plan
    (its small-array kernel) and, every 17th length, by plain calls (the
    walk's short partial-tile path up to 14 chunks per lane, the full one
    above); every count equals the oracle's."""
    lo, hi, max_len = 64, 128, 16392
    offsets, lengths = (0, 3, 16, 63), list(range(4080, max_len + 1, 8))
    region = synth.random_bytes(max_len + 64, seed=70 + w)
    host = np.concatenate([np.full(lo, 0xFF, np.uint8), region, np.full(hi, 0xFF, np.uint8)])
    buf = torch.from_numpy(host).to(dev())
    starts = [lo + o for o in offsets for _ in lengths]
    lens = [n for _ in offsets for n in lengths]
    rows = len(lens)
    want = oracle.pospopcnt_ranges(host, starts, lens, [w] * rows)
    counts = torch.zeros((rows, w), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr(), counts.data_ptr()
    descs = ppc.make_descs([base + s for s in starts], lens, [cbase + r * w * 8 for r in range(rows)], [w] * rows)
    plan = ppc.ppc_plan_create(descs, rows, ppc.ppc_plan_opts(16, 0, 0, 1, 0))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
    finally:
        ppc.ppc_plan_destroy(plan)
    got = ppc.counts_to_numpy(counts).reshape(rows, w)
    for r in range(rows):
        assert np.array_equal(got[r], want[r]), "plan: start %d, length %d" % (starts[r], lens[r])
    one = torch.zeros(w, dtype=torch.int64, device=dev())
    for r in range(0, rows, 17):
        one.zero_()
        ppc.ppc_pospopcnt(w, one, buf[starts[r]:starts[r] + lens[r]])
        assert np.array_equal(ppc.counts_to_numpy(one), want[r]), "plain: start %d, length %d" % (starts[r], lens[r])


def test_plan_graph_replays_with_eager_work_between(ppc):
    """A plan's graph (cursor reset, the persistent kernel, the small-array
    kernel) replayed five times, with eager work and a plain call between
    the replays and a synchronisation after each: every replay adds exactly
    one run's counts (tolerance 0) for the arrays of a tile or more and for
    those shorter than one tile."""
    spec = synth.batch_spec(2000, seed=33, lo=16, hi=4 * MiB, start_jitter=64)
    n = len(spec["lengths"])
    pool = make_pool(spec, seed=33)
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    want = oracle_rows(pool.cpu().numpy(), spec, range(n))
    small = sum(1 for L in spec["lengths"] if int(L) < 14 * 1024)
    assert 200 < small < n - 200  # both kernels have arrays
    plan = plan_for(ppc, pool, spec, counts, opts(ppc, tiles=16, waves=1024))
    eager = torch.zeros(16, dtype=torch.int64, device=dev())
    try:
        assert ppc.ppc_plan_get_info(plan)["graph"] == 1
        for r in range(1, 6):
            ppc.ppc_plan_run(plan)
            x = torch.randn(512, 512, device=dev())
            y = (x @ x).abs().sum()
            ppc.ppc_pospopcnt16(eager, pool[:1 << 20])
            torch.cuda.synchronize()
            assert torch.isfinite(y)
            check_rows(ppc.counts_to_numpy(counts), spec, want, reps=r)
    finally:
        ppc.ppc_plan_destroy(plan)


@pytest.mark.parametrize("w", (8, 16, 32, 64))
def test_walk_short_paths_on_last_items(ppc, w):
    """The batched walk's short paths in a plan: arrays of one whole tile
    plus 0..4,096 bytes (every 8th length) and plus 4,096..16,392 bytes
    (every 56th), at start offsets 0, 3, 16 and 63, split into items of one
    tile.  From 32 extra bytes on, at every offset, an array holds more than
    one tile, so the plan's walk takes it, and its last item holds no whole
    tile and a partial tile of at most one chunk per lane (the half-adder
    path), of 2..14 (the carry-save path without the top counter) or of 15
    and 16 (the full walk); every count equals the oracle's."""
    lo, hi, tile = 64, 128, 16384
    extra = list(range(0, 4097, 8)) + list(range(4096 + 56, 16393, 56))
    offsets = (0, 3, 16, 63)
    region = synth.random_bytes(tile + max(extra) + 64, seed=80 + w)
    host = np.concatenate([np.full(lo, 0xFF, np.uint8), region, np.full(hi, 0xFF, np.uint8)])
    buf = torch.from_numpy(host).to(dev())
    starts = [lo + o for o in offsets for _ in extra]
    lens = [tile + e for _ in offsets for e in extra]
    rows = len(lens)
    want = oracle.pospopcnt_ranges(host, starts, lens, [w] * rows)
    counts = torch.zeros((rows, w), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr(), counts.data_ptr()
    descs = ppc.make_descs([base + s for s in starts], lens, [cbase + r * w * 8 for r in range(rows)], [w] * rows)
    plan = ppc.ppc_plan_create(descs, rows, ppc.ppc_plan_opts(1, 0, 0, 1, 0))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
        info = ppc.ppc_plan_get_info(plan)
    finally:
        ppc.ppc_plan_destroy(plan)
    assert info["tiles_per_item"] == 1
    got = ppc.counts_to_numpy(counts).reshape(rows, w)
    for r in range(rows):
        assert np.array_equal(got[r], want[r]), "start %d, length %d" % (starts[r], lens[r])


@pytest.mark.parametrize("k_max", (1, 2, 3, 4, 6, 8, 11, 14, 15, 16))
def test_small_array_kernel_chunk_classes(ppc, k_max):
    """Plans give arrays shorter than one tile, of at most 14 chunks per lane,
    to a kernel of their own, built for 1, 2, 4, 8 or 14 chunks per lane by
    the batch's longest such array.  A batch whose longest array holds
    k_max * 1024 bytes (k_max chunks per lane from an aligned start; at 15
    and 16 it is no longer small), lengths from 0 up to that at every start
    residue mod 16, arrays of more than a tile beside them and arrays that
    share counter rows: after a graph replay, a second replay and a run
    without the graph every row holds three times the oracle's counts."""
    rng = np.random.default_rng(900 + k_max)
    top, lo = k_max * 1024, 64
    region = synth.random_bytes(top + 80 * 1024, seed=900 + k_max)
    host = np.concatenate([np.full(lo, 0xFF, np.uint8), region, np.full(128, 0xFF, np.uint8)])
    buf = torch.from_numpy(host).to(dev())
    assert buf.data_ptr() % 16 == 0
    fixed = [0, 1, 15, 16, 17, 31, 1023, 1024, 1025, top - 1, top, top + 15]
    lens = fixed + [int(x) for x in rng.integers(0, top + 16, size=240)] + [16400, 20000, 65539]
    offs = [0] * len(fixed) + [int(x) for x in rng.integers(0, 16, size=240)] + [0, 5, 9]
    offs[len(fixed) - 1] = 7  # top + 15 bytes from an unaligned start as well
    n = len(lens)
    starts = [lo + o for o in offs]
    widths = [int(x) for x in rng.choice(np.array([8, 16, 32, 64]), size=n)]
    rows = list(range(n))
    for a, b in ((3, n - 1), (7, 40), (41, 42)):  # shared counter rows
        rows[b] = rows[a]
    want = np.zeros((n, 64), dtype=np.uint64)
    for i, r in enumerate(oracle.pospopcnt_ranges(host, starts, lens, widths)):
        want[rows[i], :widths[i]] += r
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr(), counts.data_ptr()
    descs = ppc.make_descs([base + s for s in starts], lens, [cbase + r * 64 * 8 for r in rows], widths)
    for graph in (1, 0):
        plan = ppc.ppc_plan_create(descs, n, ppc.ppc_plan_opts(16, 0, 0, graph, 0))
        try:
            for _ in range(2 if graph else 1):
                ppc.ppc_plan_run(plan)
            torch.cuda.synchronize()
            info = ppc.ppc_plan_get_info(plan)
        finally:
            ppc.ppc_plan_destroy(plan)
        assert info["graph"] == graph
    got = ppc.counts_to_numpy(counts).reshape(n, 64)
    for i in range(n):
        assert np.array_equal(got[i], want[i] * np.uint64(3)), "row %d: start %d, length %d, w=%d" % (
            i, starts[i], lens[i], widths[i])


@pytest.mark.parametrize("tiles_per_item", (0, 1 << 18))
def test_arrays_beyond_4GiB_in_one_plan(ppc, tiles_per_item, tmp_path, monkeypatch):
    """Maximum sizes in the batched form: a 5 GiB + 13-byte array (over 2^18
    tiles of 16 KiB) from an unaligned start and a 1 GiB array, next to small
    ragged arrays, in one plan.  With 2^18 tiles per item the big array
    becomes one item of 4 GiB and one of the rest; with the tuned setting it
    becomes thousands.  Every array must match the oracle exactly."""
    monkeypatch.setenv("PPC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    big, mid = (5 << 30) + 13, 1 << 30
    small = [1, 15, 17, 4095, 16 * 1024 + 3, MiB + 77]
    lengths = [big, mid] + small
    widths = [32, 64, 8, 16, 32, 64, 8, 16]
    starts, pos = [], 3  # the first array starts 3 bytes past a 16-byte boundary
    for n in lengths:
        starts.append(pos)
        pos += n + 29
    buf = synth.device_bernoulli(pos + 64, 0.5, seed=23, device=dev())
    counts = torch.zeros((len(lengths), 64), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr(), counts.data_ptr()
    descs = ppc.make_descs([base + s for s in starts], lengths, [cbase + i * 512 for i in range(len(lengths))],
                           widths)
    opts = ppc.ppc_plan_opts(tiles_per_item, 0, 1 if tiles_per_item == 0 else 0, 1, 0)
    plan = ppc.ppc_plan_create(descs, len(lengths), opts)
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
        got = ppc.counts_to_numpy(counts)
    finally:
        ppc.ppc_plan_destroy(plan)
    host = buf.cpu().numpy()
    del buf
    torch.cuda.empty_cache()
    for i, (s, n, w) in enumerate(zip(starts, lengths, widths)):
        want = oracle.pospopcnt_mt(host[s:s + n], w, 16)
        assert np.array_equal(got[i, :w], want), (i, n, w)
        assert not got[i, w:].any()


@pytest.mark.parametrize("w", (8, 16, 32, 64))
def test_pieces_of_one_array_share_counters(ppc, w):
    """Streamed pieces inside one plan: an array cut at random multiples of
    8 bytes from its (unaligned) start into 300 pieces of uneven length,
    every piece a descriptor adding into the same counters.  Positions are
    relative to each piece's pointer, so at cuts that are multiples of w/8
    the pieces' counts add up to the whole array's (Section 4, step 1 and
    its footnote); the atomics make the sum exact in any order."""
    n = 37 * MiB + 5
    host = synth.random_bytes(n + 3, seed=60 + w)
    buf = torch.from_numpy(host).to(dev())
    rng = np.random.default_rng(w)
    cuts = np.unique(rng.integers(0, n // 8, size=299) * 8)
    bounds = [0] + [int(c) for c in cuts if 0 < c < n] + [n]
    counts = torch.zeros(w, dtype=torch.int64, device=dev())
    base = buf.data_ptr() + 3
    k = len(bounds) - 1
    descs = ppc.make_descs([base + bounds[i] for i in range(k)], [bounds[i + 1] - bounds[i] for i in range(k)],
                           [counts.data_ptr()] * k, [w] * k)
    plan = ppc.ppc_plan_create(descs, k, ppc.ppc_plan_opts(16, 0, 0, 1, 0))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
    finally:
        ppc.ppc_plan_destroy(plan)
    assert np.array_equal(ppc.counts_to_numpy(counts), oracle.pospopcnt(host[3:], w))
