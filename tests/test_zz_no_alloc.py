"""GPU parity of the allocation-free batched call (ppc_batch_noalloc).

Its output must equal, bit for bit, what a plan (ppc_plan_create +
ppc_plan_run, the batched entry point that allocates) adds for the same
descriptors, and the oracle's counts.  Two calls in a row share the
library's static scratch array; the second is smaller, so a table entry or
cursor left over from the first would show up in its counts.
"""
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
    pool = torch.full((spec["pool_bytes"] + 128,), 0xFF, dtype=torch.uint8, device=dev())
    for i, (off, n, p) in enumerate(zip(spec["offsets"], spec["lengths"], spec["p"])):
        if n:
            synth.device_bernoulli(int(n), float(p), seed=seed * 1_000_003 + i, device=dev(),
                                   out=pool[int(off):int(off) + int(n)])
    torch.cuda.synchronize()
    return pool


def descs_for(ppc, pool, spec, counts):
    n = len(spec["lengths"])
    base, cbase = pool.data_ptr(), counts.data_ptr()
    return ppc.make_descs([base + int(o) for o in spec["offsets"]], spec["lengths"],
                          [cbase + i * 512 for i in range(n)], spec["widths"])


def to_device(ppc, descs):
    raw = ppc.descs_bytes(descs)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev())


def noalloc_counts(ppc, pool, spec):
    n = len(spec["lengths"])
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    descs_dev = to_device(ppc, descs_for(ppc, pool, spec, counts))
    bad = torch.full((1,), 12345, dtype=torch.int32, device=dev())
    print("noalloc call: %d arrays, %d bytes" % (n, int(spec["lengths"].sum())), flush=True)
    ppc.ppc_batch_noalloc(descs_dev, n, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    return ppc.counts_to_numpy(counts).reshape(n, 64)


def plan_counts(ppc, pool, spec):
    n = len(spec["lengths"])
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    plan = ppc.ppc_plan_create(descs_for(ppc, pool, spec, counts), n,
                               ppc.ppc_plan_opts(16, 0, 0, 0, 0))
    try:
        ppc.ppc_plan_run(plan)
        torch.cuda.synchronize()
    finally:
        ppc.ppc_plan_destroy(plan)
    return ppc.counts_to_numpy(counts).reshape(n, 64)


def check_against_oracle(got, pool, spec):
    want = oracle.pospopcnt_ranges(pool.cpu().numpy(), spec["offsets"], spec["lengths"], spec["widths"])
    for i, row in enumerate(want):
        w = int(spec["widths"][i])
        assert np.array_equal(got[i, :w], row), "array %d (w=%d, n=%d)" % (i, w, int(spec["lengths"][i]))
        assert not got[i, w:].any()


def test_two_calls_in_a_row_match_the_plan_and_the_oracle(ppc):
    # first call: 2,500 arrays up to 8 MiB (whole items and shorter ones),
    # unaligned starts; second call: 400 arrays up to 64 KiB
    spec1 = synth.batch_spec(2500, seed=40, lo=16, hi=8 * MiB, start_jitter=64)
    spec2 = synth.batch_spec(400, seed=41, lo=16, hi=64 * 1024, start_jitter=64)
    pool1, pool2 = make_pool(spec1, seed=40), make_pool(spec2, seed=41)
    got1 = noalloc_counts(ppc, pool1, spec1)
    got2 = noalloc_counts(ppc, pool2, spec2)
    assert np.array_equal(got1, plan_counts(ppc, pool1, spec1))
    assert np.array_equal(got2, plan_counts(ppc, pool2, spec2))
    check_against_oracle(got1, pool1, spec1)
    check_against_oracle(got2, pool2, spec2)


def test_edge_only_empty_and_single_arrays(ppc):
    # every length 0..40 at start offsets 0..15, all widths, then one array
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
    pool = make_pool(spec, seed=42)
    got = noalloc_counts(ppc, pool, spec)
    assert np.array_equal(got, plan_counts(ppc, pool, spec))
    check_against_oracle(got, pool, spec)
    one = dict(offsets=np.array([3]), lengths=np.array([5 * MiB + 7]), widths=np.array([32]),
               p=np.array([0.3]), pool_bytes=5 * MiB + 64)
    pool1 = make_pool(one, seed=43)
    got1 = noalloc_counts(ppc, pool1, one)
    check_against_oracle(got1, pool1, one)


def test_invalid_descriptor_counts_nothing_and_next_call_is_clean(ppc):
    spec = synth.batch_spec(50, seed=44, lo=16, hi=256 * 1024)
    pool = make_pool(spec, seed=44)
    counts = torch.zeros((50, 64), dtype=torch.int64, device=dev())
    descs = descs_for(ppc, pool, spec, counts)
    descs[7].width = 12
    descs[9].counts = counts.data_ptr() + 4
    bad = torch.zeros(1, dtype=torch.int32, device=dev())
    ppc.ppc_batch_noalloc(to_device(ppc, descs), 50, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 2
    assert not counts.any()
    # an empty batch reports no invalid descriptor
    ppc.ppc_batch_noalloc(None, 0, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    # the same arrays, valid now, after the rejected call
    got = noalloc_counts(ppc, pool, spec)
    check_against_oracle(got, pool, spec)
    with pytest.raises(ppc.PpcError):
        ppc.ppc_batch_noalloc(to_device(ppc, descs), 65537, None)


def test_maximum_array_count(ppc):
    """PPC_NOALLOC_MAX_ARRAYS arrays in one call (short, unaligned, every
    width, a few of several MiB among them): every array equals the oracle."""
    n = 65536
    rng = np.random.default_rng(45)
    lengths = rng.integers(0, 300, size=n)
    lengths[rng.choice(n, size=8, replace=False)] = rng.integers(1 << 20, 6 << 20, size=8)
    widths = rng.choice(np.array([8, 16, 32, 64]), size=n)
    offsets = np.empty(n, dtype=np.int64)
    pos = 0
    for i in range(n):
        offsets[i] = pos + int(rng.integers(0, 16))
        pos = int(offsets[i] + lengths[i])
    spec = dict(offsets=offsets, lengths=lengths, widths=widths, p=np.full(n, 0.5), pool_bytes=pos + 64)
    pool = synth.device_bernoulli(pos + 64, 0.5, seed=45, device=dev())
    got = noalloc_counts(ppc, pool, spec)
    check_against_oracle(got, pool, spec)


def test_one_block_and_grid_setup_boundary(ppc):
    """255 and 256 arrays take the one-block setup, 257 the three grid-wide
    setup kernels; three calls in a row, each against the plan and the
    oracle (short and long arrays, unaligned starts)."""
    for k, n in enumerate((255, 256, 257)):
        spec = synth.batch_spec(n, seed=50 + k, lo=16, hi=2 * MiB, start_jitter=64)
        pool = make_pool(spec, seed=50 + k)
        got = noalloc_counts(ppc, pool, spec)
        assert np.array_equal(got, plan_counts(ppc, pool, spec))
        check_against_oracle(got, pool, spec)


def test_arrays_beyond_4GiB(ppc):
    """Maximum sizes: a 5 GiB + 13-byte array (over 2^18 tiles of 16 KiB)
    from an unaligned start and a 1 GiB array, next to small ragged arrays,
    in one call; then the same descriptors again, so every count doubles.
    Every array must match the oracle exactly."""
    big, mid = (5 << 30) + 13, 1 << 30
    small = [1, 15, 17, 4095, 16 * 1024 + 3, MiB + 77]
    lengths = [big, mid] + small
    widths = [32, 64, 8, 16, 32, 64, 8, 16]
    starts, pos = [], 3  # the first array starts 3 bytes past a 16-byte boundary
    for n in lengths:
        starts.append(pos)
        pos += n + 29
    buf = synth.device_bernoulli(pos + 64, 0.5, seed=24, device=dev())
    n = len(lengths)
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev())
    base, cbase = buf.data_ptr(), counts.data_ptr()
    descs_dev = to_device(ppc, ppc.make_descs([base + s for s in starts], lengths,
                                              [cbase + i * 512 for i in range(n)], widths))
    bad = torch.full((1,), 12345, dtype=torch.int32, device=dev())
    print("noalloc call: %d arrays, %d bytes" % (n, sum(lengths)), flush=True)
    ppc.ppc_batch_noalloc(descs_dev, n, bad)
    ppc.ppc_batch_noalloc(descs_dev, n, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    got = ppc.counts_to_numpy(counts)
    host = buf.cpu().numpy()
    del buf
    torch.cuda.empty_cache()
    for i, (s, ln, w) in enumerate(zip(starts, lengths, widths)):
        want = oracle.pospopcnt_mt(host[s:s + ln], w, 16)
        assert np.array_equal(got[i, :w], want * np.uint64(2)), (i, ln, w)
        assert not got[i, w:].any()


def random_batch(rng, kind, n_tiles=(0, 0)):
    """A seeded batch of one of three shapes: 'mix' (1-700 arrays, lengths
    log-uniform up to 2 MiB, some empty), 'tiles' (n arrays of k whole tiles
    less 0-63 bytes, so that the items share a bucket and tickets group
    several of them), 'edge' (thousands of arrays of 0-40 bytes: head/tail
    items only)."""
    if kind == "mix":
        n = int(rng.integers(1, 700))
        lengths = np.exp(rng.uniform(0.0, np.log(2 * MiB), size=n)).astype(np.int64)
        lengths[rng.random(n) < 0.05] = 0
    elif kind == "tiles":
        n, k = n_tiles
        lengths = k * 16384 - rng.integers(0, 64, size=n)
    else:
        n = int(rng.integers(2000, 6000))
        lengths = rng.integers(0, 41, size=n)
    widths = rng.choice(np.array([8, 16, 32, 64]), size=n)
    jitter = rng.integers(0, 64, size=n)
    offsets = np.empty(n, dtype=np.int64)
    pos = 0
    for i in range(n):
        pos = (pos + 255) // 256 * 256
        offsets[i] = pos + jitter[i]
        pos = int(offsets[i] + lengths[i])
    return dict(offsets=offsets, lengths=lengths.astype(np.int64), widths=widths.astype(np.int64),
                p=rng.uniform(0.0, 1.0, size=n), pool_bytes=pos + 256)


def test_random_batches_match_the_plan_and_the_oracle(ppc):
    """Twelve seeded batches of the three shapes, one call after another on
    the shared scratch: every array equals the plan's and the oracle's.  The
    'tiles' batches (n arrays of k tiles) take the cursor-free walk (300 x 1),
    and groups of two or one halved from twice that (3,000 x 4, 5,000 x 1,
    10,000 x 2)."""
    rng = np.random.default_rng(60)
    tiles = iter([(300, 1), (3000, 4), (10000, 2), (5000, 1)])
    for b, kind in enumerate(["mix"] * 6 + ["tiles"] * 4 + ["edge"] * 2):
        spec = random_batch(rng, kind, next(tiles) if kind == "tiles" else (0, 0))
        print("random batch %d (%s): %d arrays" % (b, kind, len(spec["lengths"])), flush=True)
        pool = make_pool(spec, seed=60 + b)
        got = noalloc_counts(ppc, pool, spec)
        assert np.array_equal(got, plan_counts(ppc, pool, spec)), "batch %d (%s)" % (b, kind)
        check_against_oracle(got, pool, spec)


def test_captured_in_a_graph_and_replayed(ppc):
    """The call records into a HIP graph (torch.cuda.CUDAGraph capturing on
    its own stream): two calls in one graph, on a batch of long arrays and
    on a short batch (whose arrays below one tile go to the small-array
    kernel); every replay adds exactly one count of each, with an eager
    allocation-free call on a third batch and other eager work between the
    replays (the calls share the scratch array, in stream order).  Every
    replay is checked (tolerance 0)."""
    spec = synth.batch_spec(300, seed=46, lo=16, hi=2 * MiB, start_jitter=64)
    spec2 = synth.batch_spec(50, seed=47, lo=16, hi=64 * 1024, start_jitter=64)
    spec3 = synth.batch_spec(400, seed=48, lo=16, hi=16 * 1024, start_jitter=64)
    pool, pool2, pool3 = make_pool(spec, seed=46), make_pool(spec2, seed=47), make_pool(spec3, seed=48)
    counts = torch.zeros((300, 64), dtype=torch.int64, device=dev())
    counts2 = torch.zeros((50, 64), dtype=torch.int64, device=dev())
    counts3 = torch.zeros((400, 64), dtype=torch.int64, device=dev())
    d1 = to_device(ppc, descs_for(ppc, pool, spec, counts))
    d2 = to_device(ppc, descs_for(ppc, pool2, spec2, counts2))
    d3 = to_device(ppc, descs_for(ppc, pool3, spec3, counts3))
    want = oracle.pospopcnt_ranges(pool.cpu().numpy(), spec["offsets"], spec["lengths"], spec["widths"])
    want2 = oracle.pospopcnt_ranges(pool2.cpu().numpy(), spec2["offsets"], spec2["lengths"], spec2["widths"])
    want3 = oracle.pospopcnt_ranges(pool3.cpu().numpy(), spec3["offsets"], spec3["lengths"], spec3["widths"])

    side = torch.cuda.Stream()  # warm-up off the capture (first launches, scratch address)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ppc.ppc_batch_noalloc(d1, 300)
        ppc.ppc_batch_noalloc(d3, 400)
    torch.cuda.synchronize()
    counts.zero_()
    counts3.zero_()
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ppc.ppc_batch_noalloc(d1, 300)
        ppc.ppc_batch_noalloc(d3, 400)
    torch.cuda.synchronize()
    assert not counts.any() and not counts3.any()  # capturing runs nothing

    for r in range(1, 5):
        g.replay()
        ppc.ppc_batch_noalloc(d2, 50)
        x = torch.randn(512, 512, device=dev())
        y = (x @ x).abs().sum()
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        got = ppc.counts_to_numpy(counts).reshape(300, 64)
        got2 = ppc.counts_to_numpy(counts2).reshape(50, 64)
        got3 = ppc.counts_to_numpy(counts3).reshape(400, 64)
        for i, row in enumerate(want):
            w = int(spec["widths"][i])
            assert np.array_equal(got[i, :w], row * np.uint64(r)), "replay %d, array %d" % (r, i)
        for i, row in enumerate(want3):
            w = int(spec3["widths"][i])
            assert np.array_equal(got3[i, :w], row * np.uint64(r)), "replay %d, short batch array %d" % (r, i)
        for i, row in enumerate(want2):
            w = int(spec2["widths"][i])
            assert np.array_equal(got2[i, :w], row * np.uint64(r)), "eager call %d, array %d" % (r, i)
