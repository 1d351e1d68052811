"""GPU parity of the serving form (ppc_server_*).

Each served request must equal, bit for bit, the oracle on its bytes, the
plain call run alone on the same bytes, and the same request served alone
(tolerance 0) -- whatever batch it shared on the device.
"""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MiB = 1 << 20
N_COL, COL_BYTES = 8, 4 * MiB


@pytest.fixture(scope="module")
def ppc():
    import paper_2412_16370_amd as ppc

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ppc.lib()
    return ppc


@pytest.fixture(scope="module")
def pool():
    host = synth.bernoulli(N_COL * COL_BYTES, 0.3, seed=40)
    return host, torch.from_numpy(host).to("cuda:0")


def trace(n, seed, rate, lo=1, hi=COL_BYTES):
    return synth.serve_trace(n, seed=seed, n_columns=N_COL, column_bytes=COL_BYTES, rate_per_s=rate,
                             lo=lo, hi=hi)


def want_for(host, t, i):
    c, w, o, n = (int(t[k][i]) for k in ("column", "width", "offset", "length"))
    base = c * COL_BYTES + o
    return oracle.pospopcnt(host[base:base + n], w)


def alone_plain(ppc, dev_pool, t, col_bytes=COL_BYTES):
    n = len(t["length"])
    counts = torch.zeros((n, 64), dtype=torch.int64, device="cuda:0")
    lib = ppc.lib()
    st = torch.cuda.current_stream().cuda_stream
    for i in range(n):
        addr = dev_pool.data_ptr() + int(t["column"][i]) * col_bytes + int(t["offset"][i])
        assert lib.ppc_pospopcnt(int(t["width"][i]), counts.data_ptr() + i * 512, addr,
                                 int(t["length"][i]), st) == 0
    torch.cuda.synchronize()
    return ppc.counts_to_numpy(counts).reshape(n, 64)


WAIT_S = 60.0  # no served request in these tests takes more than milliseconds


def poll_until(ppc, server, n, cap=1024):
    """Polls until n results have come back, failing the test (instead of
    hanging the run) if they have not within WAIT_S seconds."""
    out = []
    deadline = time.monotonic() + WAIT_S
    while len(out) < n:
        out += ppc.ppc_server_poll(server, cap)
        assert time.monotonic() < deadline, "only %d of %d results after %.0f s" % (len(out), n, WAIT_S)
    return out


def served_alone(ppc, server, t, i):
    assert ppc.ppc_server_submit(server, t["column"][i], t["width"][i], t["offset"][i], t["length"][i],
                                 tag=10**9 + i) == ppc.PPC_OK
    res = poll_until(ppc, server, 1)
    assert len(res) == 1 and res[0].tag == 10**9 + i and res[0].status == 0
    return np.array(res[0].counts[:res[0].width], dtype=np.uint64)


def check_all_against_oracle(host_pool, t, results, col_bytes):
    """Every served result equals the oracle on its bytes (threads over the
    host cores, one Fig. 2 loop per request)."""
    n = len(t["length"])
    starts = [int(t["column"][i]) * col_bytes + int(t["offset"][i]) for i in range(n)]
    want = oracle.pospopcnt_ranges(host_pool, starts, t["length"], t["width"])
    for i in range(n):
        r = results[i]
        w = int(t["width"][i])
        assert r.tag == i and r.status == 0 and r.width == w, "request %d" % i
        assert np.array_equal(np.array(r.counts[:w], dtype=np.uint64), want[i]), "request %d" % i
        assert not any(r.counts[w:]), "request %d" % i


def test_trace_matches_oracle_plain_and_alone(ppc, pool):
    host, dev_pool = pool
    t = trace(3000, seed=41, rate=2e6)
    cfg = ppc.ppc_server_cfg(4, 256, 0, 0, 0, 0, 0)
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES, cfg=cfg)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"],
                                                  t["length"], t["arrival_ns"])
        assert stats["n_requests"] == 3000 and stats["batches"] >= 1
        assert stats["mean_batch"] > 1.0  # requests really shared batches
        assert stats["p50_ns"] <= stats["p99_ns"] <= stats["max_ns"]
        plain = alone_plain(ppc, dev_pool, t)
        for i in range(3000):
            r = results[i]
            w = int(t["width"][i])
            assert r.tag == i and r.status == 0 and r.width == w
            got = np.array(r.counts[:w], dtype=np.uint64)
            assert np.array_equal(got, want_for(host, t, i)), "request %d" % i
            assert np.array_equal(got, plain[i, :w])
        for i in np.random.default_rng(5).choice(3000, size=40, replace=False):
            got = np.array(results[int(i)].counts[:int(t["width"][i])], dtype=np.uint64)
            assert np.array_equal(served_alone(ppc, server, t, int(i)), got)
    finally:
        ppc.ppc_server_destroy(server)


def test_admission_by_memory_queues_but_stays_exact(ppc, pool):
    host, dev_pool = pool
    t = trace(600, seed=42, rate=5e6)
    cfg = ppc.ppc_server_cfg(2, 64, 4, 0, 1 * MiB, 0, 0)  # 4 slots, 1 MiB in flight
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES, cfg=cfg)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"],
                                                  t["length"], t["arrival_ns"])
        assert stats["busy_rejections"] > 0
        assert ppc.ppc_server_get_stats(server)["max_batch_seen"] <= 4
        for i in range(600):
            w = int(t["width"][i])
            assert np.array_equal(np.array(results[i].counts[:w], dtype=np.uint64), want_for(host, t, i))
    finally:
        ppc.ppc_server_destroy(server)


def test_submit_poll_api(ppc, pool):
    host, dev_pool = pool
    t = trace(200, seed=43, rate=1e6)
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES,
                                   cfg=ppc.ppc_server_cfg(3, 16, 32, 4, 0, 0, 0))
    got = {}
    try:
        i = 0
        deadline = time.monotonic() + WAIT_S
        while i < 200 or len(got) < 200:
            assert time.monotonic() < deadline, "stuck at %d submitted, %d done" % (i, len(got))
            if i < 200:
                rc = ppc.ppc_server_submit(server, t["column"][i], t["width"][i], t["offset"][i],
                                           t["length"][i], tag=i)
                if rc == ppc.PPC_OK:
                    i += 1
            for r in ppc.ppc_server_poll(server, 64):
                assert r.status == 0 and r.t_done_ns >= r.t_submit_ns
                got[int(r.tag)] = np.array(r.counts[:r.width], dtype=np.uint64)
        for k in range(200):
            assert np.array_equal(got[k], want_for(host, t, k))
        assert ppc.ppc_server_get_stats(server)["inflight"] == 0
    finally:
        ppc.ppc_server_destroy(server)


def test_invalid_requests_rejected(ppc, pool):
    _, dev_pool = pool
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES)
    try:
        for bad in ((N_COL, 16, 0, 10), (0, 12, 0, 10), (0, 16, COL_BYTES - 5, 6),
                    (0, 16, COL_BYTES + 1, 0)):
            with pytest.raises(ppc.PpcError) as e:
                ppc.ppc_server_submit(server, *bad)
            assert e.value.status == ppc.PPC_EINVAL
        assert ppc.ppc_server_submit(server, 0, 16, COL_BYTES - 5, 5) == ppc.PPC_OK
        assert len(poll_until(ppc, server, 1)) == 1
    finally:
        ppc.ppc_server_destroy(server)


def test_onehot_u32_columns_count_the_histogram(ppc):
    words = 1 << 20  # 4 MiB per column
    pool_host, cats = synth.onehot_u32_columns(4, words, seed=4)
    dev_pool = torch.from_numpy(pool_host).to("cuda:0")
    server = ppc.ppc_server_create(dev_pool, column_bytes=4 * words)
    try:
        rng = np.random.default_rng(6)
        reqs = []
        for k in range(64):
            c = int(rng.integers(4))
            a, b = sorted(int(x) for x in rng.integers(0, words + 1, size=2))
            reqs.append((c, a, b))
        t = dict(column=[r[0] for r in reqs], width=[32] * 64, offset=[4 * r[1] for r in reqs],
                 length=[4 * (r[2] - r[1]) for r in reqs], arrival_ns=[0] * 64)
        results, _ = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                              t["arrival_ns"])
        for k, (c, a, b) in enumerate(reqs):
            hist = np.bincount(cats[c * words + a:c * words + b], minlength=32)
            assert np.array_equal(np.array(results[k].counts[:32], dtype=np.uint64), hist)
    finally:
        ppc.ppc_server_destroy(server)


@pytest.fixture(scope="module")
def full_pool(ppc):
    """The serving pool at full size: 1 GiB of one-hot uint32 columns (16 x
    64 MiB, 32 categories, Zipf s = 1.0), on the device and copied to host."""
    pool = synth.device_onehot_u32_columns(16, FULL_COL // 4, seed=4, device="cuda:0")
    torch.cuda.synchronize()
    return pool, pool.cpu().numpy()


FULL_COL = 64 * MiB


def full_trace(n, rho, seed):
    """Poisson requests (64 B .. 64 MiB, unaligned) over the full pool,
    offered at rho times 6.5 TB/s, about the plain kernel's bandwidth."""
    rate = rho * 6.5e12 / synth.log_uniform_mean(64, 64 * MiB)
    return synth.serve_trace(n, seed=seed, n_columns=16, column_bytes=FULL_COL, rate_per_s=rate, lo=64,
                             hi=64 * MiB)


def test_full_size_pool_at_half_load(ppc, full_pool):
    """The serving workload at full size, in the default server
    configuration the bench times, at half load: 20,000 Poisson requests.
    Every result equals the oracle on its bytes and the plain call on the
    same bytes, and sampled requests served alone equal their result in
    the mix (tolerance 0)."""
    pool, host = full_pool
    n = 20_000
    t = full_trace(n, 0.5, seed=4)
    server = ppc.ppc_server_create(pool, column_bytes=FULL_COL)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                                  t["arrival_ns"])
        assert stats["n_requests"] == n and stats["mean_batch"] > 1.0
        check_all_against_oracle(host, t, results, FULL_COL)
        plain = alone_plain(ppc, pool, t, col_bytes=FULL_COL)
        for i in range(n):
            w = int(t["width"][i])
            assert np.array_equal(np.array(results[i].counts[:w], dtype=np.uint64), plain[i, :w]), i
        rng = np.random.default_rng(7)
        t_one = {k: t[k] for k in ("column", "width", "offset", "length")}
        for i in rng.choice(n, size=20, replace=False):
            i = int(i)
            w = int(t["width"][i])
            got = np.array(results[i].counts[:w], dtype=np.uint64)
            assert np.array_equal(served_alone(ppc, server, t_one, i), got)
    finally:
        ppc.ppc_server_destroy(server)


def test_full_size_pool_near_saturation(ppc, full_pool):
    """The bench's second served configuration: the default server at 0.9
    of the plain kernel's bandwidth, where batches run to hundreds of
    requests and three streams overlap on the device.  Every one of 20,000
    results equals the oracle on its bytes."""
    pool, host = full_pool
    n = 20_000
    t = full_trace(n, 0.9, seed=5)
    server = ppc.ppc_server_create(pool, column_bytes=FULL_COL)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                                  t["arrival_ns"])
        big = ppc.ppc_server_get_stats(server)["max_batch_seen"]
    finally:
        ppc.ppc_server_destroy(server)
    print("rho 0.9: mean batch %.1f, largest %d, p50 %.0f us, p99 %.0f us"
          % (stats["mean_batch"], big, stats["p50_ns"] / 1e3, stats["p99_ns"] / 1e3))
    assert stats["n_requests"] == n and big >= 64
    check_all_against_oracle(host, t, results, FULL_COL)


def test_edge_requests_in_one_batch(ppc, pool):
    """Empty requests, single bytes at both ends of a column, whole columns,
    requests ending on a column's last byte and ragged ones, every width,
    all arriving at once (one or two batches): each equals the oracle."""
    host, dev_pool = pool
    reqs = []
    for w in (8, 16, 32, 64):
        for c in (0, N_COL - 1):
            reqs += [(c, w, 0, 0), (c, w, COL_BYTES, 0), (c, w, 0, 1), (c, w, COL_BYTES - 1, 1),
                     (c, w, 0, COL_BYTES), (c, w, 7, COL_BYTES - 7), (c, w, 5, 16 * 1024 + 3),
                     (c, w, COL_BYTES - 1000, 1000), (c, w, 13, 31)]
    t = dict(column=[r[0] for r in reqs], width=[r[1] for r in reqs], offset=[r[2] for r in reqs],
             length=[r[3] for r in reqs], arrival_ns=[0] * len(reqs))
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                                  t["arrival_ns"])
        for i, (c, w, o, n) in enumerate(reqs):
            r = results[i]
            assert r.tag == i and r.status == 0 and r.width == w
            want = oracle.pospopcnt(host[c * COL_BYTES + o:c * COL_BYTES + o + n], w)
            assert np.array_equal(np.array(r.counts[:w], dtype=np.uint64), want), (c, w, o, n)
            assert not any(r.counts[w:])
    finally:
        ppc.ppc_server_destroy(server)


def test_burst_fills_every_batch_to_max_batch(ppc, pool):
    """640 requests arriving at once on a server of two streams with
    max_batch = 64: every batch goes out full, exactly 64 requests, ten
    batches in all, and every result equals the oracle."""
    host, dev_pool = pool
    t = trace(640, seed=44, rate=1e6)
    t["arrival_ns"] = np.zeros(640, dtype=np.int64)
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES, cfg=ppc.ppc_server_cfg(2, 64, 0, 0, 0, 0, 0))
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                                  t["arrival_ns"])
        assert ppc.ppc_server_get_stats(server)["max_batch_seen"] == 64
    finally:
        ppc.ppc_server_destroy(server)
    assert stats["batches"] == 10 and stats["mean_batch"] == 64.0
    check_all_against_oracle(host, t, results, COL_BYTES)


def test_item_table_cap_and_tile_doubling(ppc):
    """A server whose item table (4096 items) cannot take a batch's worth of
    large requests at one tile per item.  A request of 2048 tiles would need
    2048 items, more than a quarter of the table, so its tiles per item
    double to 2 (1024 items), and the fifth such request of a batch no
    longer fits, so the batch closes at four although max_batch is 8.  Ten
    requests arriving at once therefore go out as 4 + 4 + 2 (without the
    doubling they would go 2 by 2, without the cap 8 + 2).  Then a mix of
    large and small requests on the same server.  Every result equals the
    oracle."""
    col = 32 * MiB
    host = synth.random_bytes(4 * col, seed=45)
    dev_pool = torch.from_numpy(host).to("cuda:0")
    big = dict(column=np.array([k % 4 for k in range(10)]), width=np.array([8, 16, 32, 64, 16] * 2),
               offset=np.array([3, 0, 5, 1, 0, 7, 2, 9, 4, 6]),
               arrival_ns=np.zeros(10, dtype=np.int64))
    big["length"] = col - big["offset"]  # 2048 tiles of 16 KiB, the last one partial
    cfg = ppc.ppc_server_cfg(1, 8, 0, 1, 0, 0, 0)  # one stream, 8 per batch, 1 tile per item
    server = ppc.ppc_server_create(dev_pool, column_bytes=col, cfg=cfg)
    try:
        results, stats = ppc.ppc_server_run_trace(server, big["column"], big["width"], big["offset"],
                                                  big["length"], big["arrival_ns"])
        assert ppc.ppc_server_get_stats(server)["max_batch_seen"] == 4
        assert stats["batches"] == 3
        check_all_against_oracle(host, big, results, col)
        mix = synth.serve_trace(300, seed=46, n_columns=4, column_bytes=col, rate_per_s=2e5, lo=1, hi=col)
        results, stats = ppc.ppc_server_run_trace(server, mix["column"], mix["width"], mix["offset"],
                                                  mix["length"], mix["arrival_ns"])
        check_all_against_oracle(host, mix, results, col)
    finally:
        ppc.ppc_server_destroy(server)


def test_batch_deadline_turns_into_timeout_status(ppc, pool):
    """A deadline shorter than any batch (1 us from launch): the first batch
    (800 MiB, far more than 1 us of device time) is still running when the
    host next looks, so the trace returns PPC_ETIMEDOUT instead of waiting,
    and the server then refuses new work.  The kernels themselves run to
    their normal end; destroy waits for them."""
    _, dev_pool = pool
    n = 200
    t = dict(column=np.arange(n) % N_COL, width=np.full(n, 16), offset=np.zeros(n, dtype=np.int64),
             length=np.full(n, COL_BYTES), arrival_ns=np.zeros(n, dtype=np.int64))
    cfg = ppc.ppc_server_cfg(1, 0, 0, 0, 0, 0, 1)
    server = ppc.ppc_server_create(dev_pool, column_bytes=COL_BYTES, cfg=cfg)
    try:
        with pytest.raises(ppc.PpcError) as e:
            ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"], t["arrival_ns"])
        assert e.value.status == ppc.PPC_ETIMEDOUT
        with pytest.raises(ppc.PpcError) as e:
            ppc.ppc_server_submit(server, 0, 16, 0, 64)
        assert e.value.status == ppc.PPC_ETIMEDOUT
    finally:
        ppc.ppc_server_destroy(server)
