"""GPU parity of the serving form (ppc_server_*).

Each served request must equal, bit for bit, the oracle on its bytes, the
plain call run alone on the same bytes, and the same request served alone
(tolerance 0) -- whatever batch it shared on the device.
"""
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


def served_alone(ppc, server, t, i):
    assert ppc.ppc_server_submit(server, t["column"][i], t["width"][i], t["offset"][i], t["length"][i],
                                 tag=10**9 + i) == ppc.PPC_OK
    while True:
        res = ppc.ppc_server_poll(server)
        if res:
            assert len(res) == 1 and res[0].tag == 10**9 + i and res[0].status == 0
            return np.array(res[0].counts[:res[0].width], dtype=np.uint64)


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
        while i < 200 or len(got) < 200:
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
        while not ppc.ppc_server_poll(server):
            pass
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


def test_full_size_pool_at_half_load(ppc):
    """The serving workload at full size, in the default server
    configuration the bench times: a 1 GiB pool of one-hot uint32 columns
    (16 x 64 MiB, 32 categories, Zipf s = 1.0) and 20,000 Poisson requests
    (64 B .. 64 MiB, unaligned) offered at about half the plain kernel's
    bandwidth.  Every result equals the plain call on the same bytes, a
    seeded sample equals the oracle, and sampled requests served alone
    equal their result in the mix (tolerance 0)."""
    col = 64 * MiB
    n = 20_000
    pool = synth.device_onehot_u32_columns(16, col // 4, seed=4, device="cuda:0")
    torch.cuda.synchronize()
    rate = 0.5 * 6.5e12 / synth.log_uniform_mean(64, 64 * MiB)
    t = synth.serve_trace(n, seed=4, n_columns=16, column_bytes=col, rate_per_s=rate, lo=64, hi=64 * MiB)
    server = ppc.ppc_server_create(pool, column_bytes=col)
    try:
        results, stats = ppc.ppc_server_run_trace(server, t["column"], t["width"], t["offset"], t["length"],
                                                  t["arrival_ns"])
        assert stats["n_requests"] == n and stats["mean_batch"] > 1.0
        plain = alone_plain(ppc, pool, t, col_bytes=col)
        for i in range(n):
            r = results[i]
            w = int(t["width"][i])
            assert r.tag == i and r.status == 0 and r.width == w
            assert np.array_equal(np.array(r.counts[:w], dtype=np.uint64), plain[i, :w]), "request %d" % i
        rng = np.random.default_rng(7)
        for i in rng.choice(n, size=60, replace=False):
            i = int(i)
            base = int(t["column"][i]) * col + int(t["offset"][i])
            host = pool[base:base + int(t["length"][i])].cpu().numpy()
            w = int(t["width"][i])
            assert np.array_equal(np.array(results[i].counts[:w], dtype=np.uint64), oracle.pospopcnt(host, w))
        for i in rng.choice(n, size=20, replace=False):
            i = int(i)
            w = int(t["width"][i])
            got = np.array(results[i].counts[:w], dtype=np.uint64)
            t_one = {k: t[k] for k in ("column", "width", "offset", "length")}
            assert np.array_equal(served_alone(ppc, server, t_one, i), got)
    finally:
        ppc.ppc_server_destroy(server)


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
