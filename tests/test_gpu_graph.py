"""Plain calls captured into a HIP graph.

The plain call launches with AMD's extended kernel launch; a caller may
record it into a graph (here torch.cuda.CUDAGraph, which captures the
library's launches on its capture stream).  Every replay must add exactly
the counts of one eager call.  Replays are interleaved with eager work and
synchronisations, and every replay is checked (tolerance 0)."""
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


def test_plain_and_popcount_calls_replay_exactly(ppc):
    dev = torch.device("cuda:0")
    # (width, bytes, start offset): the streaming-load path, an unaligned
    # multi-tile array, a one-block array and an edge-only array
    cases = [(8, 40 * MiB, 0), (16, 3 * MiB + 5, 3), (32, 1000, 5), (64, 7, 1)]
    hosts, bufs, want, counts = [], [], [], []
    for k, (w, n, off) in enumerate(cases):
        h = synth.bernoulli(n + off, 0.3 + 0.1 * k, seed=70 + k)
        hosts.append(h)
        bufs.append(torch.from_numpy(h).to(dev))
        want.append(oracle.pospopcnt(h[off:], w))
        counts.append(torch.zeros(w, dtype=torch.int64, device=dev))
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    want_total = oracle.popcount(hosts[1][3:])

    def calls():
        for (w, n, off), b, c in zip(cases, bufs, counts):
            ppc.ppc_pospopcnt(w, c, b[off:off + n])
        ppc.ppc_popcount(total, bufs[1][3:])

    # warm up on a side stream (the libraries' first launches), then clear
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls()
    torch.cuda.synchronize()
    for c in counts:
        c.zero_()
    total.zero_()
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    torch.cuda.synchronize()
    for c in counts:  # capturing runs nothing
        assert not c.any()
    assert not total.any()

    eager = torch.zeros(16, dtype=torch.int64, device=dev)
    for r in range(1, 6):
        g.replay()
        # the program's own eager work between replays
        x = torch.randn(512, 512, device=dev)
        y = (x @ x).abs().sum()
        ppc.ppc_pospopcnt16(eager, bufs[1][3:3 + cases[1][1]])
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for (w, _, _), c, wnt in zip(cases, counts, want):
            got = ppc.counts_to_numpy(c)
            assert np.array_equal(got, wnt * np.uint64(r)), "replay %d, w=%d" % (r, w)
        assert int(ppc.counts_to_numpy(total)[0]) == r * want_total, "replay %d, popcount" % r
        assert np.array_equal(ppc.counts_to_numpy(eager), want[1] * np.uint64(r))
