"""GPU parity of the accumulation-schedule variants (ppc_pospopcnt_variant).

The three schedules must give the oracle's counts exactly; only their cost
differs (measured by bench.py --ablation)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDTHS = (8, 16, 32, 64)


@pytest.fixture(scope="module")
def ppc():
    import paper_2412_16370_amd as ppc

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ppc.lib()
    return ppc


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_variants_match_oracle(ppc, variant):
    n_max = (64 << 20) + 77
    host = synth.bernoulli(n_max, 0.45, seed=70)
    buf = torch.from_numpy(host).to("cuda:0")
    for n in (0, 1, 17, 4095, 16384, 16385, 1_000_003, n_max - 13):
        for off in (0, 3, 13):
            for w in WIDTHS:
                counts = torch.zeros(w, dtype=torch.int64, device="cuda:0")
                ppc.ppc_pospopcnt_variant(variant, w, counts, buf[off:off + n])
                torch.cuda.synchronize()
                want = oracle.pospopcnt_mt(host[off:off + n], w, 16)
                assert np.array_equal(ppc.counts_to_numpy(counts), want), (variant, n, off, w)


@pytest.mark.parametrize("variant", [1, 2])
def test_variants_short_windows(ppc, variant):
    region = synth.random_bytes(400, seed=71)
    buf = torch.from_numpy(region).to("cuda:0")
    for w in WIDTHS:
        got = torch.zeros((16, 301, w), dtype=torch.int64, device="cuda:0")
        lib = ppc.lib()
        st = torch.cuda.current_stream().cuda_stream
        for o in range(16):
            for n in range(301):
                assert lib.ppc_pospopcnt_variant(variant, w, got.data_ptr() + ((o * 301) + n) * w * 8,
                                                 buf.data_ptr() + o, n, st) == 0
        torch.cuda.synchronize()
        want = oracle.sweep(region, w, 300, 16)
        assert np.array_equal(ppc.counts_to_numpy(got).reshape(16, 301, w), want)


def test_variant_argument_checks(ppc):
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    counts = torch.zeros(16, dtype=torch.int64, device="cuda:0")
    with pytest.raises(ppc.PpcError):
        ppc.ppc_pospopcnt_variant(3, 16, counts, buf)
    with pytest.raises(ppc.PpcError):
        ppc.ppc_pospopcnt_variant(1, 12, counts[:12], buf)
