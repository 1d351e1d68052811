"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only makes bytes: it holds none of the counting arithmetic, and
both the oracle and the HIP path receive the very same buffers from it.

Recipes (all seeded; numpy ``default_rng`` = PCG64 on the host, torch's
Philox generator on the device for the large buffers):

* ``bernoulli`` -- bytes whose bits are i.i.d. Bernoulli(p), packed
  least-significant-bit first.  p = 0.5 is plain uniform random bytes.
* ``onehot_u8`` -- one-hot bytes ``1 << k`` with category k drawn from a
  truncated Zipf law P(k) proportional to (k+1)^-s (the one-hot GROUP BY use
  of Section 1).
* ``onehot_u32_columns`` -- the serving pool: one-hot 32-bit words over 32
  categories, Zipf s = 1.0, rank r on bit r-1.
* ``batch_spec`` -- the batched workload: log-uniform lengths, uniform widths,
  a per-array density p ~ U[0, 1].
* ``serve_trace`` -- a Poisson request stream over the serving pool.
"""
from __future__ import annotations

import math

import numpy as np

MiB = 1 << 20
GiB = 1 << 30
WIDTHS = (8, 16, 32, 64)


# ---------------------------------------------------------------- host side
def random_bytes(n: int, seed: int) -> np.ndarray:
    """n uniform random bytes: every bit Bernoulli(0.5)."""
    return np.random.default_rng(seed).integers(0, 256, size=n, dtype=np.uint8)


def bernoulli(n: int, p: float, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """n bytes whose 8n bits are i.i.d. Bernoulli(p), LSB-first packing."""
    if p == 0.5:
        return random_bytes(n, seed)
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint8)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        bits = rng.random((hi - lo) * 8) < p
        out[lo:hi] = np.packbits(bits, bitorder="little")
    return out


def zipf_probs(k: int, s: float) -> np.ndarray:
    """Truncated Zipf law over k ranks: P(r) proportional to r^-s, r = 1..k."""
    w = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def onehot_u8(n_words: int, seed: int, n_cat: int = 8, s: float = 1.1):
    """One-hot uint8 column: returns (bytes, categories).  Category k is
    stored as the byte 1 << k."""
    rng = np.random.default_rng(seed)
    cats = rng.choice(n_cat, size=n_words, p=zipf_probs(n_cat, s)).astype(np.uint8)
    return (np.uint8(1) << cats).astype(np.uint8), cats


def onehot_u32_columns(n_columns: int, words_per_column: int, seed: int,
                       n_cat: int = 32, s: float = 1.0):
    """Serving pool: n_columns one-hot uint32 columns laid end to end.
    Returns (pool bytes, categories per word)."""
    rng = np.random.default_rng(seed)
    n = n_columns * words_per_column
    cats = rng.choice(n_cat, size=n, p=zipf_probs(n_cat, s)).astype(np.uint32)
    words = (np.uint32(1) << cats).astype("<u4")
    return words.view(np.uint8), cats


def batch_spec(n_arrays: int, seed: int, lo: int = 16, hi: int = 16 * MiB,
               align: int = 256, start_jitter: int = 0):
    """Batched workload description.

    Lengths are log-uniform on [lo, hi] rounded down to a multiple of the
    array's word size; widths uniform on {8,16,32,64}; per-array density
    p ~ U[0,1].  Arrays are packed into one pool at ``align``-byte starts,
    plus an optional random start jitter in [0, start_jitter).
    Returns dict(offsets, lengths, widths, p, pool_bytes).
    """
    rng = np.random.default_rng(seed)
    widths = rng.choice(np.array(WIDTHS), size=n_arrays)
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_arrays))
    s = widths // 8
    lengths = np.maximum((raw.astype(np.int64) // s) * s, s).astype(np.int64)
    p = rng.uniform(0.0, 1.0, size=n_arrays)
    jitter = (rng.integers(0, start_jitter, size=n_arrays) if start_jitter > 0
              else np.zeros(n_arrays, dtype=np.int64))
    offsets = np.empty(n_arrays, dtype=np.int64)
    pos = 0
    for i in range(n_arrays):
        pos = (pos + align - 1) // align * align
        offsets[i] = pos + jitter[i]
        pos = offsets[i] + lengths[i]
    pool = (pos + align - 1) // align * align
    return dict(offsets=offsets, lengths=lengths, widths=widths.astype(np.int64),
                p=p, pool_bytes=int(pool))


def serve_trace(n_requests: int, seed: int, n_columns: int, column_bytes: int,
                rate_per_s: float, lo: int = 64, hi: int = 64 * MiB):
    """Poisson request stream over a pool of equal columns.

    Each request: column U{0..n_columns-1}, width U{8,16,32,64}, length
    log-uniform on [lo, min(hi, column_bytes)] in whole bytes, byte offset
    U[0, column_bytes - length].  Inter-arrival times are exponential with
    mean 1/rate.  Returns dict of numpy arrays (arrival_ns is int64).
    """
    rng = np.random.default_rng(seed)
    hi = min(hi, column_bytes)
    column = rng.integers(0, n_columns, size=n_requests)
    width = rng.choice(np.array(WIDTHS), size=n_requests)
    length = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_requests)).astype(np.int64)
    length = np.clip(length, lo, hi)
    offset = (rng.random(n_requests) * (column_bytes - length + 1)).astype(np.int64)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrival_ns = np.cumsum(gaps * 1e9).astype(np.int64)
    return dict(column=column.astype(np.int64), width=width.astype(np.int64),
                offset=offset, length=length, arrival_ns=arrival_ns)


def log_uniform_mean(lo: float, hi: float) -> float:
    """Mean of a log-uniform law on [lo, hi] (used to set Poisson rates)."""
    return (hi - lo) / math.log(hi / lo)


# -------------------------------------------------------------- device side
def device_bernoulli(n: int, p: float, seed: int, device="cuda", out=None):
    """n bytes of Bernoulli(p) bits generated on the GPU with torch's
    seeded generator (for buffers too large to make on the host quickly).
    The bytes are whatever this produces; checks read them back."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=device)
    if p == 0.5:
        chunk = 1 << 28
        for lo in range(0, n, chunk):
            hi = min(n, lo + chunk)
            out[lo:hi] = torch.randint(0, 256, (hi - lo,), generator=g,
                                       device=device, dtype=torch.uint8)
        return out
    weights = (2 ** torch.arange(8, device=device, dtype=torch.int32)).to(torch.uint8)
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        bits = torch.rand((hi - lo, 8), generator=g, device=device) < p
        out[lo:hi] = (bits.to(torch.uint8) * weights).sum(dim=1, dtype=torch.uint8)
    return out


def device_onehot_u32_columns(n_columns: int, words_per_column: int, seed: int, device="cuda",
                              n_cat: int = 32, s: float = 1.0):
    """Device-generated serving pool (same law as onehot_u32_columns, drawn
    with torch's seeded generator by inverse-CDF lookup).  Returns the pool
    as a uint8 device tensor."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    cdf = torch.tensor(np.cumsum(zipf_probs(n_cat, s)), dtype=torch.float64, device=device)
    cdf[-1] = 1.0
    n = n_columns * words_per_column
    out = torch.empty(n, dtype=torch.int32, device=device)
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        u = torch.rand(hi - lo, generator=g, device=device, dtype=torch.float64)
        cat = torch.searchsorted(cdf, u, right=True).clamp_(max=n_cat - 1)
        out[lo:hi] = torch.bitwise_left_shift(torch.ones_like(cat), cat).to(torch.int32)
    return out.view(torch.uint8)
