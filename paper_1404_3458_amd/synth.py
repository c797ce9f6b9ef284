"""Seeded synthetic inputs (counter-based splitmix64).

This module holds no field or codec arithmetic: it only turns keys into
reproducible bytes, erasure patterns and workload shapes, so that the GPU
path, the CPU oracle and the benchmark regenerate identical inputs
independently.  Value ``i`` of the stream with key ``K`` is
``mix64(K + (i + 1) * 0x9E3779B97F4A7C15)`` where ``mix64`` is the
splitmix64 finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).

A key is derived from (base seed, config, stripe, stream) by folding each part
through ``mix64``.  Streams: DATA, ERASURE, SIZE, SHAPE, ARRIVAL.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 0x14043458
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

DATA, ERASURE, SIZE, SHAPE, ARRIVAL = 1, 2, 3, 4, 5


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def key(*parts: int, base: int = BASE_SEED) -> int:
    """Fold integer parts into one 64-bit stream key."""
    k = mix64(base)
    for p in parts:
        k = mix64(k ^ (int(p) & MASK64))
    return k


def u64(k: int, count: int, start: int = 0) -> np.ndarray:
    """Values start..start+count-1 of the stream with key k (numpy uint64)."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(k) + idx * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def random_bytes(k: int, nbytes: int) -> np.ndarray:
    """nbytes uniform bytes: the little-endian bytes of the u64 stream."""
    words = (nbytes + 7) // 8
    return u64(k, words).view(np.uint8)[:nbytes].copy()


def _signed(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def random_bytes_torch(k: int, nbytes: int, device="cpu", start_word: int = 0, out=None):
    """Same bytes as :func:`random_bytes`, generated with torch on ``device``.

    int64 arithmetic wraps modulo 2^64; right shifts are made logical with a
    mask.  ``start_word`` selects a window of the stream (for chunked fills);
    ``out`` (optional) is a uint8 tensor of nbytes to fill in place.
    """
    import torch

    words = (nbytes + 7) // 8
    idx = torch.arange(start_word + 1, start_word + words + 1, dtype=torch.int64, device=device)
    z = idx * _signed(GOLDEN) + _signed(k)

    def lsr(x, s):
        return (x >> s) & ((1 << (64 - s)) - 1)

    z = (z ^ lsr(z, 30)) * _signed(M1)
    z = (z ^ lsr(z, 27)) * _signed(M2)
    z = z ^ lsr(z, 31)
    b = z.view(torch.uint8)[:nbytes]
    if out is None:
        return b.clone()
    out.copy_(b)
    return out


def fill_random_torch(k: int, t, chunk_bytes: int = 1 << 28):
    """Fill a contiguous uint8 tensor with the stream's bytes, in chunks."""
    flat = t.view(-1)
    n = flat.numel()
    assert chunk_bytes % 8 == 0
    for off in range(0, n, chunk_bytes):
        m = min(chunk_bytes, n - off)
        random_bytes_torch(k, m, device=t.device, start_word=off // 8, out=flat[off:off + m])
    return t


def erasure_mask(k: int, n: int, e: int) -> np.ndarray:
    """uint8[n] with exactly e ones: the e positions with the smallest stream
    values (a uniform e-subset; ties broken by position)."""
    if e < 0 or e > n:
        raise ValueError("bad erasure count")
    v = u64(k, n)
    pos = np.argsort(v, kind="stable")[:e]
    m = np.zeros(n, dtype=np.uint8)
    m[pos] = 1
    return m


def uniform_int(k: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count integers uniform on [lo, hi] (inclusive), via 53-bit fractions."""
    v = u64(k, count)
    frac = (v >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return (lo + np.floor(frac * (hi - lo + 1))).astype(np.int64)


def uniform_float(k: int, count: int) -> np.ndarray:
    """count floats uniform on [0, 1)."""
    v = u64(k, count)
    return (v >> np.uint64(11)).astype(np.float64) / float(1 << 53)


# (n, k) classes of the mixed-stripe workload
MIXED_CLASSES = ((16, 8), (64, 48), (256, 224), (1024, 512), (4096, 2048))


def mixed_stripes(cfg_id: int, count: int, classes=MIXED_CLASSES, smin: int = 1024, smax: int = 65536):
    """Shapes of a mixed batch: per stripe (n, k, shard_bytes, erasures) with
    the class uniform over ``classes``, the shard length log-uniform on
    [smin, smax] rounded to an even byte count, and the erasure count uniform
    on [0, n - k].  Erasure positions come from :func:`erasure_mask` with key
    (cfg_id, stripe, ERASURE)."""
    cls = uniform_int(key(cfg_id, SHAPE), count, 0, len(classes) - 1)
    u = uniform_float(key(cfg_id, SIZE), count)
    f = uniform_float(key(cfg_id, ERASURE), count)
    out = []
    for i in range(count):
        n, k = classes[int(cls[i])]
        sb = 2 * int(round(smin * (smax / smin) ** float(u[i]) / 2))
        sb = min(max(sb, smin), smax)
        e = int(np.floor(f[i] * (n - k + 1)))
        out.append((n, k, sb, min(e, n - k)))
    return out
