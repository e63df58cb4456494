"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds none of the method's arithmetic: only key, value and query
generation.

The paper's experiments use 64-bit integer keys (section 5).  Here every key
set is the image of a counter under P, a keyed 4-round Feistel permutation of
64-bit words (32-bit halves, a round function built from 31-bit odd
multipliers).  P is a bijection whatever its round function, so

* members      key_i = P(2 i)          for i < n       (all distinct),
* non-members  neg_j = P(2 (n + j) + 1)                (distinct, disjoint),

and values are the low b bits of a second Feistel stream.  Query batches mix
members (drawn uniformly with replacement) and fresh non-members, each query
choosing its kind from a third stream.

All functions take and return int64 torch tensors holding the 64-bit patterns
and run unchanged on the CPU or a GPU, so the same seed gives bit-identical
inputs on both.  Every product is below 2^63 (member indices are scaled in
16-bit halves), so no signed overflow occurs.
"""
from __future__ import annotations

import torch

M32 = 0xFFFFFFFF
_C1 = 0x7FEB352D
_C2 = 0x2C1B3C6D


def _round_keys(key: int, rounds: int = 4) -> list[int]:
    # round keys from a small LCG on the Python side (plain integers)
    out, x = [], (key * 0x5851F42D4C957F2D + 0x14057B7EF767814F) & ((1 << 64) - 1)
    for _ in range(rounds):
        x = (x * 0x5851F42D4C957F2D + 0x14057B7EF767814F) & ((1 << 64) - 1)
        out.append((x >> 33) & M32)
    return out


def _f(x: torch.Tensor, k: int) -> torch.Tensor:
    y = ((x ^ k) * _C1) & M32
    y = y ^ (y >> 15)
    y = (y * _C2) & M32
    return y ^ (y >> 13)


def _join(hi: torch.Tensor, lo: torch.Tensor) -> torch.Tensor:
    # (hi << 32) | lo as an int64 bit pattern, without overflow
    hi_s = hi - ((hi >> 31) << 32)  # signed 32-bit reading of hi
    return hi_s * (1 << 32) + lo


def feistel(x: torch.Tensor, key: int) -> torch.Tensor:
    """Keyed 4-round Feistel permutation of 64-bit words (int64 patterns)."""
    lo = x & M32
    hi = (x >> 32) & M32
    for k in _round_keys(key):
        hi, lo = lo, hi ^ _f(lo, k)
    return _join(hi, lo)


def member_keys(n: int, data_seed: int, device="cpu") -> torch.Tensor:
    i = torch.arange(n, dtype=torch.int64, device=device)
    return feistel(2 * i, data_seed)


def negative_keys(n: int, count: int, data_seed: int, start: int = 0,
                  device="cpu") -> torch.Tensor:
    """count non-members P(2 (n + start + j) + 1)."""
    j = torch.arange(count, dtype=torch.int64, device=device)
    return feistel(2 * (n + start + j) + 1, data_seed)


def values(n: int, b: int, data_seed: int, device="cpu") -> torch.Tensor:
    """Uniform b-bit values (int64 patterns, b <= 64)."""
    i = torch.arange(n, dtype=torch.int64, device=device)
    v = feistel(i, data_seed ^ 0x5EED0001)
    if b >= 64:
        return v
    return v & ((1 << b) - 1) if b < 63 else v & 0x7FFFFFFFFFFFFFFF


def batch_values(n, b, data_seed: int, device="cpu") -> torch.Tensor:
    """Values of a batch: instance i's n[i] values are uniform b[i]-bit
    words (the low b[i] bits of one value stream, int64 patterns)."""
    import numpy as np
    total = int(np.sum(n))
    v = values(total, 64, data_seed, device=device)
    bits = torch.repeat_interleave(torch.as_tensor(np.asarray(b, dtype=np.int64), device=device),
                                   torch.as_tensor(np.asarray(n, dtype=np.int64), device=device))
    one = torch.ones_like(bits)
    mask = torch.where(bits >= 63, torch.full_like(bits, -1), (one << bits.clamp(max=62)) - 1)
    mask = torch.where(bits == 63, torch.full_like(bits, 0x7FFFFFFFFFFFFFFF), mask)
    return v & mask


def _scale(u: torch.Tensor, n: int) -> torch.Tensor:
    """floor(u * n / 2^32) for 32-bit u and n <= 2^32 without 64-bit
    overflow (u split into 16-bit halves)."""
    return ((u >> 16) * n + (((u & 0xFFFF) * n) >> 16)) >> 16


def queries(keys: torch.Tensor, q: int, data_seed: int, member_share_per_256: int = 128):
    """q queries: each is a member (uniform, with replacement) with
    probability member_share_per_256 / 256, else a fresh non-member.
    Returns (queries, is_member)."""
    n = keys.numel()
    device = keys.device
    j = torch.arange(q, dtype=torch.int64, device=device)
    r = feistel(j, data_seed ^ 0x0A5E7A11)
    is_member = ((r >> 56) & 0xFF) < member_share_per_256
    idx = _scale(r & M32, n)  # uniform in [0, n)
    neg = negative_keys(n, q, data_seed, start=0, device=device)
    out = torch.where(is_member, keys[idx], neg)
    return out, is_member


def batch_shape(count: int, data_seed: int, lo: int = 10, hi: int = 50000,
                bits=(1, 4, 8, 16, 32)):
    """Sizes and value widths of a batch of independent instances: sizes
    log-uniform in [lo, hi] (floor of exp of a uniform draw between ln lo and
    ln hi), widths uniform over bits, from numpy's PCG64 seeded with
    data_seed.  Returns two numpy arrays (uint64 sizes, int32 widths)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(data_seed))
    n = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), count)))
    n = np.clip(n, lo, hi).astype(np.uint64)
    b = rng.choice(np.asarray(bits, dtype=np.int32), count).astype(np.int32)
    return n, b


def queries_chunk(n: int, start: int, count: int, data_seed: int,
                  member_share_per_256: int = 128, device="cpu"):
    """Queries start .. start + count - 1 of the stream that queries(keys,
    q, data_seed) draws for the n member keys member_keys(n, data_seed),
    computed without the key array (members are recomputed from their
    index), so very large streams can be made in pieces.  Returns
    (queries, is_member)."""
    j = torch.arange(start, start + count, dtype=torch.int64, device=device)
    r = feistel(j, data_seed ^ 0x0A5E7A11)
    is_member = ((r >> 56) & 0xFF) < member_share_per_256
    idx = _scale(r & M32, n)
    mem = feistel(2 * idx, data_seed)
    neg = feistel(2 * (n + j) + 1, data_seed)
    return torch.where(is_member, mem, neg), is_member
