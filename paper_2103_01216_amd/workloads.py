"""Seeded synthetic inputs for tests, the benchmark and the smoke check.

Holds none of the shuffle's arithmetic: only array initialisation (identity
arrays, 64-byte records) and explicitly drawn swap-target arrays.  The paper
measures its random permutation on synthetic 64-bit integer arrays (Section
7.4); these generators produce the same kind of input.

64-byte records: 16 uint32 fields; field 0 = record index (low 32 bits),
field f = low 32 bits of splitmix64(16 * index + f) for f = 1..15.
"""
from __future__ import annotations

import numpy as np

GOLD = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB


def _s64(c: int) -> int:
    """uint64 constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def splitmix64_torch(x):
    """SplitMix64 output on an int64 tensor holding uint64 bit patterns."""
    z = x + _s64(GOLD)
    z = (z ^ _lsr(z, 30)) * _s64(C1)
    z = (z ^ _lsr(z, 27)) * _s64(C2)
    return z ^ _lsr(z, 31)


def identity(n: int, dtype, device):
    import torch
    return torch.arange(n, dtype=dtype, device=device)


def records64(n: int, device, start: int = 0):
    """n records of 16 uint32 fields as an (n, 16) int32 tensor."""
    import torch
    out = torch.empty((n, 16), dtype=torch.int32, device=device)
    idx = torch.arange(start, start + n, dtype=torch.int64, device=device)
    out[:, 0] = (idx & 0xFFFFFFFF).to(torch.int32)
    for f in range(1, 16):
        v = splitmix64_torch(idx * 16 + f) & 0xFFFFFFFF
        out[:, f] = v.to(torch.int32)
    return out


def records64_numpy(idx: np.ndarray) -> np.ndarray:
    """The records for the given indices, on the host, as (len, 16) uint32."""
    idx = np.asarray(idx, dtype=np.uint64)
    out = np.empty((idx.shape[0], 16), dtype=np.uint32)
    out[:, 0] = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    with np.errstate(over="ignore"):
        for f in range(1, 16):
            z = idx * np.uint64(16) + np.uint64(f) + np.uint64(GOLD)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(C1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(C2)
            z = z ^ (z >> np.uint64(31))
            out[:, f] = (z & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out


def uniform_targets(n: int, seed: int) -> np.ndarray:
    """Exactly uniform H[i] in [0, i] (numpy Generator), as uint64."""
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.zeros(0, dtype=np.uint64)
    return rng.integers(0, np.arange(1, n + 1, dtype=np.int64)).astype(np.uint64)


def adversarial_targets(n: int, kind: str) -> np.ndarray:
    """Structured targets: 'zero' (one n-long chain), 'self' (all
    self-loops), 'prev' (H[i] = i-1), 'hot4' (targets among 4 locations)."""
    i = np.arange(n, dtype=np.int64)
    if kind == "zero":
        h = np.zeros(n, dtype=np.int64)
    elif kind == "self":
        h = i.copy()
    elif kind == "prev":
        h = np.maximum(i - 1, 0)
    elif kind == "hot4":
        h = np.minimum(i, i % 4)
    else:
        raise ValueError(kind)
    return h.astype(np.uint64)


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of the SplitMix64 generator whose state
    starts at `seed` (state += golden gamma, then the output mix), uint64."""
    state = (np.uint64(seed) + np.arange(1, count + 1, dtype=np.uint64) * np.uint64(GOLD))
    with np.errstate(over="ignore"):
        z = state
        z = (z ^ (z >> np.uint64(30))) * np.uint64(C1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(C2)
        return z ^ (z >> np.uint64(31))


def batch_sizes(count: int, lo_log2: float, hi_log2: float, seed: int) -> np.ndarray:
    """Log-uniform sizes n = floor(2^U), U = lo + (hi - lo) * u with u the top
    53 bits of the i-th SplitMix64 output (state starting at `seed`) / 2^53."""
    u = (splitmix64_stream(seed, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
