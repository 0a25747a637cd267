"""CPU oracle for the in-place random permutation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and shares no code with
it.

Contents
--------
* ``knuth_oracle.c`` (plain C, loaded here through ctypes): the sequential
  Knuth shuffle of Section 4.1 of Gu, Obeya and Shun, "Parallel In-Place
  Algorithms: Theory and Practice" (0-based: i = n-1 .. 0, swap A[i] and
  A[H[i]], 0 <= H[i] <= i), its seed-mode targets
  H[i] = splitmix64(seed ^ i) mod (i+1), and a sampled form that returns, for
  chosen output positions, the source index of the record that lands there.
* ``list_oracle.c`` (plain C): list ranking by walking each list (the
  definition), and the relaxed-PIP list contraction of Section 4.2 --
  Algorithm 2 applied to blocks of k elements in index order -- with the
  per-element contraction records (neighbours at splice time, offset to the
  left one, round).
* ``alg1.py`` (pure Python, small n): the round structure of the paper's
  Algorithm 1 (parallel Knuth shuffle by deterministic reservations) and its
  relaxed-PIP form that works on the first K unfinished swaps per round.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("knuth_oracle.c", "list_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle's C files with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_splitmix64.restype = _u64
        lib.oracle_splitmix64.argtypes = [_u64]
        lib.oracle_seed_target.restype = _u64
        lib.oracle_seed_target.argtypes = [_u64, _u64]
        lib.oracle_seed_targets.restype = None
        lib.oracle_seed_targets.argtypes = [_u64, _u64, _vp]
        lib.oracle_knuth_shuffle.restype = ctypes.c_int
        lib.oracle_knuth_shuffle.argtypes = [_vp, _u64, _u32, _vp]
        lib.oracle_knuth_shuffle_seed.restype = ctypes.c_int
        lib.oracle_knuth_shuffle_seed.argtypes = [_vp, _u64, _u32, _u64]
        lib.oracle_sample_sources.restype = ctypes.c_int
        lib.oracle_sample_sources.argtypes = [_u64, _vp, _vp, _u64, _vp]
        lib.oracle_sample_sources_seed.restype = ctypes.c_int
        lib.oracle_sample_sources_seed.argtypes = [_u64, _u64, _vp, _u64, _vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def splitmix64(x: int) -> int:
    """SplitMix64 output for one 64-bit input."""
    return int(_load().oracle_splitmix64(x & (2**64 - 1)))


def seed_target(seed: int, i: int) -> int:
    """H[i] = splitmix64(seed ^ i) mod (i + 1) for one index."""
    return int(_load().oracle_seed_target(seed & (2**64 - 1), i))


def seed_targets(n: int, seed: int) -> np.ndarray:
    """H[i] = splitmix64(seed ^ i) mod (i + 1) for i in [0, n), as uint64."""
    H = np.empty(n, dtype=np.uint64)
    _load().oracle_seed_targets(n, seed & (2**64 - 1), _ptr(H))
    return H


def _records_view(A: np.ndarray):
    if not A.flags.c_contiguous:
        raise ValueError("A must be C-contiguous")
    n = A.shape[0] if A.ndim else 0
    eb = A.itemsize * (int(np.prod(A.shape[1:])) if A.ndim > 1 else 1)
    return n, eb


def knuth_shuffle(A: np.ndarray, H: np.ndarray) -> None:
    """Permute A in place by the sequential Knuth shuffle with targets H.

    A's first axis indexes records; each record is the rest of the row.
    """
    n, eb = _records_view(A)
    H = np.ascontiguousarray(H, dtype=np.uint64)
    if H.shape != (n,):
        raise ValueError("H must have one target per record")
    rc = _load().oracle_knuth_shuffle(_ptr(A), n, eb, _ptr(H))
    if rc != 0:
        raise ValueError("invalid swap targets (some H[i] > i)")


def knuth_shuffle_seed(A: np.ndarray, seed: int) -> None:
    """Permute A in place by the Knuth shuffle with seed-mode targets."""
    n, eb = _records_view(A)
    rc = _load().oracle_knuth_shuffle_seed(_ptr(A), n, eb, seed & (2**64 - 1))
    if rc != 0:
        raise ValueError("bad arguments")


def sample_sources(n: int, positions, *, H: np.ndarray | None = None,
                   seed: int | None = None) -> np.ndarray:
    """Source index of the record that the shuffle leaves at each position.

    Exactly one of H (explicit targets) or seed (seed-mode targets) is given.
    Cost is one pass over the n targets, independent of the sample count.
    """
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    out = np.empty(pos.shape[0], dtype=np.uint64)
    lib = _load()
    if (H is None) == (seed is None):
        raise ValueError("give exactly one of H or seed")
    if H is not None:
        H = np.ascontiguousarray(H, dtype=np.uint64)
        if H.shape != (n,):
            raise ValueError("H must have length n")
        rc = lib.oracle_sample_sources(n, _ptr(H), _ptr(pos), pos.shape[0],
                                       _ptr(out))
    else:
        rc = lib.oracle_sample_sources_seed(n, seed & (2**64 - 1), _ptr(pos),
                                            pos.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("bad sample positions or targets")
    return out


# ------------------------------------------------------------- list oracle

NIL = 0xFFFFFFFF


def list_rank(prev: np.ndarray, nxt: np.ndarray) -> np.ndarray:
    """Position of every element in its list (heads 0), by walking the lists."""
    prev = np.ascontiguousarray(prev, dtype=np.uint32)
    nxt = np.ascontiguousarray(nxt, dtype=np.uint32)
    n = prev.shape[0]
    rank = np.empty(n, dtype=np.uint64)
    lib = _load()
    lib.oracle_list_rank.restype = ctypes.c_int
    lib.oracle_list_rank.argtypes = [_vp, _vp, _u64, _vp]
    if lib.oracle_list_rank(_ptr(prev), _ptr(nxt), n, _ptr(rank)) != 0:
        raise ValueError("malformed list (inconsistent links or a cycle)")
    return rank


def list_contract(prev: np.ndarray, nxt: np.ndarray, k: int, *, seed: int = 0,
                  prio: np.ndarray | None = None) -> dict:
    """The relaxed-PIP list contraction (blocks of k elements in index order,
    Algorithm 2 inside each block).  Returns the per-element records
    left, right, offset, round and the total number of rounds."""
    prev = np.ascontiguousarray(prev, dtype=np.uint32)
    nxt = np.ascontiguousarray(nxt, dtype=np.uint32)
    n = prev.shape[0]
    left = np.empty(n, dtype=np.uint32)
    right = np.empty(n, dtype=np.uint32)
    offset = np.empty(n, dtype=np.uint64)
    rnd = np.empty(n, dtype=np.uint32)
    total = ctypes.c_uint64(0)
    lib = _load()
    lib.oracle_list_contract.restype = ctypes.c_int
    lib.oracle_list_contract.argtypes = [_vp, _vp, _vp, _u64, _u64, _u64, _vp, _vp, _vp,
                                         _vp, ctypes.POINTER(_u64)]
    pr = None if prio is None else np.ascontiguousarray(prio, dtype=np.uint64)
    rc = lib.oracle_list_contract(_ptr(prev), _ptr(nxt), None if pr is None else _ptr(pr),
                                  seed & (2**64 - 1), n, int(k), _ptr(left), _ptr(right),
                                  _ptr(offset), _ptr(rnd), ctypes.byref(total))
    if rc != 0:
        raise ValueError("malformed list or k = 0")
    return {"left": left, "right": right, "offset": offset, "round": rnd,
            "rounds": int(total.value)}

