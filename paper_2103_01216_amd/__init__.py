"""Python binding of librp (include/rp.h): argument marshalling only.

Every step of the shuffle runs in the HIP library; this module turns torch
tensors into device pointers and the current HIP stream into a stream handle,
and decodes the statistics record.  It raises if librp.so is missing: there
is no fallback path.

The operation is the Knuth shuffle of Gu, Obeya and Shun, "Parallel In-Place
Algorithms: Theory and Practice" (Section 4.1): for i = n-1 down to 0, swap
A[i] and A[H[i]], 0 <= H[i] <= i, computed in place with auxiliary space at
most floor(n^(1-eps)) 8-byte words.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librp.so")

RP_OK = 0
RP_PENDING = 1
RP_EINVAL = -1
RP_ENOMEM = -2
RP_EDEVICE = -3
RP_ETIMEOUT = -4

_ERRORS = {RP_EINVAL: "RP_EINVAL", RP_ENOMEM: "RP_ENOMEM",
           RP_EDEVICE: "RP_EDEVICE", RP_ETIMEOUT: "RP_ETIMEOUT"}

STATS_FIELDS = ("k", "aux_words", "aux_bound_words", "rounds", "attempts",
                "retries", "max_active", "self_loops", "grid",
                "slots_per_lane", "table_slots", "status")


class rp_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STATS_FIELDS[:-1]] + \
        [("status", ctypes.c_int64)]


class RpError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERRORS.get(code, code)}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded librp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2103_01216_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, vp, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        L.rp_aux_bound_words.restype = u64
        L.rp_aux_bound_words.argtypes = [u64, ctypes.c_double]
        L.rp_plan.restype = i32
        L.rp_plan.argtypes = [u64, u32, ctypes.c_double, i32, ctypes.POINTER(rp_stats)]
        L.rp_shuffle_inplace.restype = i32
        L.rp_shuffle_inplace.argtypes = [vp, u64, u32, vp, u64, ctypes.c_double, vp, vp]
        L.rp_seed_targets.restype = i32
        L.rp_seed_targets.argtypes = [vp, u64, u64, vp, vp]
        _lib = L
    return _lib


def _stats_dict(s: rp_stats) -> dict:
    return {f: int(getattr(s, f)) for f in STATS_FIELDS}


def rp_aux_bound_words(n: int, eps: float) -> int:
    """floor(n^(1-eps)), the auxiliary-space bound in 8-byte words."""
    return int(lib().rp_aux_bound_words(n, eps))


def rp_plan(n: int, elem_bytes: int, eps: float, device: int = -1) -> dict:
    """Launch shape, k and auxiliary words a call would use (host only)."""
    s = rp_stats()
    rc = lib().rp_plan(n, elem_bytes, eps, device, ctypes.byref(s))
    if rc != RP_OK:
        raise RpError(rc, "rp_plan")
    return _stats_dict(s)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _record_geometry(A):
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if not A.is_contiguous():
        raise ValueError("A must be contiguous")
    n = A.shape[0] if A.dim() > 0 else 0
    row = 1
    for d in A.shape[1:]:
        row *= d
    return n, A.element_size() * row


class PendingStats:
    """Statistics of one call, valid once the stream reaches its end."""

    def __init__(self, host, stream):
        self._host = host      # pinned torch tensor holding an rp_stats
        self._stream = stream

    def get(self) -> dict:
        self._stream.synchronize()
        s = rp_stats.from_address(self._host.data_ptr())
        return _stats_dict(s)


def rp_shuffle_inplace(A, *, H=None, seed: int = 0, eps: float = 0.5,
                       stream=None, stats: bool = True):
    """Permute A (device tensor, first axis = records) in place.

    H: device tensor of n targets (int64 or uint64, H[i] <= i) or None for
    seed mode, H[i] = splitmix64(seed ^ i) mod (i + 1).  Returns a
    PendingStats (or None with stats=False).  Raises RpError on an error
    code; A is then untouched.
    """
    import torch
    n, eb = _record_geometry(A)
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    hptr = None
    if H is not None:
        if not H.is_cuda or not H.is_contiguous() or H.element_size() != 8 \
                or H.numel() != n:
            raise ValueError("H must be a contiguous device tensor of n 64-bit targets")
        hptr = ctypes.c_void_p(H.data_ptr())
    host = None
    sptr = None
    if stats:
        host = torch.zeros(ctypes.sizeof(rp_stats) // 8, dtype=torch.int64,
                           pin_memory=True)
        sptr = ctypes.c_void_p(host.data_ptr())
    rc = lib().rp_shuffle_inplace(ctypes.c_void_p(A.data_ptr() if n else 0), n, eb,
                                  hptr, seed & (2**64 - 1), eps,
                                  ctypes.c_void_p(stream.cuda_stream), sptr)
    if rc != RP_OK:
        raise RpError(rc, "rp_shuffle_inplace")
    return PendingStats(host, stream) if stats else None


def rp_seed_targets(idx, seed: int, stream=None):
    """Device seed-mode targets for the indices in idx (device int64 tensor)."""
    import torch
    if not idx.is_cuda or idx.element_size() != 8 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous device tensor of 64-bit indices")
    out = torch.empty_like(idx)
    if stream is None:
        stream = torch.cuda.current_stream(idx.device)
    rc = lib().rp_seed_targets(ctypes.c_void_p(idx.data_ptr()), idx.numel(),
                               seed & (2**64 - 1), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(stream.cuda_stream))
    if rc != RP_OK:
        raise RpError(rc, "rp_seed_targets")
    return out
