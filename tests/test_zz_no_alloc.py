"""The entry point that allocates nothing (rp_shuffle_inplace_noalloc),
through the C ABI, against rp_shuffle_inplace on the same inputs: every byte
equal, on consecutive calls that reuse the library's static scratch (the
second call smaller than the first, so stale words of the first are there),
and against the oracle.  Calls needing more than the scratch are rejected
with A untouched."""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _records(n, eb, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, size=(n, eb // 4), dtype=np.uint32)


def _both(host, **kw):
    """Run both entry points on copies of `host`; return the two results and
    the no-allocation call's statistics."""
    A1 = torch.from_numpy(host.view(np.int32)).to(DEV)
    A2 = A1.clone()
    s1 = rp.rp_shuffle_inplace(A1, **kw).get()
    s2 = rp.rp_shuffle_inplace_noalloc(A2, **kw).get()
    assert s1["status"] == 0 and s2["status"] == 0, (s1, s2)
    for f in ("k", "aux_words", "aux_bound_words", "grid", "table_slots"):
        assert s1[f] == s2[f], f
    return A1.cpu().numpy().view(np.uint32), A2.cpu().numpy().view(np.uint32), s2


# (n, elem_bytes, eps, seed, explicit targets): each call smaller than the last
CALLS = [
    (1 << 26, 8, 0.5, 1, False),
    ((1 << 22) + 7, 8, 0.5, 3, False),
    (300_001, 12, 0.3, 5, False),
    (65_536, 4, 0.75, 9, False),      # one workgroup, tables in LDS
    (40_000, 8, 0.5, 0, True),
    (1_000, 16, 0.5, 2, False),
]


def test_consecutive_calls_match_entry_point_and_oracle():
    for n, eb, eps, seed, hmode in CALLS:
        print(f"noalloc: n={n} eb={eb} eps={eps} seed={seed} H={hmode}", flush=True)
        host = _records(n, eb, seed + 100)
        want = host.copy()
        kw = {"eps": eps}
        if hmode:
            H = workloads.uniform_targets(n, seed + 7)
            kw["H"] = torch.from_numpy(H.view(np.int64)).to(DEV)
            oracle.knuth_shuffle(want, H)
        else:
            kw["seed"] = seed
            oracle.knuth_shuffle_seed(want, seed)
        got_ref, got, s = _both(host, **kw)
        assert np.array_equal(got, got_ref), (n, eb, eps)
        assert np.array_equal(got, want), (n, eb, eps)
        assert s["aux_words"] <= s["aux_bound_words"]


def test_repeat_after_larger_call():
    """A small call straight after a large one, twice, on the same stream."""
    for _ in range(2):
        for n in ((1 << 24) + 3, 5_003):
            print(f"noalloc repeat: n={n}", flush=True)
            A = workloads.identity(n, torch.int64, DEV)
            B = A.clone()
            rp.rp_shuffle_inplace(B, seed=11, eps=0.5, stats=False)
            rp.rp_shuffle_inplace_noalloc(A, seed=11, eps=0.5, stats=False)
            torch.cuda.synchronize()
            assert torch.equal(A, B), n


def test_too_big_is_rejected_and_A_untouched():
    n = 1 << 28
    print("noalloc reject: n=2^28 int32 eps=0.25", flush=True)
    plan = rp.rp_plan(n, 4, 0.25, 0)
    assert plan["aux_words"] * 8 > rp.RP_NOALLOC_SCRATCH_BYTES
    A = workloads.identity(n, torch.int32, DEV)
    with pytest.raises(rp.RpError) as ei:
        rp.rp_shuffle_inplace_noalloc(A, seed=1, eps=0.25)
    assert ei.value.code == rp.RP_ETOOBIG
    torch.cuda.synchronize()
    assert torch.equal(A, workloads.identity(n, torch.int32, DEV))


def test_allocation_failure_does_not_reach_it(monkeypatch):
    """With the library's allocations forced to fail, rp_shuffle_inplace
    returns RP_ENOMEM and the no-allocation entry point still runs."""
    n = (1 << 20) + 1
    print("noalloc under RP_FAIL_ALLOC", flush=True)
    monkeypatch.setenv("RP_FAIL_ALLOC", "1")
    A = workloads.identity(n, torch.int64, DEV)
    with pytest.raises(rp.RpError) as ei:
        rp.rp_shuffle_inplace(A, seed=4, eps=0.5)
    assert ei.value.code == rp.RP_ENOMEM
    rp.rp_shuffle_inplace_noalloc(A, seed=4, eps=0.5).get()
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, 4)
    assert np.array_equal(A.cpu().numpy(), want)
