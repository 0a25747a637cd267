"""GPU parity of list ranking by in-place list contraction (rp_list_rank):
ranks equal the oracle's list walk; the contraction records equal the
oracle's relaxed-PIP contraction run with the same block size."""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_01216_amd as rp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NIL = 0xFFFFFFFF


def lists(n, n_lists, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    prev = np.full(n, NIL, dtype=np.uint32)
    nxt = np.full(n, NIL, dtype=np.uint32)
    cuts = np.sort(rng.choice(np.arange(1, n), size=n_lists - 1, replace=False)) \
        if n_lists > 1 and n > n_lists else []
    for seq in np.split(perm, cuts):
        prev[seq[1:]] = seq[:-1]
        nxt[seq[:-1]] = seq[1:]
    return prev, nxt


def to_rec(prev, nxt):
    rec = np.empty((prev.shape[0], 2), dtype=np.uint64)
    rec[:, 0] = prev
    rec[:, 1] = nxt
    return torch.from_numpy(rec.view(np.int64)).to(DEV)


def check(prev, nxt, seed=0, eps=0.5, prio=None):
    n = prev.shape[0]
    rec = to_rec(prev, nxt)
    ptensor = None if prio is None else torch.from_numpy(prio.view(np.int64)).to(DEV)
    rank, st = rp.rp_list_rank(rec, seed=seed, eps=eps, prio=ptensor)
    assert st["status"] == 0
    assert st["aux_words"] <= max(st["aux_bound_words"], 4)
    want = oracle.list_rank(prev, nxt)
    got = rank.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
    out = rec.cpu().numpy().view(np.uint64)
    ref = oracle.list_contract(prev, nxt, st["k"], seed=seed, prio=prio)
    heads = prev == NIL
    nh = ~heads
    assert np.array_equal((out[nh, 0] & 0xFFFFFFFF).astype(np.uint32), ref["left"][nh])
    assert np.array_equal((out[nh, 0] >> 32), ref["offset"][nh])
    assert np.array_equal((out[nh, 1] & 0xFFFFFFFF).astype(np.uint32), ref["right"][nh])
    assert np.array_equal((out[nh, 1] >> 32).astype(np.uint32), ref["round"][nh])
    # heads: untouched prev, next word = NIL | list length
    assert np.all(out[heads, 0] == NIL)
    assert np.all((out[heads, 1] & 0xFFFFFFFF) == NIL)
    # every head's weight is its list's length: one more than the largest
    # rank reached from it (the ranks' list ids come from the walk)
    assert int((out[heads, 1] >> 32).sum()) == n
    tails = nxt == NIL
    assert sorted((out[heads, 1] >> 32).tolist()) == sorted((want[tails] + 1).tolist())
    assert st["contract_rounds"] == ref["rounds"]
    return st


@pytest.mark.parametrize("n,n_lists", [(1, 1), (2, 1), (5, 2), (1000, 1), (1000, 13),
                                       ((1 << 16) + 3, 1), ((1 << 16) + 3, 100),
                                       (1 << 20, 1), (1 << 20, 1000)])
@pytest.mark.parametrize("eps", [0.25, 0.5, 0.75])
def test_ranks_and_records(n, n_lists, eps):
    prev, nxt = lists(n, n_lists, n + n_lists)
    check(prev, nxt, seed=n_lists, eps=eps)


def test_explicit_priorities():
    n = 50000
    prev, nxt = lists(n, 3, 4)
    prio = np.random.default_rng(5).integers(0, 2**64, size=n, dtype=np.uint64)
    prio[:100] = 7          # ties are broken by index
    check(prev, nxt, prio=prio, eps=0.4)


def test_ordered_lists():
    n = 4097
    idx = np.arange(n, dtype=np.uint32)
    prev = np.concatenate([[NIL], idx[:-1]]).astype(np.uint32)
    nxt = np.concatenate([idx[1:], [NIL]]).astype(np.uint32)
    check(prev, nxt, seed=1, eps=0.5)
    check(nxt.copy(), prev.copy(), seed=2, eps=0.5)    # reversed: head is n-1


def test_large():
    n = 1 << 24
    prev, nxt = lists(n, 17, 99)
    st = check(prev, nxt, seed=3, eps=0.5)
    assert st["phases"] == -(-n // st["k"])


@pytest.mark.parametrize("eps", [0.125, 0.05])
def test_block_elements_per_lane(eps):
    """Blocks larger than the grid holds at one element per lane (here
    623K and 1.9M elements) are held with 2 or 4 per lane (which one depends
    on the kernels' occupancy); the records and ranks are the oracle's
    either way."""
    n = 1 << 22
    prev, nxt = lists(n, 5, 21)
    st = check(prev, nxt, seed=4, eps=eps)
    assert -(-st["k"] // (st["grid"] * 256)) in (2, 4), st


def test_rejects_inconsistent_links_untouched():
    n = 1000
    prev, nxt = lists(n, 1, 1)
    j = int(np.flatnonzero(nxt != NIL)[5])
    nxt[j] = (int(nxt[j]) + 1) % n        # prev of the new target is not j
    assert prev[nxt[j]] != j
    rec = to_rec(prev, nxt)
    before = rec.clone()
    with pytest.raises(rp.RpError):
        rp.rp_list_rank(rec, seed=1)
    assert torch.equal(rec, before)


def test_cycle_reported():
    n = 64
    prev, nxt = lists(n, 1, 3)
    head = int(np.flatnonzero(prev == NIL)[0])
    tail = int(np.flatnonzero(nxt == NIL)[0])
    prev[head] = tail
    nxt[tail] = head          # one cycle, no head: consistent links
    rec = to_rec(prev, nxt)
    _, st = rp.rp_list_rank(rec, seed=1, eps=0.5)
    assert st["status"] == rp.RP_EINVAL
