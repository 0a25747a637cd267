"""Pins of the list oracle (host only).

The list-ranking oracle is checked against lists built from known orders; the
contraction oracle (Algorithm 2 applied block by block, Section 4.2) against
what the contraction must produce whatever its schedule: every spliced
element sits between its nearest neighbours of higher key in the original
list (an independent stack computation), its offset is the distance to its
left one, the ranks rebuilt from the records are the list positions, and the
round counts of closed-form cases.
"""
import numpy as np
import pytest

import oracle

NIL = oracle.NIL


def make_lists(orders, n):
    """prev/next arrays for lists given as sequences of element ids."""
    prev = np.full(n, NIL, dtype=np.uint32)
    nxt = np.full(n, NIL, dtype=np.uint32)
    for seq in orders:
        for a, b in zip(seq[:-1], seq[1:]):
            nxt[a] = b
            prev[b] = a
    return prev, nxt


def random_lists(n, n_lists, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    cuts = np.sort(rng.choice(np.arange(1, n), size=n_lists - 1, replace=False)) if n_lists > 1 else []
    return [list(s) for s in np.split(perm, cuts)]


def keyfn(k, prio, heads):
    def key(x):
        if x in heads:
            return (float("inf"),)
        return (x // k, int(prio[x]), x)
    return key


def nearest_higher(orders, k, prio):
    """Independent: for every non-head element, the nearest elements of
    higher key to its left and right in its original list (stack scans)."""
    heads = {seq[0] for seq in orders}
    key = keyfn(k, prio, heads)
    left, right = {}, {}
    for seq in orders:
        stack = []
        for x in seq:
            while stack and key(stack[-1]) < key(x):
                stack.pop()
            left[x] = stack[-1] if stack else NIL
            stack.append(x)
        stack = []
        for x in reversed(seq):
            while stack and key(stack[-1]) < key(x):
                stack.pop()
            right[x] = stack[-1] if stack else NIL
            stack.append(x)
    return left, right, heads


def rebuild_ranks(rec, orders, n, k):
    """Ranks from the contraction records: heads 0, then blocks and rounds in
    reverse, rank(i) = rank(left(i)) + offset(i)."""
    heads = {seq[0] for seq in orders}
    rank = np.full(n, -1, dtype=np.int64)
    for h in heads:
        rank[h] = 0
    items = sorted((i for i in range(n) if i not in heads),
                   key=lambda i: (i // k, int(rec["round"][i])), reverse=True)
    for i in items:
        L = int(rec["left"][i])
        assert rank[L] >= 0
        rank[i] = rank[L] + int(rec["offset"][i])
    return rank


def test_rank_matches_construction():
    n = 5000
    orders = random_lists(n, 7, 1)
    prev, nxt = make_lists(orders, n)
    rank = oracle.list_rank(prev, nxt)
    for seq in orders:
        assert list(rank[seq]) == list(range(len(seq)))


def test_rank_rejects_malformed():
    prev, nxt = make_lists([[0, 1, 2, 3]], 4)
    nxt[3] = 0
    prev[0] = 3          # a cycle: no head
    with pytest.raises(ValueError):
        oracle.list_rank(prev, nxt)
    prev, nxt = make_lists([[0, 1, 2, 3]], 4)
    prev[2] = 0          # inconsistent link
    with pytest.raises(ValueError):
        oracle.list_rank(prev, nxt)


@pytest.mark.parametrize("n,n_lists,k", [(1, 1, 1), (2, 1, 1), (10, 1, 3), (200, 3, 16),
                                         (3000, 1, 3000), (3000, 5, 64), (4097, 2, 1000)])
def test_contraction_is_nearest_higher_key(n, n_lists, k):
    orders = random_lists(n, n_lists, n + k)
    prev, nxt = make_lists(orders, n)
    prio = np.random.default_rng(k).integers(0, 2**64, size=n, dtype=np.uint64)
    rec = oracle.list_contract(prev, nxt, k, prio=prio)
    left, right, heads = nearest_higher(orders, k, prio)
    pos = {}
    for seq in orders:
        for t, x in enumerate(seq):
            pos[x] = t
    for i in range(n):
        if i in heads:
            assert rec["left"][i] == NIL and rec["right"][i] == NIL
            continue
        assert rec["left"][i] == left[i], i
        assert rec["right"][i] == right[i], i
        assert int(rec["offset"][i]) == pos[i] - pos[int(left[i])]
    ranks = rebuild_ranks(rec, orders, n, k)
    assert np.array_equal(ranks.astype(np.uint64), oracle.list_rank(prev, nxt))


def test_closed_form_rounds():
    n = 50
    orders = [list(range(n))]           # one list in index order, head 0
    prev, nxt = make_lists(orders, n)
    inc = np.arange(n, dtype=np.uint64)
    # increasing along the list: only the first non-head element is ever a
    # local minimum, so one splice per round
    rec = oracle.list_contract(prev, nxt, n, prio=inc)
    assert rec["rounds"] == n - 1
    assert list(rec["round"][1:]) == list(range(n - 1))
    # decreasing: only the last element each time
    rec = oracle.list_contract(prev, nxt, n, prio=inc[::-1].copy())
    assert rec["rounds"] == n - 1
    assert list(rec["round"][1:]) == list(range(n - 2, -1, -1))
    # alternating low/high after the head: every low element is a local
    # minimum at once (round 0); the high ones only later
    alt = np.array([0] + [1 if i % 2 else 100 + i for i in range(1, n)], dtype=np.uint64)
    rec = oracle.list_contract(prev, nxt, n, prio=alt)
    lows = [i for i in range(1, n) if i % 2]
    assert all(rec["round"][i] == 0 for i in lows)
    assert all(rec["round"][i] > 0 for i in range(1, n) if i % 2 == 0)
    # k = 1: every block is one element, spliced in the block's first round
    rec = oracle.list_contract(prev, nxt, 1, prio=inc)
    assert all(r == 0 for r in rec["round"])
    assert rec["rounds"] == n - 1


def test_random_priorities_take_logarithmic_rounds():
    n = 1 << 14
    orders = random_lists(n, 1, 5)
    prev, nxt = make_lists(orders, n)
    rec = oracle.list_contract(prev, nxt, n, seed=3)
    assert rec["rounds"] < 8 * np.log2(n)


def test_seed_mode_is_splitmix_priorities():
    n = 777
    orders = random_lists(n, 2, 9)
    prev, nxt = make_lists(orders, n)
    prio = np.array([oracle.splitmix64(11 ^ i) for i in range(n)], dtype=np.uint64)
    a = oracle.list_contract(prev, nxt, 50, seed=11)
    b = oracle.list_contract(prev, nxt, 50, prio=prio)
    for f in ("left", "right", "offset", "round"):
        assert np.array_equal(a[f], b[f])
