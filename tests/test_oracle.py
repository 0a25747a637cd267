"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself or retypes its loop: each
checks it against a value the paper prints, a published reference output, a
closed form derived by hand, a bijection/uniformity property of the Knuth
shuffle, or an independent implementation of a different algorithm from the
paper (Algorithm 1's rounds) that the paper proves reaches the same result.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.alg1 import parallel_knuth_rounds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GOLD = 0x9E3779B97F4A7C15
M64 = 2**64 - 1


def _shuffled(A, H):
    A = np.array(A, copy=True)
    oracle.knuth_shuffle(A, np.asarray(H, dtype=np.uint64))
    return A


# ---------------------------------------------------------------- SplitMix64

def test_splitmix64_matches_published_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_state0.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 4
    for k, hexout in rows:
        x = (int(k) * GOLD) & M64
        assert oracle.splitmix64(x) == int(hexout, 16)


def test_seed_targets_compose_xor_and_mod():
    n, seed = 5000, 0xDEADBEEFCAFEF00D
    H = oracle.seed_targets(n, seed)
    for i in [0, 1, 2, 3, 17, 255, 256, 4095, n - 1]:
        assert int(H[i]) == oracle.splitmix64(seed ^ i) % (i + 1)
    assert np.all(H <= np.arange(n, dtype=np.uint64))
    assert H[0] == 0


def test_seed_targets_edge_seeds():
    for seed in (0, M64):
        H = oracle.seed_targets(64, seed)
        for i in (0, 1, 63):
            assert int(H[i]) == oracle.splitmix64(seed ^ i) % (i + 1)


# ------------------------------------------------- the paper's worked example

def _fig3():
    g = json.load(open(os.path.join(GOLDEN, "paper_fig3_example.json")))
    H0 = [h - 1 for h in g["H"]]  # 1-based -> 0-based
    first = sorted((a - 1, b - 1) for a, b in g["first_step_swaps"])
    return H0, first


def test_paper_example_first_parallel_step():
    H0, first = _fig3()
    A = list(range(len(H0)))
    _, rounds = parallel_knuth_rounds(A, H0)
    assert sorted(rounds[0]) == sorted(first)


def test_paper_example_first_step_same_under_single_reservation():
    H0, first = _fig3()
    _, rounds = parallel_knuth_rounds(list(range(8)), H0, rule="oneres")
    assert sorted(rounds[0]) == sorted(first)


def test_paper_example_sequential_result():
    # Sequential loop by hand, 1-based, A = [1..8]:
    #  i=8 swap(8,2) -> 1 8 3 4 5 6 7 2     i=4 swap(4,4) -> unchanged
    #  i=7 swap(7,4) -> 1 8 3 7 5 6 4 2     i=3 swap(3,2) -> 1 6 5 7 8 3 4 2
    #  i=6 swap(6,3) -> 1 8 6 7 5 3 4 2     i=2 swap(2,1) -> 6 1 5 7 8 3 4 2
    #  i=5 swap(5,2) -> 1 5 6 7 8 3 4 2     i=1 swap(1,1) -> unchanged
    H0, _ = _fig3()
    out = _shuffled(np.arange(1, 9, dtype=np.int64), H0)
    assert out.tolist() == [6, 1, 5, 7, 8, 3, 4, 2]
    A1, rounds = parallel_knuth_rounds(list(range(1, 9)), H0)
    assert A1 == out.tolist()
    # Algorithm 1 on the full prefix: the chains of the figure drain in
    # {8-2, 7-4, 6-3}, {5-2, 4 self}, {3-2}, {2-1}, {1 self}.
    assert [[(a + 1, b + 1) for a, b in r] for r in rounds] == [
        [(6, 3), (7, 4), (8, 2)], [(4, 4), (5, 2)], [(3, 2)], [(2, 1)], [(1, 1)]]


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1001])
def test_closed_forms(n):
    A = np.arange(n, dtype=np.int64) * 3 + 11
    idx = np.arange(n, dtype=np.uint64)
    # H[i] = i: every swap is a self-loop -> identity.
    assert np.array_equal(_shuffled(A, idx), A)
    # H = 0: swaps (n-1,0), (n-2,0), ... carry A[j+1] into j -> left rotation.
    assert np.array_equal(_shuffled(A, np.zeros(n, np.uint64)), np.roll(A, -1))
    # H[i] = i-1 (H[0] = 0): adjacent swaps from the top -> right rotation.
    Hm = np.maximum(idx.astype(np.int64) - 1, 0).astype(np.uint64)
    assert np.array_equal(_shuffled(A, Hm), np.roll(A, 1))


def test_records_move_whole():
    n, eb = 257, 64
    rng = np.random.default_rng(3)
    A = rng.integers(0, 2**32, size=(n, eb // 4), dtype=np.uint32)
    H = np.array([rng.integers(0, i + 1) for i in range(n)], dtype=np.uint64)
    out = A.copy()
    oracle.knuth_shuffle(out, H)
    # Row-wise result equals shuffling the row indices and gathering.
    perm = _shuffled(np.arange(n, dtype=np.int64), H)
    assert np.array_equal(out, A[perm])


# ---------------------------------------------------- bijection / uniformity

@pytest.mark.parametrize("n", range(1, 9))
def test_all_target_vectors_give_each_permutation_once(n):
    seen = set()
    base = np.arange(n, dtype=np.int64)
    for H in itertools.product(*[range(i + 1) for i in range(n)]):
        seen.add(tuple(_shuffled(base, H).tolist()))
    assert len(seen) == math.factorial(n)
    assert seen == set(itertools.permutations(range(n)))


@pytest.mark.parametrize("n", [5, 6])
def test_chi_square_uniform_targets(n):
    cells = math.factorial(n)
    trials = cells * 60
    rng = np.random.default_rng(20210301 + n)
    counts = {}
    base = np.arange(n, dtype=np.int64)
    for _ in range(trials):
        H = np.array([rng.integers(0, i + 1) for i in range(n)], dtype=np.uint64)
        key = tuple(_shuffled(base, H).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == cells
    obs = np.array(list(counts.values()), dtype=np.float64)
    _, p = stats.chisquare(obs)
    assert p > 1e-3


# ------------------------------------------------------ validity and errors

def test_output_is_permutation_large():
    n = 1 << 18
    A = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(A, 7)
    assert np.array_equal(np.sort(A), np.arange(n))
    assert not np.array_equal(A, np.arange(n))


def test_seed_mode_equals_explicit_targets():
    n, seed = 50_000, 123
    A = np.arange(n, dtype=np.int64)
    B = A.copy()
    oracle.knuth_shuffle_seed(A, seed)
    oracle.knuth_shuffle(B, oracle.seed_targets(n, seed))
    assert np.array_equal(A, B)


def test_invalid_targets_rejected_untouched():
    A = np.arange(10, dtype=np.int64)
    H = np.zeros(10, np.uint64)
    H[6] = 7
    with pytest.raises(ValueError):
        oracle.knuth_shuffle(A, H)
    assert np.array_equal(A, np.arange(10))


def test_empty_and_single():
    A = np.zeros(0, np.int64)
    oracle.knuth_shuffle(A, np.zeros(0, np.uint64))
    B = np.array([42], np.int64)
    oracle.knuth_shuffle(B, np.zeros(1, np.uint64))
    assert B.tolist() == [42]


# ---------------------------------------------------------- sampled oracle

@pytest.mark.parametrize("seed", [0, 1, 99])
def test_sampled_sources_match_full_shuffle(seed):
    n = (1 << 16) + 3
    full = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(full, seed)
    rng = np.random.default_rng(seed)
    pos = np.concatenate([[0, 1, n - 2, n - 1], rng.integers(0, n, 300), [5, 5]])
    src = oracle.sample_sources(n, pos, seed=seed)
    assert np.array_equal(src.astype(np.int64), full[pos])
    H = oracle.seed_targets(n, seed)
    assert np.array_equal(oracle.sample_sources(n, pos, H=H), src)


def test_sampled_sources_closed_form():
    n = 1000
    pos = np.arange(n)
    src = oracle.sample_sources(n, pos, H=np.zeros(n, np.uint64))
    assert np.array_equal(src.astype(np.int64), (pos + 1) % n)


# ------------------------------------------ Algorithm 1 rounds vs the loop

@pytest.mark.parametrize("prefix", [None, 1, 2, 7, 64])
@pytest.mark.parametrize("rule", ["alg1", "oneres"])
def test_rounds_reach_sequential_result(prefix, rule):
    rng = np.random.default_rng(11)
    for n in (1, 2, 9, 300):
        H = [int(rng.integers(0, i + 1)) for i in range(n)]
        A, rounds = parallel_knuth_rounds(list(range(n)), H, prefix, rule)
        assert A == _shuffled(np.arange(n, dtype=np.int64), H).tolist()
        done = set()
        for r in rounds:
            locs = [x for s, h in r for x in ((s,) if s == h else (s, h))]
            assert len(locs) == len(set(locs))  # winners are location-disjoint
            assert r, "every round commits at least the top unfinished swap"
            top = max(set(range(n)) - done)
            assert top in {s for s, _ in r}
            done |= {s for s, _ in r}
        assert done == set(range(n))
        if prefix is not None:
            assert len(rounds) >= math.ceil(n / prefix)
