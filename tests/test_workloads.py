"""Seeded input generators (host only): the SplitMix64 stream that draws the
batched and served request sizes matches the published generator's outputs,
and the size recipe stays in its stated range."""
import os

import numpy as np

from paper_2103_01216_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.txt")


def test_stream_matches_published_outputs():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    want = [int(h, 16) for _, h in rows]
    got = workloads.splitmix64_stream(0, len(want))
    assert [int(x) for x in got] == want


def test_stream_equals_one_input_function():
    idx = np.arange(1, 65, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64(12345) + (idx - np.uint64(1)) * np.uint64(workloads.GOLD)
    import torch
    x = torch.from_numpy(states.view(np.int64))
    want = workloads.splitmix64_torch(x).numpy().view(np.uint64)
    assert np.array_equal(workloads.splitmix64_stream(12345, 64), want)


def test_batch_sizes_range_and_spread():
    s = workloads.batch_sizes(4096, 8, 20, 12345)
    assert s.min() >= 2 ** 8 and s.max() < 2 ** 20
    lg = np.log2(s)
    # log-uniform: each of the 12 octaves holds about 1/12 of the sizes
    counts = np.histogram(lg, bins=12, range=(8, 20))[0]
    assert counts.min() > 4096 / 12 * 0.75 and counts.max() < 4096 / 12 * 1.25
    assert np.array_equal(s, workloads.batch_sizes(4096, 8, 20, 12345))
