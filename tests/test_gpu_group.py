"""GPU parity of rp_shuffle_group: several shuffles in one cooperative launch,
each on its own group of workgroups.

Every request's output must be its own Knuth shuffle (the oracle), the same
bytes as a call of its own, with the plan (k, auxiliary words) a call of its
own on the same two-barrier rounds kernel would get; a bad request rejects the
whole group with every array untouched.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _want(n, seed):
    w = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(w, seed)
    return w


@pytest.mark.parametrize("eps", [0.5, 0.65, 0.4])
def test_group_equals_oracle(eps, monkeypatch):
    sizes = [(1 << 20) + 7, 1000, (1 << 18) + 3, 50_000, 2, 1]
    seeds = [11 * i + 3 for i in range(len(sizes))]
    arrays = [workloads.identity(n, torch.int64, DEV) for n in sizes]
    stats = rp.rp_shuffle_group(arrays, seeds=seeds, eps=eps)
    for A, n, sd, st in zip(arrays, sizes, seeds, stats):
        assert st["status"] == 0
        assert st["aux_words"] <= st["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
        assert np.array_equal(A.cpu().numpy(), _want(n, sd)), (n, eps)
        if n > 1:
            # group launches run every shuffle on the two-barrier rounds
            # kernel, planned as a call of its own on that kernel would be
            monkeypatch.setenv("RP_ONEBAR", "0")
            alone = rp.rp_plan(n, 8, eps, device=0)
            monkeypatch.delenv("RP_ONEBAR")
            assert st["k"] == alone["k"] and st["aux_words"] == alone["aux_words"]


def test_group_equals_calls_of_their_own(monkeypatch):
    sizes = [(1 << 24) + 5, 1 << 22, (1 << 23) + 1, 3 << 20]
    seeds = [5, 6, 7, 8]
    grouped = [workloads.identity(n, torch.int64, DEV) for n in sizes]
    alone = [workloads.identity(n, torch.int64, DEV) for n in sizes]
    stats = rp.rp_shuffle_group(grouped, seeds=seeds, eps=0.5)
    # the same kernel alone: identical rounds and attempts, not just bytes
    monkeypatch.setenv("RP_ONEBAR", "0")
    for A, B, sd, st in zip(grouped, alone, seeds, stats):
        s = rp.rp_shuffle_inplace(B, seed=sd, eps=0.5).get()
        assert st["status"] == 0 and s["status"] == 0
        assert torch.equal(A, B)
        assert st["rounds"] == s["rounds"] and st["attempts"] == s["attempts"]
    torch.cuda.empty_cache()


@pytest.mark.parametrize("eb", [4, 12, 16, 64])
def test_group_record_sizes(eb):
    sizes = [70_000, 4097, 300_001]
    rng = np.random.default_rng(eb)
    host = [rng.integers(0, 2**32, size=(n, eb // 4), dtype=np.uint32) for n in sizes]
    arrays = [torch.from_numpy(h.view(np.int32)).to(DEV) for h in host]
    stats = rp.rp_shuffle_group(arrays, seeds=[1, 2, 3], eps=0.5)
    for A, h, sd, st in zip(arrays, host, [1, 2, 3], stats):
        want = h.copy()
        oracle.knuth_shuffle_seed(want, sd)
        assert st["status"] == 0
        assert np.array_equal(A.cpu().numpy().view(np.uint32), want)


def test_group_explicit_targets_and_rejection():
    sizes = [5000, 20_000, 777]
    Hs = [workloads.uniform_targets(n, 40 + i) for i, n in enumerate(sizes)]
    arrays = [torch.arange(n, dtype=torch.int64, device=DEV) for n in sizes]
    stats = rp.rp_shuffle_group(arrays, H=[torch.from_numpy(h.view(np.int64)).to(DEV) for h in Hs],
                                eps=0.5)
    for A, n, h, st in zip(arrays, sizes, Hs, stats):
        want = np.arange(n, dtype=np.int64)
        oracle.knuth_shuffle(want, h)
        assert st["status"] == 0 and np.array_equal(A.cpu().numpy(), want)
    # one invalid target list rejects the whole group, every array untouched
    Hs[1][150] = 151
    arrays = [torch.arange(n, dtype=torch.int64, device=DEV) for n in sizes]
    with pytest.raises(rp.RpError) as e:
        rp.rp_shuffle_group(arrays, H=[torch.from_numpy(h.view(np.int64)).to(DEV) for h in Hs],
                            eps=0.5)
    assert e.value.code == rp.RP_EINVAL
    torch.cuda.synchronize()
    for A, n in zip(arrays, sizes):
        assert torch.equal(A.cpu(), torch.arange(n, dtype=torch.int64))


def test_group_rejections():
    a = workloads.identity(1000, torch.int64, DEV)
    b = workloads.identity(1000, torch.int32, DEV)
    with pytest.raises(rp.RpError):           # mixed record sizes
        rp.rp_shuffle_group([a, b], seeds=[1, 2], eps=0.5)
    many = [workloads.identity(100, torch.int64, DEV) for _ in range(17)]
    with pytest.raises(rp.RpError):           # more than 16
        rp.rp_shuffle_group(many, seeds=list(range(17)), eps=0.5)
    big = workloads.identity(1 << 22, torch.int64, DEV)
    with pytest.raises(rp.RpError):           # needs more than one slot per lane
        rp.rp_shuffle_group([big], seeds=[1], eps=0.05)
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), torch.arange(1000, dtype=torch.int64))
    assert torch.equal(big[:10].cpu(), torch.arange(10, dtype=torch.int64))


def test_group_of_sixteen_within_capacity():
    sizes = [(1 << 16) + 17 * i for i in range(16)]
    seeds = [100 + i for i in range(16)]
    arrays = [workloads.identity(n, torch.int64, DEV) for n in sizes]
    stats = rp.rp_shuffle_group(arrays, seeds=seeds, eps=0.5)
    for A, n, sd, st in zip(arrays, sizes, seeds, stats):
        assert st["status"] == 0 and np.array_equal(A.cpu().numpy(), _want(n, sd))


def test_group_beyond_capacity_is_refused(monkeypatch):
    cap = rp.rp_group_capacity(8)
    n, eps = 1 << 22, 0.35
    # the grid a group gives the shuffle: its two-barrier plan
    monkeypatch.setenv("RP_ONEBAR", "0")
    g = rp.rp_plan(n, 8, eps, device=0)["grid"]
    count = -(-(cap + 1) // g)
    if count > 16:
        pytest.skip(f"capacity {cap} not reachable with 16 requests of grid {g}")
    arrays = [workloads.identity(n, torch.int64, DEV) for _ in range(count)]
    with pytest.raises(rp.RpError) as e:
        rp.rp_shuffle_group(arrays, seeds=list(range(count)), eps=eps)
    assert e.value.code == rp.RP_EINVAL
    torch.cuda.synchronize()
    assert all(torch.equal(A[:8].cpu(), torch.arange(8, dtype=torch.int64)) for A in arrays)
    del arrays
    torch.cuda.empty_cache()
