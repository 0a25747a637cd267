"""GPU: the auxiliary bound checked where the memory is obtained, and the
error paths forced from the host.

rp_last_call_aux_bytes records the sizes the call passed to its allocation
calls and the dynamic LDS of its launch, independently of the plan that
rp_stats reports; it must stay within floor(n^(1-eps)) 8-byte words
(Section 3.2's auxiliary space) for every variant but the non-in-place one.
An injected allocation failure must leave A untouched, and a lowered round
limit must end the kernel normally with RP_ETIMEOUT and A a permutation of
its input.  Nothing here faults or stalls the device: both conditions are
set on the host.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("n,eps,eb", [(1000, 0.5, 16), ((1 << 16) + 3, 0.9, 4), (1 << 20, 0.5, 8),
                                      (1 << 20, 0.65, 8), ((1 << 18) + 1, 0.25, 8),
                                      ((1 << 24) + 5, 0.1, 8), ((1 << 16) + 3, 0.5, 12)])
@pytest.mark.parametrize("variant", ["final", "oneres", "twores"])
def test_allocated_aux_within_bound(n, eps, eb, variant):
    rows = np.random.default_rng(n).integers(0, 2**32, size=(n, eb // 4), dtype=np.uint32)
    A = torch.from_numpy(rows.view(np.int32)).to(DEV)
    s = rp.rp_shuffle_variant(A, variant=variant, seed=5, eps=eps).get()
    assert s["status"] == 0
    got = rp.rp_last_call_aux_bytes()
    bound = rp.rp_aux_bound_words(n, eps)
    assert s["aux_bound_words"] == bound
    assert 0 < got <= 8 * bound, (got, bound, s)
    # the plan's own count agrees with what was obtained (up to the 8-byte
    # padding of an odd slot count held in LDS)
    assert 8 * s["aux_words"] - 8 <= got <= 8 * s["aux_words"], (got, s)


def test_linear_variant_exceeds_bound_and_says_so():
    n = 1 << 20
    A = workloads.identity(n, torch.int64, DEV)
    s = rp.rp_shuffle_variant(A, variant="linear", seed=5, eps=0.5).get()
    got = rp.rp_last_call_aux_bytes()
    assert got >= 8 * n > 8 * s["aux_bound_words"]
    assert got <= 8 * s["aux_words"]


def test_injected_allocation_failure_leaves_A_untouched(monkeypatch):
    n = (1 << 16) + 3
    A = workloads.identity(n, torch.int64, DEV)
    monkeypatch.setenv("RP_FAIL_ALLOC", "1")
    with pytest.raises(rp.RpError) as e:
        rp.rp_shuffle_inplace(A, seed=1, eps=0.5)
    assert e.value.code == rp.RP_ENOMEM
    torch.cuda.synchronize()
    assert torch.equal(A.cpu(), torch.arange(n, dtype=torch.int64))
    assert rp.rp_last_call_aux_bytes() == 0
    monkeypatch.delenv("RP_FAIL_ALLOC")
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, 1)
    assert rp.rp_shuffle_inplace(A, seed=1, eps=0.5).get()["status"] == 0
    assert np.array_equal(A.cpu().numpy(), want)


@pytest.mark.parametrize("n,eps", [((1 << 16) + 3, 0.5), (1 << 20, 0.65), ((1 << 18) + 1, 0.2)])
def test_round_limit_ends_with_timeout(monkeypatch, n, eps):
    """A round limit below what the shuffle needs: every workgroup leaves at
    that round, the call reports RP_ETIMEOUT with exactly that many rounds,
    and A holds a permutation of its input (committed swaps are whole)."""
    A = workloads.identity(n, torch.int64, DEV)
    monkeypatch.setenv("RP_MAX_ROUNDS", "5")
    s = rp.rp_shuffle_inplace(A, seed=3, eps=eps).get()
    assert s["status"] == rp.RP_ETIMEOUT, s
    assert s["rounds"] == 5
    out = A.cpu().numpy()
    assert np.array_equal(np.sort(out), np.arange(n, dtype=np.int64))
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, 3)
    assert not np.array_equal(out, want)
    # without the limit the same call completes
    monkeypatch.delenv("RP_MAX_ROUNDS")
    A = workloads.identity(n, torch.int64, DEV)
    assert rp.rp_shuffle_inplace(A, seed=3, eps=eps).get()["status"] == 0
    assert np.array_equal(A.cpu().numpy(), want)
