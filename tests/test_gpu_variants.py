"""GPU parity of the reservation variants (rp_shuffle_variant): each one must
give exactly the permutation of the sequential Knuth shuffle; they differ
only in rounds, retries and memory."""
import numpy as np
import pytest
import torch

import oracle
import oracle_cache
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
VARIANTS = ["oneres", "twores", "linear", "flat", "naive"]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", [2, 7, 1000, (1 << 16) + 3, 1 << 20])
def test_seed_mode_exact(variant, n):
    for seed in (1, 2):
        a = torch.arange(n, dtype=torch.int64, device=DEV)
        st = rp.rp_shuffle_variant(a, variant=variant, seed=seed, eps=0.5).get()
        want = np.arange(n, dtype=np.int64)
        oracle.knuth_shuffle_seed(want, seed)
        assert np.array_equal(a.cpu().numpy(), want)
        assert st["status"] == 0
        if variant == "linear":
            assert st["aux_words"] >= n
        else:
            assert st["aux_words"] <= st["aux_bound_words"]
        assert st["attempts"] == n - st["self_loops"] + st["retries"]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["zero", "self", "prev", "hot4"])
def test_structured_targets(variant, kind):
    n = 5000
    h = workloads.adversarial_targets(n, kind)
    H = torch.from_numpy(h.view(np.int64)).to(DEV)
    a = torch.arange(n, dtype=torch.int32, device=DEV)
    rp.rp_shuffle_variant(a, variant=variant, H=H, eps=0.5).get()
    want = np.arange(n, dtype=np.int32)
    oracle.knuth_shuffle(want, h)
    assert np.array_equal(a.cpu().numpy(), want)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("eps", [0.25, 0.75])
def test_eps_and_records(variant, eps):
    n = 20011
    host = np.random.default_rng(3).integers(0, 2**32, size=(n, 4), dtype=np.uint32)
    a = torch.from_numpy(host.view(np.int32)).to(DEV)
    rp.rp_shuffle_variant(a, variant=variant, seed=77, eps=eps).get()
    want = host.copy()
    oracle.knuth_shuffle_seed(want, 77)
    assert np.array_equal(a.cpu().numpy().view(np.uint32), want)


@pytest.mark.parametrize("variant", VARIANTS)
def test_large_equals_final(variant):
    n = 1 << 26
    a = torch.arange(n, dtype=torch.int64, device=DEV)
    b = torch.arange(n, dtype=torch.int64, device=DEV)
    rp.rp_shuffle_inplace(a, seed=5, eps=0.5, stats=False)
    st = rp.rp_shuffle_variant(b, variant=variant, seed=5, eps=0.5).get()
    assert st["status"] == 0
    assert torch.equal(a, b)
    assert torch.equal(b, oracle_cache.device_copy(n, 5, DEV))
