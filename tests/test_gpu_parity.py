"""GPU parity: librp (through its C ABI) against the CPU oracle, bit-exact.

Every input is seeded and synthetic.  The result of a Knuth shuffle is unique
given (A, H), so the bar is equality of every byte, over the whole array at
every size, the largest benchmark configurations included.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle_cache
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(A, **kw):
    st = rp.rp_shuffle_inplace(A, **kw)
    s = st.get()
    assert s["status"] == 0, s
    return s


def _check_stats(s, n, H_np=None):
    assert s["aux_words"] <= s["aux_bound_words"]
    if H_np is not None:
        selfl = int(np.sum(H_np == np.arange(n, dtype=np.uint64)))
        nonself = n - selfl
        assert s["self_loops"] == selfl
        assert s["attempts"] == nonself + s["retries"]
        # each round attempts at most max_active swaps
        if s["max_active"] > 0:
            assert s["rounds"] >= -(-nonself // s["max_active"])
        # Each round either commits a swap (the top active one always wins)
        # or only retires self-loops while consuming k fresh indices.
        assert s["rounds"] <= nonself + -(-n // max(1, s["k"])) + 2


def _host_records(n, eb, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, size=(n, eb // 4), dtype=np.uint32)


# ---------------------------------------------------------------- H drawing

def test_seed_targets_exact_mod():
    rng = np.random.default_rng(5)
    idx = np.concatenate([
        np.arange(0, 1 << 16, dtype=np.uint64),
        rng.integers(0, 2**32, 20000, dtype=np.uint64),
        np.array([2**32 - 1, 2**32 - 2, 2**31 - 1, 2**31, 2**31 + 1]
                 + [2**j - 1 for j in range(1, 33)] + [2**j for j in range(32)],
                 dtype=np.uint64)])
    for seed in (0, 1, 2**64 - 1, 0xDEADBEEF):
        got = rp.rp_seed_targets(torch.from_numpy(idx.view(np.int64)).to(DEV), seed)
        got = got.cpu().numpy().view(np.uint64)
        want = np.array([oracle.seed_target(seed, int(i)) for i in idx[:2000]]
                        + [oracle.seed_target(seed, int(i)) for i in idx[2000:]],
                        dtype=np.uint64)
        assert np.array_equal(got, want), seed


# ------------------------------------------------------- small exact parity

@pytest.mark.parametrize("n", [2, 3, 7, 8, 1000, (1 << 16) + 3])
@pytest.mark.parametrize("eps", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("eb", [4, 8, 16, 64, 12, 252, 256])
def test_seed_mode_parity_small(n, eps, eb):
    for seed in (0, 1):
        host = _host_records(n, eb, seed + 17)
        want = host.copy()
        oracle.knuth_shuffle_seed(want, seed)
        A = torch.from_numpy(host.view(np.int32)).to(DEV)
        s = _run(A, seed=seed, eps=eps)
        got = A.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (n, eps, eb, seed, s)
        _check_stats(s, n, oracle.seed_targets(n, seed))


@pytest.mark.parametrize("seed", range(16))
def test_config_n2p20_int64_eps_half(seed):
    n = 1 << 20
    A = workloads.identity(n, torch.int64, DEV)
    s = _run(A, seed=seed, eps=0.5)
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, seed)
    assert np.array_equal(A.cpu().numpy(), want)
    assert s["aux_bound_words"] == 1024 and s["aux_words"] <= 1024
    if seed == 0:
        _check_stats(s, n, oracle.seed_targets(n, seed))


# ----------------------------------------------------------- explicit H

@pytest.mark.parametrize("kind", ["zero", "self", "prev", "hot4"])
@pytest.mark.parametrize("n", [2, 100, 3001])
def test_adversarial_targets(kind, n):
    H = workloads.adversarial_targets(n, kind)
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle(want, H)
    for eps in (0.3, 0.7):
        A = workloads.identity(n, torch.int64, DEV)
        s = _run(A, H=torch.from_numpy(H.view(np.int64)).to(DEV), eps=eps)
        assert np.array_equal(A.cpu().numpy(), want), (kind, n, eps)
        _check_stats(s, n, H)


@pytest.mark.parametrize("n", [1000, 50_000, 1 << 18])
def test_uniform_targets_parity(n):
    H = workloads.uniform_targets(n, 99)
    for eb in (4, 8, 64):
        host = _host_records(n, eb, 3)
        want = host.copy()
        oracle.knuth_shuffle(want, H)
        A = torch.from_numpy(host.view(np.int32)).to(DEV)
        s = _run(A, H=torch.from_numpy(H.view(np.int64)).to(DEV), eps=0.5)
        assert np.array_equal(A.cpu().numpy().view(np.uint32), want)
        _check_stats(s, n, H)


def test_seed_mode_equals_h_mode():
    n, seed = 200_000, 42
    H = oracle.seed_targets(n, seed)
    A1 = workloads.identity(n, torch.int64, DEV)
    A2 = A1.clone()
    _run(A1, seed=seed, eps=0.4)
    _run(A2, H=torch.from_numpy(H.view(np.int64)).to(DEV), eps=0.4)
    assert torch.equal(A1, A2)


def test_invalid_targets_leave_A_untouched():
    n = 10_000
    H = workloads.uniform_targets(n, 1)
    H[5000] = 5001
    A = workloads.identity(n, torch.int64, DEV)
    with pytest.raises(rp.RpError) as ei:
        rp.rp_shuffle_inplace(A, H=torch.from_numpy(H.view(np.int64)).to(DEV), eps=0.5)
    assert ei.value.code == rp.RP_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(A.cpu(), torch.arange(n))


def test_trivial_sizes():
    for n in (0, 1):
        A = torch.arange(n, dtype=torch.int64, device=DEV)
        s = rp.rp_shuffle_inplace(A, seed=3, eps=0.5).get()
        assert s["rounds"] == 0
        assert A.cpu().tolist() == list(range(n))


# ------------------------------------------------------ schedule invariance

@pytest.mark.parametrize("grid,slots", [("1", "1"), ("3", "2"), ("17", "4"), ("64", "8"), ("", "")])
def test_schedule_invariance(monkeypatch, grid, slots):
    n, seed = (1 << 18) + 11, 7
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, seed)
    monkeypatch.setenv("RP_GRID", grid)
    monkeypatch.setenv("RP_SLOTS", slots)
    for eps in (0.2, 0.5):
        A = workloads.identity(n, torch.int64, DEV)
        s = _run(A, seed=seed, eps=eps)
        assert np.array_equal(A.cpu().numpy(), want), (grid, slots, eps, s)
        if grid:
            assert s["grid"] <= int(grid)


def test_spare_words_widen_table():
    """When the grid, not the bound, limits the active swaps, the planner
    spends spare words on more reservation slots per swap; the output is the
    same Knuth shuffle."""
    n, seed = (1 << 24) + 5, 3
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, seed)
    A = workloads.identity(n, torch.int64, DEV)
    s = _run(A, seed=seed, eps=0.1)
    assert s["table_slots"] > s["k"], s
    assert s["aux_words"] <= s["aux_bound_words"]
    assert np.array_equal(A.cpu().numpy(), want)


def test_repeat_runs_identical():
    n = 300_001
    outs = []
    for _ in range(3):
        A = workloads.identity(n, torch.int32, DEV)
        _run(A, seed=11, eps=0.35)
        outs.append(A.cpu())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


# ------------------------------------------------------------ full sizes
#
# Every benchmark configuration is compared with the oracle over the whole
# array: the oracle shuffles the identity array on the host once per
# (n, seed) (tests/oracle_cache.py) and the comparison runs on the device.

def _equal_to_oracle(A, n, seed):
    want = oracle_cache.device_copy(n, seed, A.device)
    ok = bool(torch.equal(A.to(torch.int64), want))
    if not ok:
        bad = int((A.to(torch.int64) != want).sum())
        raise AssertionError(f"{bad} of {n} positions differ from the oracle")
    del want


@pytest.mark.parametrize("dtype", [torch.int32, torch.int64])
@pytest.mark.parametrize("eps", [0.25, 0.5, 0.75])
def test_n2p28(dtype, eps):
    n, seed = 1 << 28, 1
    print(f"n=2^28 {dtype} eps={eps}", flush=True)
    A = workloads.identity(n, dtype, DEV)
    s = _run(A, seed=seed, eps=eps)
    assert s["aux_words"] <= s["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
    _equal_to_oracle(A, n, seed)
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("eps", [0.2, 0.5])
def test_n2p30_int64(eps):
    n, seed = 1 << 30, 1
    print(f"n=2^30 int64 eps={eps}", flush=True)
    A = workloads.identity(n, torch.int64, DEV)
    s = _run(A, seed=seed, eps=eps)
    assert s["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
    assert s["aux_words"] <= s["aux_bound_words"]
    if eps == 0.5:
        assert s["aux_bound_words"] == 32768
    else:
        # the grid caps k; the spare words widen the reservation array
        assert s["table_slots"] > s["k"]
    _equal_to_oracle(A, n, seed)
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("eps", [0.25, 0.5])
def test_h_mode_n2p26(eps):
    """Explicit targets at a size that spans the whole grid: exactly uniform
    H[i] in [0, i] from a seeded host generator, read by the kernel instead of
    computed; the whole array against the oracle over the same H."""
    n = 1 << 26
    rng = np.random.default_rng(2026)
    H = rng.integers(0, np.arange(1, n + 1, dtype=np.int64), dtype=np.int64)
    A = workloads.identity(n, torch.int64, DEV)
    s = _run(A, H=torch.from_numpy(H).to(DEV), eps=eps)
    assert s["aux_words"] <= s["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
    assert s["self_loops"] == int(np.sum(H == np.arange(n)))
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle(want, H.astype(np.uint64))
    assert np.array_equal(A.cpu().numpy(), want)
    del A
    torch.cuda.empty_cache()


def test_records64_n2p26():
    """2^26 records of 64 bytes: every byte of the output equals the input
    record the oracle's permutation puts there."""
    n, seed = 1 << 26, 1
    A = workloads.records64(n, DEV)
    s = _run(A, seed=seed, eps=0.5)
    assert s["aux_bound_words"] == 8192 and s["aux_words"] <= 8192
    perm = oracle_cache.device_copy(n, seed, DEV)
    want = workloads.records64(n, DEV)[perm]
    assert torch.equal(A, want)
    del A, want, perm
    torch.cuda.empty_cache()


def test_rank_throttle_engages_under_full_parity(monkeypatch):
    """The refill throttle keeps every active swap's rank within the
    priority field; a lowered rank limit makes it engage at 2^20 and the
    output is still exactly the oracle's."""
    n, seed = 1 << 20, 4
    want = np.arange(n, dtype=np.int64)
    oracle.knuth_shuffle_seed(want, seed)
    for cap in ("700", "2000"):
        monkeypatch.setenv("RP_RANK_CAP", cap)
        A = workloads.identity(n, torch.int64, DEV)
        s = _run(A, seed=seed, eps=0.5)
        assert s["throttled_rounds"] > 0, s
        assert np.array_equal(A.cpu().numpy(), want), cap
    monkeypatch.delenv("RP_RANK_CAP")
    A = workloads.identity(n, torch.int64, DEV)
    s = _run(A, seed=seed, eps=0.5)
    assert s["throttled_rounds"] == 0
    assert np.array_equal(A.cpu().numpy(), want)


def test_inflight_words_reported():
    """Register-held state: source, target and both records per active
    swap, counted over the largest round (at least k)."""
    n = 1 << 20
    for dtype, eb in ((torch.int32, 4), (torch.int64, 8)):
        A = workloads.identity(n, dtype, DEV)
        s = _run(A, seed=2, eps=0.5)
        held = max(s["max_active"], s["k"])
        assert s["inflight_words"] == -(-held * (8 + 2 * eb) // 8)
        assert s["max_active"] <= s["k"] * 11 // 10
