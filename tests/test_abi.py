"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/rp.h declares, plans within the auxiliary bound, and rejects
bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert "rp_shuffle_inplace" in names
    L = rp.lib()
    for name in names:
        assert hasattr(L, name), name


def test_stats_struct_matches_header():
    text = open(HEADER).read()
    body = text[text.index("typedef struct rp_stats"):text.index("} rp_stats;")]
    fields = re.findall(r"(?:uint64_t|int64_t)\s+([a-z_]+);", body)
    assert tuple(fields) == rp.STATS_FIELDS
    assert ctypes.sizeof(rp.rp_stats) == 8 * len(fields)


@pytest.mark.parametrize("n,eps,expect", [
    (1 << 20, 0.5, 1024),
    (1 << 28, 0.25, 2097152),
    (1 << 28, 0.5, 16384),
    (1 << 28, 0.75, 128),
    (1 << 30, 0.5, 32768),
    (1 << 26, 0.5, 8192),
    (1, 0.5, 1),
    (7, 0.9, 1),
    (1000, 0.5, 31),
])
def test_aux_bound(n, eps, expect):
    assert rp.rp_aux_bound_words(n, eps) == expect


def test_aux_bound_is_floor():
    for n in [2, 3, 10, 999, 12345, 10**6, 10**8, 2**31 + 7]:
        for eps in [0.1, 0.2, 1 / 3, 0.5, 0.6, 0.9]:
            b = rp.rp_aux_bound_words(n, eps)
            x = n ** (1 - eps)
            assert b <= x * (1 + 1e-12) and b + 1 > x * (1 - 1e-12)


@pytest.mark.parametrize("n", [2, 3, 8, 1000, 1 << 16, 1 << 20, 1 << 26, 1 << 28, 1 << 30])
@pytest.mark.parametrize("eps", [0.1, 0.25, 0.5, 0.75, 0.9])
@pytest.mark.parametrize("eb", [4, 8, 64])
def test_plan_within_bound(n, eps, eb):
    p = rp.rp_plan(n, eb, eps)
    assert 1 <= p["k"] <= max(1, n)
    assert p["aux_words"] <= p["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
    assert p["k"] <= p["grid"] * 256 * p["slots_per_lane"]


def test_plan_scales_with_bound():
    small = rp.rp_plan(1 << 30, 8, 0.75)["k"]
    mid = rp.rp_plan(1 << 30, 8, 0.5)["k"]
    big = rp.rp_plan(1 << 30, 8, 0.25)["k"]
    assert small < mid < big


@pytest.mark.parametrize("eb", [0, 3, 6, 260])
def test_rejects_bad_elem_bytes(eb):
    rc = rp.lib().rp_shuffle_inplace(ctypes.c_void_p(16), 10, eb, None, 0, 0.5, None, None)
    assert rc == rp.RP_EINVAL


@pytest.mark.parametrize("eps", [0.0, 1.0, -0.5, 1.5, float("nan")])
def test_rejects_bad_eps(eps):
    rc = rp.lib().rp_shuffle_inplace(ctypes.c_void_p(16), 10, 8, None, 0, eps, None, None)
    assert rc == rp.RP_EINVAL


def test_rejects_huge_n_and_null():
    L = rp.lib()
    assert L.rp_shuffle_inplace(ctypes.c_void_p(16), 1 << 32, 8, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_inplace(None, 5, 8, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert L.rp_plan(1 << 32, 8, 0.5, -1, None) == rp.RP_EINVAL


def test_trivial_sizes_are_noops_without_device():
    L = rp.lib()
    s = rp.rp_stats()
    assert L.rp_shuffle_inplace(None, 0, 8, None, 0, 0.5, None, ctypes.byref(s)) == rp.RP_OK
    assert L.rp_shuffle_inplace(ctypes.c_void_p(16), 1, 8, None, 0, 0.5, None, ctypes.byref(s)) == rp.RP_OK
    assert s.rounds == 0
    # nothing was allocated by either call
    assert rp.rp_last_call_aux_bytes() == 0


def test_rejects_misaligned_arrays():
    """Records move in 8-byte words when their size is a multiple of 8 and in
    4-byte words otherwise; targets, list words and ranks are 64-bit.  A
    misaligned array is refused before any device work."""
    L = rp.lib()
    assert L.rp_shuffle_inplace(ctypes.c_void_p(4), 5, 8, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_inplace(ctypes.c_void_p(2), 5, 12, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_inplace(ctypes.c_void_p(12), 5, 64, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_inplace(ctypes.c_void_p(16), 5, 8, ctypes.c_void_p(4), 0, 0.5, None,
                                None) == rp.RP_EINVAL
    assert L.rp_shuffle_variant(ctypes.c_void_p(4), 5, 8, None, 0, 0.5, 0, None, None) == rp.RP_EINVAL
    rec = rp._list_lib().rp_list_rank
    assert rec(ctypes.c_void_p(4), 5, None, 0, 0.5, ctypes.c_void_p(16), None, None) == rp.RP_EINVAL
    assert rec(ctypes.c_void_p(16), 5, None, 0, 0.5, ctypes.c_void_p(20), None, None) == rp.RP_EINVAL
    assert rec(ctypes.c_void_p(16), 5, ctypes.c_void_p(3), 0, 0.5, ctypes.c_void_p(16), None,
               None) == rp.RP_EINVAL
    bad = rp.rp_batch_request(ctypes.c_void_p(4), 5, 8, 0, None, 1, 0.5)
    bid = ctypes.c_uint64(0)
    assert rp._batch_lib().rp_batch_submit(ctypes.byref(bad), 1, None, None,
                                           ctypes.byref(bid)) == rp.RP_EINVAL


def test_rejected_call_allocates_nothing():
    L = rp.lib()
    assert L.rp_shuffle_inplace(None, 5, 8, None, 0, 0.5, None, None) == rp.RP_EINVAL
    assert rp.rp_last_call_aux_bytes() == 0


def test_workload_splitmix_matches_oracle():
    import torch
    import oracle
    xs = [0, 1, 2, 12345, 2**63, 2**64 - 1, 0x9E3779B97F4A7C15]
    t = torch.tensor([x - 2**64 if x >= 2**63 else x for x in xs], dtype=torch.int64)
    got = workloads.splitmix64_torch(t).tolist()
    assert [g & (2**64 - 1) for g in got] == [oracle.splitmix64(x) for x in xs]


def test_records_generator_host_device_agree():
    rec = workloads.records64(64, "cpu", start=1000).numpy().view(np.uint32)
    assert np.array_equal(rec, workloads.records64_numpy(np.arange(1000, 1064)))
    assert rec[5, 0] == 1005


def test_variant_rejects_unknown():
    L = rp.lib()
    assert L.rp_shuffle_variant(None, 0, 8, None, 0, 0.5, 7, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_variant(None, 0, 8, None, 0, 0.5, -1, None, None) == rp.RP_EINVAL
    assert L.rp_shuffle_variant(None, 0, 8, None, 0, 1.5, 0, None, None) == rp.RP_EINVAL


def test_set_mem_budget_host_only():
    L = rp.lib()
    L.rp_set_mem_budget.restype = ctypes.c_int
    L.rp_set_mem_budget.argtypes = [ctypes.c_uint64]
    assert L.rp_set_mem_budget(0) == rp.RP_EINVAL
    assert L.rp_set_mem_budget(64 << 30) == rp.RP_OK


_sizes = st.one_of(
    st.integers(min_value=2, max_value=(1 << 32) - 1),
    st.builds(lambda e, d: max(2, min((1 << 32) - 1, (1 << e) + d)),
              st.integers(min_value=1, max_value=31), st.integers(min_value=-3, max_value=3)))


@settings(max_examples=400, deadline=None, derandomize=True)
@given(n=_sizes, eps=st.floats(min_value=0.01, max_value=0.99),
       eb=st.sampled_from([4, 8, 12, 16, 20, 64, 128, 252, 256]))
def test_plan_properties_over_the_argument_space(n, eps, eb):
    """Every plan (host only; an MI355X assumed) keeps its auxiliary words
    within floor(n^(1-eps)), has at least one active swap and no more than n,
    and counts at least one in-flight word per active swap."""
    p = rp.rp_plan(n, eb, eps)
    assert p["status"] == 0
    assert p["aux_bound_words"] == rp.rp_aux_bound_words(n, eps)
    assert p["aux_words"] <= p["aux_bound_words"]
    assert 1 <= p["k"] <= n
    assert p["k"] <= p["grid"] * 256 * p["slots_per_lane"]
    assert p["inflight_words"] >= p["k"]
    if p["k"] > 1:
        assert p["table_slots"] >= 1
    # a larger eps never allows more auxiliary words
    if eps + 0.05 < 1.0:
        assert rp.rp_aux_bound_words(n, eps + 0.05) <= p["aux_bound_words"]
