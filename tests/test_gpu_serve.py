"""GPU tests of the serving form (rp_server_*): every request's result is the
Knuth shuffle of its own array with its own seed, whether it ran alone or in
a mix of requests admitted while others were running; admission never lets
the arrays exceed the memory budget."""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2103_01216_amd as rp
from paper_2103_01216_amd import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DTYPE = {4: torch.int32, 8: torch.int64}


def _wait_all(srv, tickets, timeout=90.0):
    """Poll until every ticket is done (bounded)."""
    left = set(tickets)
    deadline = time.monotonic() + timeout
    while left:
        for t in srv.completed():
            left.discard(t)
        if not left:
            break
        assert time.monotonic() < deadline, f"{len(left)} requests unfinished"
        time.sleep(0.002)


def _result(srv, t, n, eb):
    out = torch.empty(n, dtype=DTYPE[eb], device=DEV)
    srv.copy_out(t, out)
    torch.cuda.synchronize()
    return out


def _check_exact(got, n, seed, eb):
    want = np.arange(n, dtype=np.int64 if eb == 8 else np.int32)
    oracle.knuth_shuffle_seed(want, seed)
    assert np.array_equal(got.cpu().numpy(), want), (n, seed)


@pytest.mark.parametrize("mode", [rp.RP_SERVE_BATCHED, rp.RP_SERVE_PLAIN])
def test_mix_equals_alone(mode):
    sizes = workloads.batch_sizes(80, 10, 18, 21)
    seeds = [10**6 + i for i in range(len(sizes))]
    gaps = np.random.default_rng(7).exponential(1.0 / 2000.0, size=len(sizes))
    with rp.Server(1 << 30, mode=mode) as srv:
        tickets = []
        for n, s, g in zip(sizes, seeds, gaps):
            time.sleep(float(g))
            tickets.append(srv.submit(int(n), 8, s))
        _wait_all(srv, tickets)
        for t, n, s in zip(tickets, sizes, seeds):
            info = srv.info(t)
            assert info["state"] == rp.RP_REQ_DONE and info["status"] == 0
            assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_launch_ns"] <= info["t_done_ns"]
            got = _result(srv, t, int(n), 8)
            _check_exact(got, int(n), s, 8)
            if mode == rp.RP_SERVE_BATCHED:
                assert info["aux_words"] <= rp.rp_aux_bound_words(int(n), 0.5)
            assert srv.release(t)
        st = srv.stats()
        assert st["done"] == len(sizes) and st["bytes_in_use"] == 0
    # the same requests alone (one plain call each) give the same bytes
    for i in (0, 7, 33, 79):
        a = torch.arange(int(sizes[i]), dtype=torch.int64, device=DEV)
        rp.rp_shuffle_inplace(a, seed=seeds[i], eps=0.5, stats=False)
        torch.cuda.synchronize()
        _check_exact(a, int(sizes[i]), seeds[i], 8)


def test_admission_respects_budget():
    budget = 8 << 20                      # 8 MiB: a few requests at a time
    sizes = [(1 << 18) + 17 * i for i in range(24)]   # ~2 MiB each (int64)
    with rp.Server(budget) as srv:
        tickets = [srv.submit(n, 8, 500 + i) for i, n in enumerate(sizes)]
        done = []
        deadline = time.monotonic() + 90
        while len(done) < len(tickets):
            for t in srv.completed():
                done.append(t)
                i = tickets.index(t)
                got = _result(srv, t, sizes[i], 8)
                _check_exact(got, sizes[i], 500 + i, 8)
                assert srv.release(t)
            assert time.monotonic() < deadline
            time.sleep(0.001)
        st = srv.stats()
        assert st["peak_bytes"] <= budget
        assert st["admitted"] == len(sizes)
    # some requests had to wait for memory (the budget holds 3 of them)
    assert st["peak_bytes"] >= 2 * sizes[0] * 8


@pytest.mark.parametrize("large_alone", [False, True])
def test_large_requests_and_record_sizes(large_alone):
    reqs = [((1 << 22) + 5, 8, 71), ((1 << 23) + 1, 4, 72), (3000, 8, 73),
            (5000, 16, 74), (70000, 4, 75)]
    with rp.Server(1 << 30, large_log2=22, large_alone=large_alone) as srv:
        tickets = [srv.submit(n, eb, s) for n, eb, s in reqs]
        _wait_all(srv, tickets)
        for t, (n, eb, s) in zip(tickets, reqs):
            info = srv.info(t)
            assert info["status"] == 0
            if eb in DTYPE:
                _check_exact(_result(srv, t, n, eb), n, s, eb)
            else:
                out = torch.empty((n, eb // 4), dtype=torch.int32, device=DEV)
                srv.copy_out(t, out)
                torch.cuda.synchronize()
                want = np.zeros((n, eb // 4), dtype=np.int32)
                want[:, 0] = np.arange(n)
                oracle.knuth_shuffle_seed(want, s)
                assert np.array_equal(out.cpu().numpy(), want)
            assert srv.release(t)


def test_copy_in_requests():
    n, seed = 12345, 99
    src = torch.randint(0, 2**31 - 1, (n,), dtype=torch.int64, device=DEV)
    with rp.Server(1 << 26) as srv:
        t = srv.submit(n, 8, seed, src=src)
        _wait_all(srv, [t])
        got = _result(srv, t, n, 8)
        want = src.cpu().numpy().copy()
        oracle.knuth_shuffle_seed(want, seed)
        assert np.array_equal(got.cpu().numpy(), want)
        assert srv.release(t)


def test_rejections_and_auto_release():
    with rp.Server(1 << 20, auto_release=True) as srv:
        with pytest.raises(rp.RpError):
            srv.submit(1 << 20, 8, 1)           # larger than the whole budget
        with pytest.raises(rp.RpError):
            srv.submit(0, 8, 1)
        with pytest.raises(rp.RpError):
            srv.submit(100, 6, 1)
        tickets = [srv.submit(1000 + i, 8, i) for i in range(10)]
        _wait_all(srv, tickets)
        for t in tickets:
            info = srv.info(t)
            assert info["state"] == rp.RP_REQ_DONE and info["A"] is None
            assert srv.release(t)
        assert srv.stats()["bytes_in_use"] == 0


def test_large_alone_in_a_mix():
    """Large requests that run alone on the whole GPU while small ones keep
    arriving: every result is still the request's own shuffle."""
    rng = np.random.default_rng(17)
    sizes = [int(x) for x in workloads.batch_sizes(60, 10, 24, 33)]
    seeds = [5 * 10**5 + i for i in range(len(sizes))]
    gaps = rng.exponential(1.0 / 300.0, size=len(sizes))
    with rp.Server(4 << 30, large_log2=21, large_alone=True) as srv:
        tickets = []
        for n, sd, g in zip(sizes, seeds, gaps):
            time.sleep(float(g))
            tickets.append(srv.submit(n, 8, sd))
        _wait_all(srv, tickets, timeout=120)
        for t, n, sd in zip(tickets, sizes, seeds):
            info = srv.info(t)
            assert info["status"] == 0
            _check_exact(_result(srv, t, n, 8), n, sd, 8)
            assert srv.release(t)


def test_default_budget():
    rp.rp_set_mem_budget(64 << 20)
    try:
        with rp.Server(0) as srv:
            with pytest.raises(rp.RpError):
                srv.submit((64 << 20) // 8 + 1, 8, 1)     # larger than the default arena
            t = srv.submit(1000, 8, 2)
            _wait_all(srv, [t])
            _check_exact(_result(srv, t, 1000, 8), 1000, 2, 8)
            assert srv.release(t)
    finally:
        rp.rp_set_mem_budget(64 << 30)
