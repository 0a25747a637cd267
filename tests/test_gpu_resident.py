"""GPU tests of the serving form's resident mode (RP_SERVE_RESIDENT): one
kernel stays on the device and takes each request as it arrives, small ones
on one workgroup, large ones on a gang of workgroups.  Every request's result
must be the Knuth shuffle of its own array with its own seed (the oracle),
the same bytes as the request run alone, whatever ran beside it; the kernel
must leave when the server is idle and come back for new work."""
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
RES = rp.RP_SERVE_RESIDENT


def _wait_all(srv, tickets, timeout=90.0):
    left = set(tickets)
    deadline = time.monotonic() + timeout
    while left:
        for t in srv.completed():
            left.discard(t)
        if not left:
            break
        assert time.monotonic() < deadline, f"{len(left)} requests unfinished"
        time.sleep(0.002)


def _check(srv, t, n, eb, seed, src=None):
    """The request's array against the oracle's shuffle of its input."""
    if eb in DTYPE:
        out = torch.empty(n, dtype=DTYPE[eb], device=DEV)
        want = (np.arange(n, dtype=np.int64 if eb == 8 else np.int32) if src is None
                else src.cpu().numpy().copy())
    else:
        out = torch.empty((n, eb // 4), dtype=torch.int32, device=DEV)
        want = np.zeros((n, eb // 4), dtype=np.int32)
        want[:, 0] = np.arange(n)
    srv.copy_out(t, out)
    torch.cuda.synchronize()
    oracle.knuth_shuffle_seed(want, seed)
    assert np.array_equal(out.cpu().numpy(), want), (n, eb, seed)


def test_resident_mix_equals_oracle_and_alone():
    """A Poisson mix of small requests (one workgroup each) and a few large
    ones (gangs), admitted while others run."""
    sizes = [int(x) for x in workloads.batch_sizes(90, 10, 18, 21)]
    sizes[10] = (1 << 22) + 3
    sizes[40] = (1 << 23) + 11
    seeds = [10**6 + i for i in range(len(sizes))]
    gaps = np.random.default_rng(7).exponential(1.0 / 2000.0, size=len(sizes))
    with rp.Server(1 << 30, mode=RES) as srv:
        tickets = []
        for n, s, g in zip(sizes, seeds, gaps):
            time.sleep(float(g))
            tickets.append(srv.submit(n, 8, s))
        _wait_all(srv, tickets)
        for t, n, s in zip(tickets, sizes, seeds):
            info = srv.info(t)
            assert info["state"] == rp.RP_REQ_DONE and info["status"] == 0, info
            assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_launch_ns"] <= info["t_done_ns"]
            assert 0 < info["aux_words"] <= rp.rp_aux_bound_words(n, 0.5)
            assert info["rounds"] > 0
            _check(srv, t, n, 8, s)
            assert srv.release(t)
        st = srv.stats()
        assert st["done"] == len(sizes) and st["bytes_in_use"] == 0
        assert st["launches"] >= 1
    # the same requests alone (one plain call each): the same bytes
    for i in (0, 10, 40, 89):
        a = torch.arange(sizes[i], dtype=torch.int64, device=DEV)
        rp.rp_shuffle_inplace(a, seed=seeds[i], eps=0.5, stats=False)
        torch.cuda.synchronize()
        want = np.arange(sizes[i], dtype=np.int64)
        oracle.knuth_shuffle_seed(want, seeds[i])
        assert np.array_equal(a.cpu().numpy(), want)


@pytest.mark.parametrize("eb", [4, 8, 12, 16, 64])
def test_resident_gangs_by_record_size(eb):
    """Large requests on gangs (every record size the one-barrier rounds
    hold in registers, and the generic one), beside a small one."""
    reqs = [((1 << 20) + 7, 31), ((1 << 21) + 1, 32), (5000, 33)]
    with rp.Server(1 << 30, mode=RES, large_log2=20) as srv:
        tickets = [srv.submit(n, eb, s) for n, s in reqs]
        _wait_all(srv, tickets)
        for t, (n, s) in zip(tickets, reqs):
            info = srv.info(t)
            assert info["status"] == 0, info
            assert info["aux_words"] <= rp.rp_aux_bound_words(n, 0.5)
            _check(srv, t, n, eb, s)
            assert srv.release(t)


@pytest.mark.parametrize("eps", [0.5, 0.3])
def test_resident_concurrent_gangs(eps):
    """Several large requests at once: gangs form one after another (later
    ones smaller, then single workgroups), all exact."""
    sizes = [(1 << 22) + 101 * i for i in range(6)]
    seeds = [700 + i for i in range(6)]
    with rp.Server(1 << 30, mode=RES) as srv:
        tickets = [srv.submit(n, 8, s, eps=eps) for n, s in zip(sizes, seeds)]
        _wait_all(srv, tickets)
        for t, n, s in zip(tickets, sizes, seeds):
            info = srv.info(t)
            assert info["status"] == 0, info
            assert info["aux_words"] <= rp.rp_aux_bound_words(n, eps)
            _check(srv, t, n, 8, s)
            assert srv.release(t)


def test_resident_gang_not_formed_runs_on_one_workgroup(monkeypatch):
    """With no time for a gang to form, its leader gives the request back and
    the server posts it again for one workgroup: the result is the same."""
    monkeypatch.setenv("RP_RES_FORM_US", "0")
    sizes = [(1 << 22) + 9, (1 << 22) + 19, 3000]
    seeds = [901, 902, 903]
    with rp.Server(1 << 30, mode=RES) as srv:
        tickets = [srv.submit(n, 8, s) for n, s in zip(sizes, seeds)]
        _wait_all(srv, tickets)
        for t, n, s in zip(tickets, sizes, seeds):
            info = srv.info(t)
            assert info["status"] == 0, info
            _check(srv, t, n, 8, s)
            assert srv.release(t)


def test_resident_idle_stop_and_relaunch():
    """The kernel leaves once the server is idle and is launched again for
    the next request."""
    with rp.Server(1 << 28, mode=RES) as srv:
        t1 = [srv.submit(20_000 + i, 8, 40 + i) for i in range(8)]
        _wait_all(srv, t1)
        l1 = srv.stats()["launches"]
        assert l1 >= 1
        time.sleep(0.3)            # well beyond the idle stop
        t2 = [srv.submit(30_000 + i, 4, 60 + i) for i in range(8)]
        _wait_all(srv, t2)
        assert srv.stats()["launches"] == l1 + 1
        for i, t in enumerate(t1):
            _check(srv, t, 20_000 + i, 8, 40 + i)
        for i, t in enumerate(t2):
            _check(srv, t, 30_000 + i, 4, 60 + i)


def test_resident_copy_in():
    """Inputs copied by the kernel from device memory and from pinned host
    memory; pageable host memory is refused."""
    n1, n2 = 12345, (1 << 22) + 77
    src1 = torch.randint(0, 2**31 - 1, (n1,), dtype=torch.int64, device=DEV)
    src2 = torch.randint(0, 2**31 - 1, (n2,), dtype=torch.int64).pin_memory()
    with rp.Server(1 << 28, mode=RES) as srv:
        t1 = srv.submit(n1, 8, 5, src=src1)
        t2 = srv.submit(n2, 8, 6, src=src2)
        _wait_all(srv, [t1, t2])
        _check(srv, t1, n1, 8, 5, src=src1)
        _check(srv, t2, n2, 8, 6, src=src2)
        with pytest.raises(rp.RpError):
            srv.submit(100, 8, 7, src=torch.zeros(100, dtype=torch.int64))


def test_resident_rejections_and_auto_release():
    with rp.Server(1 << 20, mode=RES, auto_release=True) as srv:
        with pytest.raises(rp.RpError):
            srv.submit(1 << 20, 8, 1)       # larger than the whole budget
        with pytest.raises(rp.RpError):
            srv.submit(100, 6, 1)
        tickets = [srv.submit(1000 + i, 8, i) for i in range(10)]
        _wait_all(srv, tickets)
        for t in tickets:
            info = srv.info(t)
            assert info["state"] == rp.RP_REQ_DONE and info["A"] is None
            assert srv.release(t)
        assert srv.stats()["bytes_in_use"] == 0
