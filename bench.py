#!/usr/bin/env python3
"""Benchmark: in-place random permutation of n = 2^30 int64 on one MI355X.

One step = one complete call of rp_shuffle_inplace on the 8 GiB array (every
round of the RP-Final path: refill, reserve, commit, clean), eps = 0.5, so
auxiliary space is at most floor(n^0.5) = 32768 words.  A is resident in HBM
before the timed region; the shuffle's work does not depend on A's contents,
so consecutive steps shuffle the same array again (seed = 1 + step).

Prints one JSON line (see the "metric"/"roofline"/"cpu_baseline" fields).
The first warm-up step runs on the identity array; its whole output is
compared with the CPU oracle's (run on a host thread beside the GPU steps; its
time is the CPU baseline).

`--workload serve` replays Poisson arrival traces (exponential gaps, seed 7)
at each rate for --duration seconds, n = floor(2^U) with U ~ Uniform[10, 26)
from a SplitMix64 stream (seed 7), int64 A[i] = i, request seed 10^6 + id,
eps = 0.5, through a server with a 64 GiB arena: resident (one kernel takes
each request as it arrives; requests of n >= 2^20 on gangs of
workgroups), batched (launches of every admitted request; large ones in group
launches), and one plain launch per request; it reports elements/s and
p50/p99 latency.

`--workload ablation` times the reservation variants (final, one reservation
without the dense window, Algorithm 1's two reservations with H of the active
swaps in registers, in a prefix-sized array (flat) or in a hashed table
(naive), the non-in-place linear array) on the n = 2^30 int64 workload, each
checked byte-equal to the final variant's result, and sweeps the auxiliary
bound at n = 10^8 int64 (the paper's aux-space table: 0.4 %, 1 %, 2 %, 4 % of
n, plus smaller bounds).  With --variants-once it only runs each variant once
(seed 1, after one rp_shuffle_inplace call as the reference), the launches a
counter profile attributes in that order.

`--workload list` ranks one random list of n = 10^8 elements (two 64-bit
pointer words each, the paper's list-contraction inputs) by in-place list
contraction, at several auxiliary bounds, checked against the CPU oracle.

`--workload scale` times the plain method at the other stated sizes: n = 2^20
int64 at eps 0.5, n = 2^28 int32 and int64 at eps 0.25 / 0.5 / 0.75, n = 2^26 records of 64 bytes at
eps 0.5, and n = 2^30 int64 at eps 0.2 / 0.25 / 1/3 / 0.5; each checked as a
permutation with sampled positions against the CPU oracle.

`--workload batch` measures the batched form instead: 4096 independent
shuffles, n = floor(2^U) with U ~ Uniform[8, 20) drawn from a SplitMix64
stream (seed 12345), int32 A[i] = i, instance seed 1000 + id, eps = 0.5, as
one persistent launch per step under the autotuned schedule, beside one plain
launch per instance over the same arrays.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
COPY_BYTES = 2 << 30            # reference copy of the plain workload
KERNEL_NAME = "rp_rounds1_kernel"
WORKLOAD = {"n": 1 << 30, "elem_bytes": 8, "eps": 0.5, "seed": 1}
BATCH = {"count": 4096, "lo_log2": 8, "hi_log2": 20, "size_seed": 12345,
         "seed_base": 1000, "eps": 0.5}
CSRC = os.path.join(ROOT, "paper_2103_01216_amd", "csrc")
TRAFFIC = {
    "plain": (os.path.join(ROOT, "profiles", "rp_rounds1_kernel_n2p30_int64_eps0.5_traffic.json"),
              [os.path.join(CSRC, f) for f in ("rp.hip", "rp_device.h")]),
    "batch": (os.path.join(ROOT, "profiles", "rp_batch_kernel_4096_loguniform_int32_traffic.json"),
              [os.path.join(CSRC, f) for f in ("rp_batch.hip", "rp_device.h")]),
}


def _src_hash(workload: str = "plain") -> str:
    """sha256[:16] over the sources the workload's kernel is compiled from."""
    h = hashlib.sha256()
    for path in TRAFFIC[workload][1]:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic_bytes(workload: str = "plain"):
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC[workload][0]) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != _src_hash(workload):
        return None
    return rec.get("hbm_bytes_per_launch")


def host_info():
    """CPU model and the cores this process may use, for the baseline record."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


class OracleRun:
    """The sequential Knuth shuffle of the headline input (n = 2^30 int64,
    A[i] = i, seed mode) on one host core, in a thread of its own (the C
    oracle runs outside the interpreter lock), so that the GPU steps proceed
    meanwhile.  Its result is the full-array parity reference and its time is
    the CPU baseline."""

    def __init__(self, n, seed, log):
        import threading
        import numpy as np
        self.n, self.seed, self.log = n, seed, log
        self.want = np.arange(n, dtype=np.int64)
        self.seconds = None
        self._th = threading.Thread(target=self._run, daemon=True)
        self._th.start()

    def _run(self):
        import oracle
        t0 = time.perf_counter()
        oracle.knuth_shuffle_seed(self.want, self.seed)
        self.seconds = time.perf_counter() - t0
        self.log(f"cpu oracle: n={self.n} int64 in {self.seconds:.2f} s (one core)")

    def join(self):
        self._th.join()
        return self.want


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload",
                    choices=("plain", "batch", "serve", "ablation", "list", "scale", "floor"),
                    default="plain")
    ap.add_argument("--duration", type=float, default=60.0,
                    help="serve workload: seconds of arrivals per rate")
    ap.add_argument("--rates", default="50,200,1000",
                    help="serve workload: arrival rates (requests/s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants-once", action="store_true",
                    help="ablation workload: one launch per variant, no timing or sweep")
    ap.add_argument("--serve-modes", default="resident,batched,plain",
                    help="serving modes to replay (resident, batched, plain)")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="plain workload: arrival rate of the short served leg")
    ap.add_argument("--serve-duration", type=float, default=8.0,
                    help="plain workload: seconds of arrivals of the served leg (0: none)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch workload: skip the one-launch-per-instance comparison")
    ap.add_argument("--schedule", default=None,
                    help="batch workload: CUTOFF,RATIO16,WPC[,LANES[,LATE]] instead of autotuning")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not "
              "supported: the single-GPU kernel is the whole path, and a "
              "sharded form is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args, log)
    elif args.workload == "serve":
        run_serve(args, log)
    elif args.workload == "ablation":
        run_ablation(args, log)
    elif args.workload == "list":
        run_list(args, log)
    elif args.workload == "scale":
        run_scale(args, log)
    elif args.workload == "floor":
        run_floor(args, log)
    else:
        run_plain(args, log)


def random_access_floor(rp, A, eb, stream, log, reps=3):
    """Median time of the shuffle's data movement alone (rp_probe_random_rmw:
    every swap's two reads and two writes, no reservation) on A, which it
    leaves scrambled."""
    import torch
    ts = []
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rp.rp_probe_random_rmw(A, seed=1 + r, stream=stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ms = sorted(ts)[len(ts) // 2]
    n = A.shape[0]
    log(f"random-access floor: n={n} x {eb} B in {ms:.2f} ms "
        f"({4 * eb * n / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic)")
    return ms


def reference_copy(rp, stream, log, nbytes=COPY_BYTES):
    """Median time of a streaming copy of `nbytes` (rp_probe_copy): the
    achievable HBM rate, and the known byte count that scales the rocprofv3
    FETCH_SIZE / WRITE_SIZE counters of the same run."""
    import torch
    src = torch.zeros(nbytes // 8, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    ts = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rp.rp_probe_copy(dst, src, stream=stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ms = sorted(ts)[1]
    log(f"reference copy: {nbytes / 2**30:.0f} GiB in {ms:.2f} ms "
        f"({2 * nbytes / (ms * 1e-3) / 1e9:.0f} GB/s read+write)")
    del src, dst
    torch.cuda.empty_cache()
    return ms


SERVE_MODES = (("resident", "RP_SERVE_RESIDENT"), ("batched", "RP_SERVE_BATCHED"),
               ("plain", "RP_SERVE_PLAIN"))


def _serve_modes(names):
    want = [m.strip() for m in names.split(",") if m.strip()]
    bad = [m for m in want if m not in dict(SERVE_MODES)]
    if bad or not want:
        raise SystemExit(f"unknown serving mode(s) {bad}; choose from {[m for m, _ in SERVE_MODES]}")
    return [(m, c) for m, c in SERVE_MODES if m in want]


def serve_leg(rp, rate, duration, log, args_modes="resident,batched,plain"):
    """A short served run at one Poisson rate through the resident server,
    the batched server and one plain launch per request, on the same trace
    (the serving workload's request mix)."""
    import numpy as np
    from paper_2103_01216_amd import workloads
    count = max(1, int(rate * duration))
    gaps = np.random.default_rng(SERVE["arrival_seed"]).exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    sizes = workloads.batch_sizes(count, SERVE["lo_log2"], SERVE["hi_log2"], SERVE["size_seed"])
    seeds = [SERVE["seed_base"] + i for i in range(count)]
    rec = {"rate_per_s": rate, "duration_s": duration, "requests": count,
           "offered_elements_per_s": float(sizes.sum()) / float(arrivals[-1]),
           "request_sizes": "n=floor(2^U), U~Uniform[10,26), int64, eps=0.5"}
    for name, const in _serve_modes(args_modes):
        mode = getattr(rp, const)
        lats, elems, span, unfinished, st, detail = _replay(rp, mode, arrivals, sizes, seeds,
                                                            log, drain_s=duration)
        lat_ms = np.array(lats) * 1e3
        rec[name] = {"elements_per_s": elems / span,
                     "p50_ms": float(np.percentile(lat_ms, 50)),
                     "p99_ms": float(np.percentile(lat_ms, 99)),
                     "completed": count - unfinished, "unfinished": unfinished}
        if detail:
            rec[name].update(detail)
        log(f"served {rate:g}/s {name}: {elems / span:.3g} elements/s, "
            f"p50 {rec[name]['p50_ms']:.2f} ms, p99 {rec[name]['p99_ms']:.2f} ms, "
            f"unfinished {unfinished}")
    return rec


def run_plain(args, log):
    warmup = max(1, args.warmup)
    import numpy as np
    import torch
    import paper_2103_01216_amd as rp

    n, eb, eps = WORKLOAD["n"], WORKLOAD["elem_bytes"], WORKLOAD["eps"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    A = torch.empty(n, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"allocated A: n=2^30 int64 ({A.numel() * 8 / 2**30:.0f} GiB)")
    floor_ms = random_access_floor(rp, A, eb, stream, log)
    copy_ms = reference_copy(rp, stream, log)
    A.copy_(torch.arange(n, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()

    stats = None
    parity = {"checked": False}
    oracle_run = None
    got_host = None
    for w in range(warmup):
        stats = rp.rp_shuffle_inplace(A, seed=WORKLOAD["seed"] + w, eps=eps,
                                      stream=stream).get()
        log(f"warmup {w}: rounds={stats['rounds']} k={stats['k']} "
            f"aux={stats['aux_words']}/{stats['aux_bound_words']} words "
            f"inflight={stats['inflight_words']} words")
        if w == 0 and not (args.no_check and args.no_cpu_baseline):
            # The whole output of the first step comes back to the host and is
            # compared with the oracle's whole output once the oracle is done.
            oracle_run = OracleRun(n, WORKLOAD["seed"], log)
            got_host = A.cpu().numpy()

    # Timed region: K steps, HIP events on the stream the kernels run on.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        rp.rp_shuffle_inplace(A, seed=WORKLOAD["seed"] + warmup + i, eps=eps,
                              stream=stream, stats=False)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms = sum(step_ms) / len(step_ms)
    value = n * args.steps / wall
    log(f"steps ms: {', '.join(f'{x:.2f}' for x in step_ms)}; wall {wall:.3f} s")
    del A
    torch.cuda.empty_cache()

    cpu = None
    if oracle_run is not None:
        want = oracle_run.join()
        if not args.no_check:
            exact = bool(np.array_equal(got_host, want))
            mism = 0 if exact else int(np.count_nonzero(got_host != want))
            log(f"parity: whole array of the first step vs the oracle: "
                f"{'equal' if exact else f'{mism} positions differ'}")
            parity = {"checked": True, "whole_array_equal": exact, "positions": n,
                      "mismatches": mism}
            if not exact:
                log("PARITY FAILURE")
                sys.exit(1)
        cpu = {"value": n / oracle_run.seconds, "unit": "elements/s", "cores": 1,
               "kind": "oracle",
               "sample": "the whole headline input: sequential Knuth shuffle (seed mode, "
                         "targets drawn inline) of n=2^30 int64 A[i]=i, seed 1, on one "
                         "host core, run beside the GPU steps",
               "seconds": oracle_run.seconds, **host_info()}
        del want, got_host

    served = None
    if args.serve_duration > 0:
        served = serve_leg(rp, args.serve_rate, args.serve_duration, log, args.serve_modes)

    alg_bytes = 4 * eb * n                      # A[s], A[H[s]]: read + write
    achieved = alg_bytes / (ms * 1e-3) / 1e9    # GB/s over the kernel's time
    floor_gbps = alg_bytes / (floor_ms * 1e-3) / 1e9
    traffic = _traffic_bytes()
    out = {
        "metric": "in-place shuffle elements/s at n=2^30 int64 (% HBM peak)",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "plain in-place shuffle, n=2^30 int64, A[i]=i "
                               "initially, H[i]=splitmix64(seed^i) mod (i+1), eps=0.5",
                   "n": n, "elem_bytes": eb, "eps": eps,
                   "k": stats["k"], "rounds": stats["rounds"],
                   "attempts": stats["attempts"], "retries": stats["retries"],
                   "aux_words": stats["aux_words"],
                   "aux_bound_words": stats["aux_bound_words"],
                   "inflight_words": stats["inflight_words"],
                   "k_over_bound": stats["k"] / stats["aux_bound_words"],
                   "throttled_rounds": stats["throttled_rounds"],
                   "grid": stats["grid"], "slots_per_lane": stats["slots_per_lane"],
                   "round_us": ms * 1e3 / max(1, stats["rounds"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "traffic_gbps": (traffic / (ms * 1e-3) / 1e9) if traffic else None,
                     "traffic_frac": (traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS)
                     if traffic else None,
                     "kernel": KERNEL_NAME, "kernel_ms_events": ms,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "reference_copy_bytes": COPY_BYTES,
                     "reference_copy_gbps": 2 * COPY_BYTES / (copy_ms * 1e-3) / 1e9,
                     "random_access_floor_ms": floor_ms,
                     "random_access_floor_gbps": floor_gbps,
                     "frac_of_random_access_floor": floor_ms / ms},
        "parity": parity,
    }
    if served is not None:
        out["served"] = served
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def run_floor(args, log):
    """Ceilings the shuffle's time is compared with: the random-access floor
    of its data movement at the two headline shapes, a streaming copy, the
    flag barrier of a round, and device-scope atomics into a table of the
    headline's size."""
    import torch
    import paper_2103_01216_amd as rp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for name, n, eb in (("n2p30_int64", 1 << 30, 8), ("n2p26_rec64", 1 << 26, 64)):
        A = torch.zeros((n, eb // 8), dtype=torch.int64, device=dev)
        ms = random_access_floor(rp, A, eb, stream, log, reps=5)
        res[name] = {"ms": ms, "swaps_per_s": n / (ms * 1e-3),
                     "algorithmic_gbps": 4 * eb * n / (ms * 1e-3) / 1e9}
        del A
        torch.cuda.empty_cache()
    nbytes = 4 << 30
    src = torch.zeros(nbytes // 8, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    ts = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rp.rp_probe_copy(dst, src, stream=stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ms = sorted(ts)[2]
    res["copy_4GiB"] = {"ms": ms, "gbps": 2 * nbytes / (ms * 1e-3) / 1e9}
    log(f"copy 4 GiB: {ms:.2f} ms, {2 * nbytes / (ms * 1e-3) / 1e9:.0f} GB/s read+write")
    del src, dst
    torch.cuda.empty_cache()
    bar = {}
    for g in (2, 64, 228, 456, 1024):
        us = rp.rp_probe_barrier(g, 20000, stream=stream)
        bar[str(g)] = us
        log(f"flag barrier on {g} workgroups: {us:.2f} us")
    res["barrier_us_by_grid"] = bar
    T, grid = 57440, 228
    ns_tp = rp.rp_probe_atomics(T, grid, 256, False, stream=stream)
    ns_lat = rp.rp_probe_atomics(T, grid, 256, True, stream=stream)
    ops = grid * 256 * 256
    res["atomics"] = {"table_slots": T, "lanes": grid * 256, "per_lane": 256,
                      "throughput_per_s": ops / (ns_tp * 1e-9),
                      "chained_ns_per_op": ns_lat / 256}
    log(f"atomic max into {T} slots: {ops / (ns_tp * 1e-9):.3g}/s in flight, "
        f"{ns_lat / 256:.0f} ns each when chained")
    out = {"metric": "device ceilings for the shuffle (random-access floor, copy, barrier, atomics)",
           "value": res["n2p30_int64"]["algorithmic_gbps"], "unit": "GB/s", "n_gpus": 1,
           "steps": 5, "warmup": 0, "ms_per_step": res["n2p30_int64"]["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": "probes: swap data movement of n=2^30 int64 and n=2^26 x 64 B "
                                  "(seed-mode targets, no reservation), 4 GiB copy, flag "
                                  "barriers, atomic max into 57440 slots",
                      "results": res}}
    print(json.dumps(out), flush=True)


def run_batch(args, log):
    """The batched form on the 4096-instance workload (see module docstring)."""
    warmup = max(1, args.warmup)
    import numpy as np
    import torch
    import paper_2103_01216_amd as rp
    from paper_2103_01216_amd import workloads

    count, eps = BATCH["count"], BATCH["eps"]
    sizes = workloads.batch_sizes(count, BATCH["lo_log2"], BATCH["hi_log2"], BATCH["size_seed"])
    seeds = [BATCH["seed_base"] + i for i in range(count)]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(offs[-1])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    # One allocation; request i is the view [offs[i], offs[i+1]).
    seg_start = torch.repeat_interleave(torch.from_numpy(offs[:-1]).to(dev),
                                        torch.from_numpy(sizes).to(dev))
    ident = (torch.arange(total, dtype=torch.int64, device=dev) - seg_start).to(torch.int32)
    big = ident.clone()
    arrays = [big[int(offs[i]):int(offs[i + 1])] for i in range(count)]
    torch.cuda.synchronize()
    log(f"batch: {count} instances, {total} int32 elements "
        f"(n from {sizes.min()} to {sizes.max()})")
    # the known byte count that scales this run's rocprofv3 traffic counters
    copy_ms = reference_copy(rp, stream, log)

    if args.schedule:
        v = [int(x) for x in args.schedule.split(",")]
        sched = {"wave_cutoff": v[0], "table_ratio_x16": v[1], "workgroups_per_cu": v[2],
                 "workgroup_lanes": v[3] if len(v) > 3 else 256,
                 "late_loads": v[4] if len(v) > 4 else 0, "tuned_ms_x1000": 0}
        log(f"schedule given: {sched}")
    else:
        t0 = time.perf_counter()
        sched = rp.rp_batch_autotune(arrays, seeds=seeds, eps=eps, stream=stream)
        log(f"autotune: {sched} in {time.perf_counter() - t0:.1f} s")
    reqs = rp.rp_batch_requests(arrays, seeds=seeds, eps=eps)

    parity = {"checked": False}
    results = None
    for w in range(warmup):
        if w == 0:
            big.copy_(ident)
        b = rp.rp_batch_submit(arrays, requests=reqs, stream=stream, schedule=sched)
        results = b.results()
        b.release()
        if w == 0 and not args.no_check:
            import oracle
            seen = torch.zeros(total, dtype=torch.bool, device=dev)
            seen[seg_start + big.long()] = True
            perm_ok = bool(seen.all())
            del seen
            pick = sorted(set(list(range(0, count, 97)) + [int(np.argmax(sizes))]))
            exact = True
            for i in pick:
                want = np.arange(int(sizes[i]), dtype=np.int32)
                oracle.knuth_shuffle_seed(want, seeds[i])
                exact = exact and bool(np.array_equal(arrays[i].cpu().numpy(), want))
            status_ok = all(r["status"] == 0 for r in results)
            aux_ok = all(r["aux_words"] <= rp.rp_aux_bound_words(int(n), eps)
                         for r, n in zip(results, sizes))
            log(f"parity: permutation={perm_ok} exact={exact} ({len(pick)} instances) "
                f"status_ok={status_ok} aux_within_bound={aux_ok}")
            parity = {"checked": True, "all_permutations": perm_ok,
                      "instances_exact_vs_oracle": len(pick), "exact": exact,
                      "aux_within_bound": aux_ok}
            if not (perm_ok and exact and status_ok and aux_ok):
                log("PARITY FAILURE")
                sys.exit(1)
            first = big.clone()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        b = rp.rp_batch_submit(arrays, requests=reqs, stream=stream, schedule=sched)
        ev[i][1].record(stream)
        b.results()
        b.release()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    step_ms = [a.elapsed_time(c) for a, c in ev]
    ms = sum(step_ms) / len(step_ms)
    value = total * args.steps / wall
    log(f"batch steps ms: {', '.join(f'{x:.2f}' for x in step_ms)}; wall {wall:.3f} s")

    plain = None
    if not args.no_plain:
        # Same arrays, one rp_shuffle_inplace launch per instance, identity input.
        big.copy_(ident)
        for i in range(8):
            rp.rp_shuffle_inplace(arrays[i], seed=seeds[i], eps=eps, stream=stream, stats=False)
        big.copy_(ident)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(count):
            rp.rp_shuffle_inplace(arrays[i], seed=seeds[i], eps=eps, stream=stream, stats=False)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        same = bool(torch.equal(big, first)) if parity["checked"] else None
        log(f"plain per-instance launches: {pw:.3f} s; equal to the batched result: {same}")
        plain = {"value": total / pw, "unit": "elements/s", "wall_s": pw,
                 "launches": count, "equal_to_batched_result": same}

    alg_bytes = 4 * 4 * total                    # A[s], A[H[s]]: read + write, int32
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    out = {
        "metric": "batched in-place shuffle elements/s (4096 instances, one launch) "
                  "vs one plain launch per instance",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batched: 4096 shuffles, n=floor(2^U), U~Uniform[8,20) "
                               "from SplitMix64 stream seed 12345, int32 A[i]=i, "
                               "seed 1000+id, eps=0.5",
                   "instances": count, "total_elements": total,
                   "schedule": sched,
                   "rounds_total": sum(r["rounds"] for r in results),
                   "plain_per_instance": plain,
                   "speedup_vs_plain": (value / plain["value"]) if plain else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": _traffic_bytes("batch"),
                     "kernel": "rp_batch_kernel", "kernel_ms_events": ms,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "reference_copy_bytes": COPY_BYTES,
                     "reference_copy_gbps": 2 * COPY_BYTES / (copy_ms * 1e-3) / 1e9},
        "parity": parity,
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = list(range(0, count, 4))
        hosts = [np.arange(int(sizes[i]), dtype=np.int32) for i in sample]
        t0 = time.perf_counter()
        for a, i in zip(hosts, sample):
            oracle.knuth_shuffle_seed(a, seeds[i])
        dt = time.perf_counter() - t0
        n_s = int(sum(int(sizes[i]) for i in sample))
        log(f"cpu oracle: {len(sample)} instances, {n_s} elements in {dt:.2f} s")
        out["cpu_baseline"] = {"value": n_s / dt, "unit": "elements/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"every 4th instance of the batch ({len(sample)} "
                                         f"shuffles, {n_s} int32 elements), sequential "
                                         "Knuth shuffle on one host core"}
    print(json.dumps(out), flush=True)


SERVE = {"lo_log2": 10, "hi_log2": 26, "size_seed": 7, "arrival_seed": 7,
         "seed_base": 10**6, "eps": 0.5, "budget": 64 << 30, "elem_bytes": 8}
# Large/small split of the latency detail: the batched server's large-request
# threshold (its default large_log2, 22).  The resident server already puts
# requests from 2^20 on gangs; the split is kept at 2^22 for both modes.
SERVE_LARGE = 1 << 22


def _replay(rp, mode, arrivals, sizes, seeds, log, drain_s):
    """Submit each request at its arrival time; collect completion times.
    Returns (latencies_s, completed_elements, span_s, unfinished, server
    stats, large-request detail)."""
    import threading
    import numpy as np
    srv = rp.Server(SERVE["budget"], mode=mode, auto_release=True,
                    large_alone=(mode == rp.RP_SERVE_BATCHED))
    tickets = {}
    lat = {}
    stop = threading.Event()

    def collect():
        while not stop.is_set() or len(lat) < len(tickets):
            for t in srv.completed():
                info = srv.info(t)
                lat[t] = (info["t_done_ns"] - info["t_submit_ns"]) * 1e-9, info
                srv.release(t)
            if stop.is_set() and len(lat) >= len(tickets):
                break
            time.sleep(0.0005)
            if stop.is_set() and time.perf_counter() > deadline[0]:
                break

    deadline = [float("inf")]
    th = threading.Thread(target=collect, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for i, (ta, n) in enumerate(zip(arrivals, sizes)):
        wait = t0 + ta - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets[srv.submit(int(n), SERVE["elem_bytes"], seeds[i], SERVE["eps"])] = i
    t_submitted = time.perf_counter()
    deadline[0] = t_submitted + drain_s
    stop.set()
    th.join()
    t_end = time.perf_counter()
    done = dict(lat)
    unfinished = len(tickets) - len(done)
    st = srv.stats()
    if unfinished:
        log(f"  {unfinished} requests unfinished {drain_s:.0f} s after the last arrival; "
            "their latency is counted as at least the time they waited")
    now_ns = time.monotonic_ns()
    lats = []
    t_first = min(i["t_submit_ns"] for _, i in done.values()) if done else 0
    t_last = max(i["t_done_ns"] for _, i in done.values()) if done else 0
    for t in tickets:
        if t in done:
            lats.append(done[t][0])
        else:
            lats.append((now_ns - srv.info(t)["t_submit_ns"]) * 1e-9)
    elems = sum(int(sizes[tickets[t]]) for t in done)
    # requests of at least SERVE_LARGE elements: their latency percentiles,
    # and in resident mode how many ran on one workgroup instead of a gang
    big = [(done[t][0], done[t][1]["workgroups"]) for t in done
           if int(sizes[tickets[t]]) >= SERVE_LARGE]
    detail = None
    if big:
        bl = np.array([b[0] for b in big]) * 1e3
        detail = {"large_requests": len(big), "large_p50_ms": float(np.percentile(bl, 50)),
                  "large_p99_ms": float(np.percentile(bl, 99)),
                  "large_on_one_workgroup": sum(1 for b in big if b[1] == 1)}
        small = [done[t][0] for t in done if int(sizes[tickets[t]]) < SERVE_LARGE]
        if small:
            sl = np.array(small) * 1e3
            detail["small_p50_ms"] = float(np.percentile(sl, 50))
            detail["small_p99_ms"] = float(np.percentile(sl, 99))
    srv.close()
    span = max((t_last - t_first) * 1e-9, 1e-9)
    return lats, elems, span, unfinished, st, detail


def run_serve(args, log):
    """The serving form on Poisson arrival traces (see module docstring)."""
    import numpy as np
    import torch
    import paper_2103_01216_amd as rp
    from paper_2103_01216_amd import workloads

    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda:0")
    rates = [float(r) for r in args.rates.split(",")]
    per_rate = {}
    for lam in rates:
        count = int(lam * args.duration)
        gaps = np.random.default_rng(SERVE["arrival_seed"]).exponential(1.0 / lam, size=count)
        arrivals = np.cumsum(gaps)
        sizes = workloads.batch_sizes(count, SERVE["lo_log2"], SERVE["hi_log2"],
                                      SERVE["size_seed"])
        seeds = [SERVE["seed_base"] + i for i in range(count)]
        offered = float(sizes.sum()) / float(arrivals[-1])
        rec = {"requests": count, "offered_elements_per_s": offered}
        for name, const in _serve_modes(args.serve_modes):
            mode = getattr(rp, const)
            log(f"rate {lam:g}/s, {name}: {count} requests, offered {offered:.3g} elements/s")
            lats, elems, span, unfinished, st, detail = _replay(
                rp, mode, arrivals, sizes, seeds, log, drain_s=max(30.0, args.duration / 2))
            lat_ms = np.array(lats) * 1e3
            rec[name] = {"elements_per_s": elems / span,
                         "p50_ms": float(np.percentile(lat_ms, 50)),
                         "p99_ms": float(np.percentile(lat_ms, 99)),
                         "completed": count - unfinished, "unfinished": unfinished,
                         "launches": st["launches"], "peak_bytes": st["peak_bytes"]}
            if detail:
                rec[name].update(detail)
            log(f"  {name}: {elems / span:.3g} elements/s, p50 {rec[name]['p50_ms']:.2f} ms, "
                f"p99 {rec[name]['p99_ms']:.2f} ms, launches {st['launches']}; {detail}")
        per_rate[f"{lam:g}"] = rec
    top = per_rate[f"{rates[-1]:g}"]
    first_mode = _serve_modes(args.serve_modes)[0][0]
    out = {
        "metric": "served shuffle elements/s with p50/p99 latency (Poisson arrivals)",
        "value": top[first_mode]["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": len(rates),
        "warmup": 0,
        "ms_per_step": args.duration * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals (seed 7), n=floor(2^U), "
                               "U~Uniform[10,26) from SplitMix64 stream seed 7, int64 "
                               "A[i]=i, seed 1e6+id, eps=0.5, 64 GiB arena",
                   "duration_s": args.duration, "rates": per_rate,
                   "value_is": f"{first_mode} elements/s at {rates[-1]:g} requests/s"},
    }
    print(json.dumps(out), flush=True)


def run_ablation(args, log):
    """Reservation variants and the auxiliary-space sweep (module docstring)."""
    import math
    import torch
    import paper_2103_01216_amd as rp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    def timed(A, variant, eps, seed):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        st = None
        for i in range(args.steps):
            ev[i][0].record(stream)
            h = rp.rp_shuffle_variant(A, variant=variant, seed=seed + i, eps=eps, stream=stream)
            ev[i][1].record(stream)
            st = h.get()
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        return ms, st

    n = WORKLOAD["n"]
    A = torch.arange(n, dtype=torch.int64, device=dev)
    ref = torch.arange(n, dtype=torch.int64, device=dev)
    rp.rp_shuffle_inplace(ref, seed=WORKLOAD["seed"], eps=0.5, stream=stream, stats=False)
    variants = {}
    names = ("final", "oneres", "twores", "flat", "naive", "linear")
    if args.variants_once:
        for name in names:
            A.copy_(torch.arange(n, dtype=torch.int64, device=dev))
            st = rp.rp_shuffle_variant(A, variant=name, seed=WORKLOAD["seed"], eps=0.5,
                                       stream=stream).get()
            same = bool(torch.equal(A, ref))
            log(f"n=2^30 {name}: rounds {st['rounds']}, attempts {st['attempts']}, "
                f"k {st['k']}, aux {st['aux_words']} words, equal to final: {same}")
            if not same:
                log("PARITY FAILURE")
                sys.exit(1)
        return
    for name in names:
        A.copy_(torch.arange(n, dtype=torch.int64, device=dev))
        rp.rp_shuffle_variant(A, variant=name, seed=WORKLOAD["seed"], eps=0.5,
                              stream=stream, stats=False)
        torch.cuda.synchronize()
        same = bool(torch.equal(A, ref))
        ms, st = timed(A, name, 0.5, 100)
        variants[name] = {"ms": ms, "elements_per_s": n / (ms * 1e-3), "equal_to_final": same,
                          "rounds": st["rounds"], "attempts": st["attempts"],
                          "retries": st["retries"], "k": st["k"],
                          "aux_words": st["aux_words"], "aux_bound_words": st["aux_bound_words"]}
        log(f"n=2^30 {name}: {ms:.1f} ms, rounds {st['rounds']}, k {st['k']}, "
            f"retries {st['retries']}, aux {st['aux_words']} words, equal to final: {same}")
        if not same:
            log("PARITY FAILURE")
            sys.exit(1)
    # The final variant at the paper's auxiliary fractions, same n.
    big_aux = []
    for label, frac in (("0.4%", 0.004), ("4%", 0.04)):
        eps = -math.log(frac) / math.log(n)
        ms, st = timed(A, "final", eps, 150)
        big_aux.append({"aux": label, "eps": eps, "ms": ms, "rounds": st["rounds"],
                        "k": st["k"], "aux_words": st["aux_words"],
                        "aux_bound_words": st["aux_bound_words"]})
        log(f"n=2^30 final, aux {label} (eps {eps:.4f}): {ms:.1f} ms, rounds {st['rounds']}, "
            f"k {st['k']}")
    del A, ref
    torch.cuda.empty_cache()

    n2 = 10**8
    A = torch.arange(n2, dtype=torch.int64, device=dev)
    sweep = []
    points = [("0.4%", 0.004), ("1%", 0.01), ("2%", 0.02), ("4%", 0.04)]
    for label, frac in points:
        eps = -math.log(frac) / math.log(n2)
        ms, st = timed(A, "final", eps, 200)
        sweep.append({"aux": label, "eps": eps, "ms": ms, "rounds": st["rounds"], "k": st["k"],
                      "aux_words": st["aux_words"], "aux_bound_words": st["aux_bound_words"]})
        log(f"n=1e8 aux {label} (eps {eps:.4f}): {ms:.1f} ms, rounds {st['rounds']}, k {st['k']}")
    for eps in (0.4, 0.5, 0.6, 0.75):
        ms, st = timed(A, "final", eps, 300)
        sweep.append({"aux": f"n^{1 - eps:.2f}", "eps": eps, "ms": ms, "rounds": st["rounds"],
                      "k": st["k"], "aux_words": st["aux_words"],
                      "aux_bound_words": st["aux_bound_words"]})
        log(f"n=1e8 eps {eps}: {ms:.1f} ms, rounds {st['rounds']}, k {st['k']}, "
            f"aux {st['aux_words']} words")
    out = {
        "metric": "reservation variants and auxiliary-space sweep (ms per shuffle)",
        "value": variants["final"]["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": variants["final"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "variants at n=2^30 int64 eps=0.5 (seed mode); aux sweep of the "
                               "final variant at n=1e8 int64",
                   "variants": variants, "final_aux_n2p30": big_aux,
                   "aux_sweep_n1e8": sweep},
    }
    print(json.dumps(out), flush=True)


def run_list(args, log):
    """List ranking by in-place list contraction (module docstring)."""
    import math
    import numpy as np
    import torch
    import paper_2103_01216_amd as rp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    n = 10**8
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    order = torch.randperm(n, device=dev, generator=g)       # the list's order
    nil = (1 << 32) - 1
    src = torch.empty((n, 2), dtype=torch.int64, device=dev)
    src[order[1:], 0] = order[:-1]
    src[order[0], 0] = nil
    src[order[:-1], 1] = order[1:]
    src[order[-1], 1] = nil
    want = torch.empty(n, dtype=torch.int64, device=dev)
    want[order] = torch.arange(n, dtype=torch.int64, device=dev)
    del order
    rec = src.clone()
    rank = torch.empty(n, dtype=torch.int64, device=dev)
    log("list: n = 1e8, one random list")
    points = [("n^0.5", 0.5), ("1.4% of n", -math.log(0.014) / math.log(n)), ("n^0.75", 0.25)]
    results = []
    for label, eps in points:
        rec.copy_(src)
        _, st = rp.rp_list_rank(rec, seed=11, eps=eps, rank=rank, stream=stream)
        ok = bool(torch.equal(rank, want))
        if not ok or st["status"] != 0:
            log(f"PARITY FAILURE at eps {eps}")
            sys.exit(1)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for i in range(args.steps):
            rec.copy_(src)
            ev[i][0].record(stream)
            rp.rp_list_rank(rec, seed=11 + i, eps=eps, rank=rank, stream=stream, stats=False)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        results.append({"aux": label, "eps": eps, "ms": ms, "elements_per_s": n / (ms * 1e-3),
                        "k": st["k"], "phases": st["phases"],
                        "contract_rounds": st["contract_rounds"],
                        "rebuild_rounds": st["rebuild_rounds"], "grid": st["grid"],
                        "aux_words": st["aux_words"], "ranks_exact": ok})
        log(f"  aux {label} (eps {eps:.3f}): {ms:.1f} ms, k {st['k']}, phases {st['phases']}, "
            f"rounds {st['contract_rounds']} + {st['rebuild_rounds']}, grid {st['grid']}")
    best = min(results, key=lambda r: r["ms"])
    # 48 B per element: the two pointer words read and written once, one rank
    # written and one rank read
    alg = 48 * n
    out = {
        "metric": "list ranking by in-place list contraction, elements/s (n=1e8)",
        "value": best["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": best["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "uint64",
        "data": "synthetic",
        "config": {"workload": "one random list of 1e8 elements (torch.randperm, seed 7), "
                               "(prev, next) 64-bit words, seed-mode priorities",
                   "points": results},
        "roofline": {"bound": "hbm", "achieved": alg / (best["ms"] * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": alg / (best["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "rp_list_kernel", "algorithmic_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        import oracle
        m = 10**7
        perm = np.random.default_rng(7).permutation(m).astype(np.uint32)
        prev = np.full(m, nil, dtype=np.uint32)
        nxt = np.full(m, nil, dtype=np.uint32)
        prev[perm[1:]] = perm[:-1]
        nxt[perm[:-1]] = perm[1:]
        t0 = time.perf_counter()
        oracle.list_rank(prev, nxt)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m / dt, "unit": "elements/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "sequential walk of one random list of 1e7 elements"}
        log(f"cpu oracle: 1e7-element list walked in {dt:.2f} s")
    print(json.dumps(out), flush=True)


def run_scale(args, log):
    """The plain method at the other stated sizes (module docstring)."""
    import numpy as np
    import torch
    import oracle
    import paper_2103_01216_amd as rp
    from paper_2103_01216_amd import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    cases = [("2^20 int64", 1 << 20, torch.int64, 0.5)]
    cases += [("2^28 int32", 1 << 28, torch.int32, e) for e in (0.25, 0.5, 0.75)]
    cases += [("2^28 int64", 1 << 28, torch.int64, e) for e in (0.25, 0.5, 0.75)]
    cases += [("2^26 x 64 B records", 1 << 26, "rec64", 0.5)]
    cases += [("2^30 int64", 1 << 30, torch.int64, e) for e in (0.2, 0.25, 1.0 / 3.0, 0.5)]
    rows = []
    A = None
    for label, n, dt, eps in cases:
        del A
        torch.cuda.empty_cache()
        A = workloads.records64(n, dev) if dt == "rec64" else workloads.identity(n, dt, dev)
        eb = A.element_size() * (A.shape[1] if A.dim() > 1 else 1)
        st = rp.rp_shuffle_inplace(A, seed=1, eps=eps, stream=stream).get()
        key = A[:, 0] if A.dim() > 1 else A
        seen = torch.zeros(n, dtype=torch.bool, device=dev)
        seen[key.long()] = True
        perm = bool(seen.all())
        del seen
        pos = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(3).integers(0, n, 256)]))
        src = oracle.sample_sources(n, pos, seed=1)
        got = key[torch.from_numpy(pos.astype(np.int64)).to(dev)].cpu().numpy()
        exact = bool(np.array_equal(got.astype(np.int64), src.astype(np.int64)))
        if not (perm and exact and st["status"] == 0):
            log(f"PARITY FAILURE: {label} eps {eps}")
            sys.exit(1)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for i in range(args.steps):
            ev[i][0].record(stream)
            rp.rp_shuffle_inplace(A, seed=2 + i, eps=eps, stream=stream, stats=False)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        times = sorted(a.elapsed_time(b) for a, b in ev)
        ms = times[len(times) // 2]
        gbps = 4 * eb * n / (ms * 1e-3) / 1e9
        rows.append({"case": label, "eps": eps, "ms_median": ms,
                     "elements_per_s": n / (ms * 1e-3), "algorithmic_gbps": gbps,
                     "frac_of_peak": gbps / HBM_PEAK_GBPS, "rounds": st["rounds"],
                     "round_us": ms * 1e3 / max(1, st["rounds"]), "k": st["k"],
                     "max_active": st["max_active"], "inflight_words": st["inflight_words"],
                     "aux_words": st["aux_words"], "aux_bound_words": st["aux_bound_words"],
                     "grid": st["grid"], "slots_per_lane": st["slots_per_lane"]})
        log(f"{label} eps {eps:.3f}: {ms:.1f} ms, {n / (ms * 1e-3):.3g} el/s, {gbps:.0f} GB/s "
            f"({100 * gbps / HBM_PEAK_GBPS:.2f} %), rounds {st['rounds']}, k {st['k']}, "
            f"aux {st['aux_words']}/{st['aux_bound_words']}")
    best = max(rows, key=lambda r: r["frac_of_peak"])
    out = {
        "metric": "in-place shuffle elements/s and % of HBM peak at the stated sizes",
        "value": best["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": best["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed",
        "data": "synthetic",
        "config": {"workload": "plain method at 2^20 int64 eps 0.5, 2^28 int32/int64 x eps "
                               "{0.25,0.5,0.75}, "
                               "2^26 x 64 B records eps 0.5, 2^30 int64 x eps {0.2,0.25,1/3,0.5}",
                   "cases": rows, "value_is": f"elements/s of {best['case']} eps {best['eps']:.3f}"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
