#!/usr/bin/env python3
"""Benchmark: in-place random permutation of n = 2^30 int64 on one MI355X.

One step = one complete call of rp_shuffle_inplace on the 8 GiB array (every
round of the RP-Final path: refill, reserve, commit, clean), eps = 0.5, so
auxiliary space is at most floor(n^0.5) = 32768 words.  A is resident in HBM
before the timed region; the shuffle's work does not depend on A's contents,
so consecutive steps shuffle the same array again (seed = 1 + step).

Prints one JSON line (see the "metric"/"roofline"/"cpu_baseline" fields).
The first warm-up step runs on the identity array and is checked against the
CPU oracle (sampled positions, exact) and for being a permutation.
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
WORKLOAD = {"n": 1 << 30, "elem_bytes": 8, "eps": 0.5, "seed": 1}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rp_rounds_kernel_n2p30_int64_eps0.5_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2103_01216_amd", "csrc", f)
               for f in ("rp.hip", "rp_device.h")]


def _src_hash() -> str:
    """sha256[:16] over the sources the shuffle kernel is compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic_bytes():
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != _src_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(log):
    """Time the CPU oracle (sequential Knuth shuffle, one core) on a sample."""
    import numpy as np
    import oracle
    n = 1 << 27
    A = np.arange(n, dtype=np.int64)
    t0 = time.perf_counter()
    oracle.knuth_shuffle_seed(A, WORKLOAD["seed"])
    dt = time.perf_counter() - t0
    log(f"cpu oracle: n=2^27 int64 in {dt:.2f} s")
    return {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": "full sequential Knuth shuffle (seed mode, targets drawn "
                      "inline) of a 2^27-element int64 array (1 GiB) on one "
                      "host core; per-element rate quoted for the 2^30 workload"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not "
              "supported by this build (the single-GPU kernel is the whole "
              "path; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)
    warmup = max(1, args.warmup)

    import numpy as np
    import torch
    import paper_2103_01216_amd as rp

    n, eb, eps = WORKLOAD["n"], WORKLOAD["elem_bytes"], WORKLOAD["eps"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    A = torch.arange(n, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"allocated A: n=2^30 int64 ({A.numel() * 8 / 2**30:.0f} GiB)")

    stats = None
    parity = {"checked": False}
    for w in range(warmup):
        stats = rp.rp_shuffle_inplace(A, seed=WORKLOAD["seed"] + w, eps=eps,
                                      stream=stream).get()
        log(f"warmup {w}: rounds={stats['rounds']} k={stats['k']} "
            f"aux={stats['aux_words']}/{stats['aux_bound_words']} words")
        if w == 0 and not args.no_check:
            import oracle
            seen = torch.zeros(n, dtype=torch.bool, device=dev)
            seen[A] = True
            perm_ok = bool(seen.all())
            del seen
            rng = np.random.default_rng(7)
            pos = np.unique(np.concatenate([[0, 1, n - 2, n - 1],
                                            rng.integers(0, n, 1024)]))
            t0 = time.perf_counter()
            src = oracle.sample_sources(n, pos, seed=WORKLOAD["seed"])
            got = A[torch.from_numpy(pos.astype(np.int64)).to(dev)].cpu().numpy()
            exact = bool(np.array_equal(got, src.astype(np.int64)))
            log(f"parity: permutation={perm_ok} sampled_exact={exact} "
                f"({len(pos)} positions, oracle {time.perf_counter() - t0:.1f} s)")
            parity = {"checked": True, "permutation": perm_ok,
                      "sampled_positions_exact": exact, "positions": int(len(pos))}
            if not (perm_ok and exact):
                log("PARITY FAILURE")
                sys.exit(1)

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

    alg_bytes = 4 * eb * n                      # A[s], A[H[s]]: read + write
    achieved = alg_bytes / (ms * 1e-3) / 1e9    # GB/s over the kernel's time
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
                   "aux_words": stats["aux_words"],
                   "aux_bound_words": stats["aux_bound_words"],
                   "grid": stats["grid"], "slots_per_lane": stats["slots_per_lane"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "kernel": "rp_rounds_kernel", "kernel_ms_events": ms,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "parity": parity,
    }
    if not args.no_cpu_baseline:
        del A
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
