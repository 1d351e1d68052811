#!/usr/bin/env python3
"""Benchmark: pospopcnt on 256 MiB arrays on one MI355X.

One step = one plain pospopcnt call at each width w = 8, 16, 32, 64, each on
its own 256 MiB device buffer of Bernoulli(0.5) bits (four buffers in
rotation, 1 GiB in all, so no call finds its input in the 256 MB Infinity
Cache left behind by the previous one).  Inputs are resident in HBM before
the timed region starts.

Printed: one JSON line with the whole-job throughput (GB/s, 1 GB = 1e9 B),
the roofline object of the dominant kernel (achieved bytes/s from HIP events
around every timed launch, against the 8 TB/s HBM peak), the read-only
roofline kernel on the same buffers, density variants, the batched and the
served forms, and the CPU oracle timed on this host as a reported baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
MiB = 1 << 20
CALL_BYTES = 256 * MiB
WIDTHS = (8, 16, 32, 64)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_16370_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pospopcnt_256MiB_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def time_calls(fn, bufs, reps, torch):
    """Run fn(buf) over the buffers in rotation `reps` times with an event
    pair around each call on the launch stream; returns per-call ms."""
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for i in range(reps):
        ev[i][0].record(stream)
        fn(bufs[i % len(bufs)], i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def cpu_baseline(seconds_target=15.0):
    """The oracle on this host: multithreaded word loop over a bounded
    sample of the same workload (256 MiB of Bernoulli(0.5) bytes at each
    width, as many passes as fit the time target)."""
    import oracle
    import synth

    threads = min(16, os.cpu_count() or 1)
    sample = synth.random_bytes(64 * MiB, seed=0)
    done = 0
    t0 = time.perf_counter()
    while True:
        for w in WIDTHS:
            oracle.pospopcnt_mt(sample, w, threads)
            done += sample.size
        if time.perf_counter() - t0 > seconds_target / 2:
            break
    mt = done / (time.perf_counter() - t0) / 1e9
    t0 = time.perf_counter()
    oracle.pospopcnt(sample[: 16 * MiB], 16)
    st = 16 * MiB / (time.perf_counter() - t0) / 1e9
    return {"value": round(mt, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "%d MiB passes of 64 MiB random bytes over w=8,16,32,64 "
                      "(multithreaded word loop, split at word boundaries)" % (done // MiB),
            "single_thread_GBps": round(st, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short fixed run for rocprofv3: 3 plain calls per width, 3 read-roofline "
                         "calls and 3 plain 256 MiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_16370_amd as ppc
    import synth

    ppc.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("device: %s" % torch.cuda.get_device_name(dev))

    bufs = [synth.device_bernoulli(CALL_BYTES, 0.5, seed=10 + i, device=dev) for i in range(4)]
    counts = {w: torch.zeros(w, dtype=torch.int64, device=dev) for w in WIDTHS}
    torch.cuda.synchronize()
    log("inputs resident: 4 x 256 MiB")

    if args.profile:
        sink = torch.zeros(1, dtype=torch.int64, device=dev)
        dst = torch.empty(CALL_BYTES, dtype=torch.uint8, device=dev)
        for i in range(3):
            for j, w in enumerate(WIDTHS):
                ppc.ppc_pospopcnt(w, counts[w], bufs[(i + j) % 4])
        for i in range(3):
            ppc.ppc_read_roofline(sink, bufs[i % 4])
        for i in range(3):
            dst.copy_(bufs[i % 4])
        torch.cuda.synchronize()
        log("profile run done")
        return

    def step_calls(i0):
        for j, w in enumerate(WIDTHS):
            ppc.ppc_pospopcnt(w, counts[w], bufs[(i0 + j) % 4])

    for i in range(args.warmup):
        step_calls(i)
    torch.cuda.synchronize()

    # whole-job timing: K steps between two synchronisations
    stream = torch.cuda.current_stream()
    ev = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        for j, w in enumerate(WIDTHS):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ppc.ppc_pospopcnt(w, counts[w], bufs[(i + j) % 4])
            b.record(stream)
            ev.append((w, a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_call = {w: [] for w in WIDTHS}
    for w, a, b in ev:
        per_call[w].append(a.elapsed_time(b))
    all_ms = [x for v in per_call.values() for x in v]
    avg_ms = sum(all_ms) / len(all_ms)
    total_bytes = args.steps * len(WIDTHS) * CALL_BYTES
    value = total_bytes / wall / 1e9
    achieved = CALL_BYTES / (avg_ms * 1e-3) / 1e9
    log("plain: %.1f GB/s whole-job, kernel avg %.2f us -> %.1f GB/s" % (value, avg_ms * 1e3, achieved))

    # read-only roofline kernel on the same buffers
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    for i in range(args.warmup):
        ppc.ppc_read_roofline(sink, bufs[i % 4])
    rl = time_calls(lambda b, i: ppc.ppc_read_roofline(sink, b), bufs, 4 * args.steps, torch)
    rl_gbps = CALL_BYTES / (sum(rl) / len(rl) * 1e-3) / 1e9
    log("read roofline: %.1f GB/s" % rl_gbps)

    # density does not change the speed (all-integer, data-independent work)
    density = {}
    for p in (0.01, 0.99):
        dbufs = [synth.device_bernoulli(CALL_BYTES, p, seed=20 + i, device=dev) for i in range(4)]
        c16 = torch.zeros(16, dtype=torch.int64, device=dev)
        ms = time_calls(lambda b, i: ppc.ppc_pospopcnt16(c16, b), dbufs, 4 * args.steps, torch)
        density[str(p)] = round(CALL_BYTES / (sum(ms) / len(ms) * 1e-3) / 1e9, 1)
        del dbufs
    density["0.5"] = round(CALL_BYTES / (sum(per_call[16]) / len(per_call[16]) * 1e-3) / 1e9, 1)

    per_width = {str(w): round(CALL_BYTES / (sum(v) / len(v) * 1e-3) / 1e9, 1)
                 for w, v in per_call.items()}
    result = {
        "metric": "pospopcnt GB/s & % HBM peak (256 MiB); batched vs plain; served p50/p99",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic: seeded Bernoulli(0.5) bits generated on the device",
        "config": {"workload": "pospopcnt plain call, one 256 MiB array per call, "
                               "w = 8,16,32,64 per step, 4 rotating 256 MiB buffers",
                   "bytes_per_call": CALL_BYTES, "calls_per_step": len(WIDTHS)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_from_profiles()},
        "kernel_avg_us": round(avg_ms * 1e3, 2),
        "per_width_GBps": per_width,
        "density_GBps_w16": density,
        "read_roofline_GBps": round(rl_gbps, 1),
        "frac_of_read_roofline": round(achieved / rl_gbps, 4),
    }
    del bufs
    torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
