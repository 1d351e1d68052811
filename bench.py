#!/usr/bin/env python3
"""Benchmark: pospopcnt on 256 MiB arrays on one MI355X.

One step = one plain pospopcnt call at each width w = 8, 16, 32, 64, each on
its own 256 MiB device buffer of Bernoulli(0.5) bits (four buffers in
rotation, 1 GiB in all, so no call finds its input in the 256 MB Infinity
Cache left behind by the previous one).  Inputs are resident in HBM before
the timed region starts.

Printed: one JSON line with the whole-job throughput (GB/s, 1 GB = 1e9 B),
the roofline object of the dominant kernel (achieved bytes/s from HIP events
on the launch stream around back-to-back launches, and from events each
launch's own dispatch records on an idle queue, against the 8 TB/s HBM
peak), the read-only roofline kernel on the same buffers, every width at
three bit densities, the batched and the served forms, and the CPU oracle
timed on this host as a reported baseline.
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
    """Hash of the code (comments and blank lines stripped) of the sources
    the plain pospopcnt kernel is built from."""
    import re

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_16370_amd", "csrc")
    for name in ("ppc_device.hpp", "ppc_plain.hip"):
        with open(os.path.join(csrc, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
        h.update(name.encode() + b"\0" + code.encode())
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


def dispatch_timed(fn, bufs, reps, torch):
    """Run fn(buf, start_event, stop_event) over the buffers in rotation;
    the library's dispatch records the events, so each interval is one
    kernel's execution.  Returns per-call ms."""
    import paper_2412_16370_amd as ppc

    ev = [(ppc.HipEvent(), ppc.HipEvent()) for _ in range(reps)]
    for i in range(reps):
        fn(bufs[i % len(bufs)], ev[i][0], ev[i][1])
    torch.cuda.synchronize()
    return [a.elapsed_ms(b) for a, b in ev]


def cpu_model() -> str:
    """The host CPU's model name as lscpu reports it, with its family, model
    and stepping numbers (and its BIOS name too when the two differ), else
    /proc/cpuinfo's."""
    import subprocess

    names, ids = [], {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key in ("Model name", "BIOS Model name") and val and val not in names:
                names.append(val)
            if key in ("CPU family", "Model", "Stepping") and val:
                ids.setdefault(key, val)
    except (OSError, subprocess.SubprocessError):
        pass
    if names and ids:
        names[0] += " (family %s, model %s, stepping %s)" % (
            ids.get("CPU family", "?"), ids.get("Model", "?"), ids.get("Stepping", "?"))
    if not names:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        names.append(line.split(":", 1)[1].strip())
                        break
        except OSError:
            pass
    return " / ".join(names) or "unknown"


def cpu_baseline(runs=10):
    """The oracle on this host: the Fig. 2 word loop over the config-2 input
    (one 256 MiB array of Bernoulli(0.5) bytes) at every width, single-
    threaded and on every core this process may use (split at word
    boundaries), and over the config-1 input (2 MiB, w = 16); each figure is
    the median of `runs` timed runs."""
    import oracle
    import synth

    threads = oracle.host_threads()

    def med_gbps(fn, nbytes):
        t = []
        for _ in range(runs):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        t.sort()
        return {"median": round(nbytes / t[len(t) // 2] / 1e9, 4), "min": round(nbytes / t[-1] / 1e9, 4),
                "max": round(nbytes / t[0] / 1e9, 4)}

    t_start = time.perf_counter()
    sample = synth.random_bytes(CALL_BYTES, seed=10)
    per_width = {}
    for w in WIDTHS:
        per_width[str(w)] = {"single_thread_GBps": med_gbps(lambda: oracle.pospopcnt(sample, w), CALL_BYTES),
                             "all_cores_GBps": med_gbps(lambda: oracle.pospopcnt_mt(sample, w, threads),
                                                        CALL_BYTES)}
    cfg1 = synth.random_bytes(2 * MiB, seed=0)
    config1 = {"single_thread_GBps": med_gbps(lambda: oracle.pospopcnt(cfg1, 16), 2 * MiB),
               "all_cores_GBps": med_gbps(lambda: oracle.pospopcnt_mt(cfg1, 16, threads), 2 * MiB)}
    mt = sorted(v["all_cores_GBps"]["median"] for v in per_width.values())
    return {"value": round(sum(mt) / len(mt), 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "one 256 MiB array of random bytes at w = 8, 16, 32, 64 (the config-2 input at p = 0.5), "
                      "%d timed runs per width and thread count; value = mean over widths of the all-core "
                      "medians" % runs,
            "per_width_256MiB": per_width, "config1_2MiB_w16": config1,
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "seconds": round(time.perf_counter() - t_start, 1)}


def batched_leg(ppc, torch, synth, dev, reps):
    """10,000 arrays, log-uniform 16 B .. 16 MiB, mixed widths, per-array
    density p ~ U[0,1]: one graph launch of the persistent batched kernel
    against 10,000 plain calls on one stream (same GPU, same bytes)."""
    spec = synth.batch_spec(10_000, seed=3)
    n = len(spec["lengths"])
    pool = torch.full((spec["pool_bytes"] + 128,), 0xFF, dtype=torch.uint8, device=dev)
    for i, (off, ln, p) in enumerate(zip(spec["offsets"], spec["lengths"], spec["p"])):
        synth.device_bernoulli(int(ln), float(p), seed=3 * 1_000_003 + i, device=dev,
                               out=pool[int(off):int(off) + int(ln)])
    counts = torch.zeros((n, 64), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    total = int(spec["lengths"].sum())
    base, cbase = pool.data_ptr(), counts.data_ptr()
    addrs = [base + int(o) for o in spec["offsets"]]
    caddr = [cbase + i * 512 for i in range(n)]
    t0 = time.perf_counter()
    plan = ppc.ppc_plan_create(ppc.make_descs(addrs, spec["lengths"], caddr, spec["widths"]), n, None)
    create_s = time.perf_counter() - t0
    info = ppc.ppc_plan_get_info(plan)
    stream = torch.cuda.current_stream()
    ppc.ppc_plan_run(plan)
    torch.cuda.synchronize()
    ms = time_calls(lambda b, i: ppc.ppc_plan_run(plan), [None], reps, torch)
    ppc.ppc_plan_destroy(plan)
    batched_ms = sorted(ms)[len(ms) // 2]
    # the allocation-free batched call on the same arrays: descriptors in
    # device memory, tables built on the device every call
    raw = ppc.descs_bytes(ppc.make_descs(addrs, spec["lengths"], caddr, spec["widths"]))
    descs_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    torch.cuda.synchronize()
    na_ms = sorted(time_calls(lambda b, i: ppc.ppc_batch_noalloc(descs_dev, n), [None], reps, torch))
    noalloc_ms = na_ms[len(na_ms) // 2]
    del descs_dev
    # the same arrays as 10,000 plain calls back to back on one stream
    lib = ppc.lib()
    widths = [int(w) for w in spec["widths"]]
    lens = [int(x) for x in spec["lengths"]]
    st = stream.cuda_stream
    plain_ms = []
    for r in range(max(2, reps // 4)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for i in range(n):
            lib.ppc_pospopcnt(widths[i], caddr[i], addrs[i], lens[i], st)
        b.record(stream)
        torch.cuda.synchronize()
        plain_ms.append(a.elapsed_time(b))
    plain_med = sorted(plain_ms)[len(plain_ms) // 2]
    del pool, counts
    torch.cuda.empty_cache()
    return {"n_arrays": n, "total_bytes": total,
            "batched_GBps": round(total / (batched_ms * 1e-3) / 1e9, 1),
            "batched_ms": round(batched_ms, 3),
            "plain_calls_GBps": round(total / (plain_med * 1e-3) / 1e9, 1),
            "plain_calls_ms": round(plain_med, 3),
            "speedup_vs_plain": round(plain_med / batched_ms, 3),
            "noalloc_GBps": round(total / (noalloc_ms * 1e-3) / 1e9, 1), "noalloc_ms": round(noalloc_ms, 3),
            "tiles_per_item": info["tiles_per_item"], "waves": info["waves"],
            "n_items": info["n_items"], "tuned": ["given", "measured", "cache"][info["tuned"]],
            "plan_create_s": round(create_s, 3)}


def served_leg(ppc, torch, synth, dev, plain_gbps, n_requests=100_000, rho=0.5):
    """1 GiB pool of one-hot uint32 columns (16 x 64 MiB, 32 categories, Zipf
    s = 1.0); Poisson requests (column, width, offset, length log-uniform
    64 B .. 64 MiB) offered at rho x the plain kernel's bandwidth."""
    col_bytes = 64 * MiB
    pool = synth.device_onehot_u32_columns(16, col_bytes // 4, seed=4, device=dev)
    torch.cuda.synchronize()
    mean_len = synth.log_uniform_mean(64, 64 * MiB)
    rate = rho * plain_gbps * 1e9 / mean_len
    t = synth.serve_trace(n_requests, seed=4, n_columns=16, column_bytes=col_bytes, rate_per_s=rate,
                          lo=64, hi=64 * MiB)
    out = {"n_requests": n_requests, "offered_load": rho, "offered_req_per_s": round(rate),
           "offered_GBps": round(rho * plain_gbps, 1)}
    one = ppc.ppc_server_cfg(1, 1, 0, 0, 0, 0, 0)  # one stream, one request per batch

    def run(name, cfg, trace, k):
        server = ppc.ppc_server_create(pool, column_bytes=col_bytes, cfg=cfg)
        try:
            _, st = ppc.ppc_server_run_trace(server, trace["column"][:k], trace["width"][:k], trace["offset"][:k],
                                             trace["length"][:k], trace["arrival_ns"][:k])
        finally:
            ppc.ppc_server_destroy(server)
        log("served %s: p50 %.1f us p99 %.1f us, %.1f GB/s, mean batch %.1f" % (
            name, st["p50_ns"] / 1e3, st["p99_ns"] / 1e3, st["gbps"], st["mean_batch"]))
        return {"requests": k, "p50_us": round(st["p50_ns"] / 1e3, 1),
                "p99_us": round(st["p99_ns"] / 1e3, 1), "mean_us": round(st["mean_ns"] / 1e3, 1),
                "max_us": round(st["max_ns"] / 1e3, 1), "GBps": round(st["gbps"], 1),
                "batches": st["batches"], "mean_batch": round(st["mean_batch"], 2),
                "busy_rejections": st["busy_rejections"],
                "host_dispatch_ms": round(st["host_dispatch_ns"] / 1e6, 2),
                "host_retire_ms": round(st["host_retire_ns"] / 1e6, 2),
                "makespan_ms": round(st["makespan_ns"] / 1e6, 2)}

    out["continuous"] = run("continuous", None, t, n_requests)
    # one request at a time at the same offered load: it cannot keep up (its
    # queue grows for the whole trace), so this run measures its capacity
    k1 = min(n_requests, 20_000)
    out["one_at_a_time_overloaded"] = run("one_at_a_time (overloaded)", one, t, k1)
    out["one_at_a_time_overloaded"]["note"] = "offered the same load; capacity = GBps; latency unbounded"
    # sequential baseline at a load it sustains: half of that capacity, the
    # same trace shape, served one at a time and continuously
    cap = out["one_at_a_time_overloaded"]["GBps"]
    rate_lo = 0.5 * cap * 1e9 / mean_len
    t_lo = synth.serve_trace(10_000, seed=6, n_columns=16, column_bytes=col_bytes, rate_per_s=rate_lo,
                             lo=64, hi=64 * MiB)
    out["at_half_sequential_capacity"] = {
        "offered_GBps": round(0.5 * cap, 1), "offered_req_per_s": round(rate_lo),
        "one_at_a_time": run("one_at_a_time at half its capacity", one, t_lo, 10_000),
        "continuous": run("continuous at half the sequential capacity", None, t_lo, 10_000)}
    # the same server near saturation: 0.9 of the plain bandwidth, 50,000 requests
    rate_hi = 0.9 * plain_gbps * 1e9 / mean_len
    t_hi = synth.serve_trace(50_000, seed=5, n_columns=16, column_bytes=col_bytes, rate_per_s=rate_hi,
                             lo=64, hi=64 * MiB)
    server = ppc.ppc_server_create(pool, column_bytes=col_bytes)
    try:
        _, st = ppc.ppc_server_run_trace(server, t_hi["column"], t_hi["width"], t_hi["offset"], t_hi["length"],
                                         t_hi["arrival_ns"])
    finally:
        ppc.ppc_server_destroy(server)
    out["continuous_at_0.9"] = {"requests": 50_000, "offered_GBps": round(0.9 * plain_gbps, 1),
                                "p50_us": round(st["p50_ns"] / 1e3, 1), "p99_us": round(st["p99_ns"] / 1e3, 1),
                                "GBps": round(st["gbps"], 1), "mean_batch": round(st["mean_batch"], 2),
                                "busy_rejections": st["busy_rejections"]}
    log("served at 0.9: p50 %.1f us p99 %.1f us, %.1f GB/s" % (st["p50_ns"] / 1e3, st["p99_ns"] / 1e3, st["gbps"]))
    # plain calls for the first 20,000 requests, back to back (closed loop)
    lib = ppc.lib()
    k = min(n_requests, 20_000)
    counts = torch.zeros((k, 64), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    base, cb, st = pool.data_ptr(), counts.data_ptr(), stream.cuda_stream
    a.record(stream)
    for i in range(k):
        lib.ppc_pospopcnt(int(t["width"][i]), cb + i * 512,
                          base + int(t["column"][i]) * col_bytes + int(t["offset"][i]),
                          int(t["length"][i]), st)
    b.record(stream)
    torch.cuda.synchronize()
    out["plain_back_to_back_GBps"] = round(int(t["length"][:k].sum()) / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    del pool, counts
    torch.cuda.empty_cache()
    return out


def size_sweep(ppc, torch, synth, dev, out_path):
    """Speed by array length (the paper's main experiment, Section 5.3) on
    the GPU: for each size, calls are repeated on the same buffer and the
    same counters (loop-carried, as in Section 5.1) until at least 20 ms
    and 10 calls; the median kernel time (events recorded by the dispatch)
    gives GB/s.  The wall time per call is taken separately, over untimed
    calls back to back through the raw C entry point (no per-call Python
    marshalling, no events)."""
    sizes = sorted([1 << i for i in range(1, 31)] + [3 << i for i in range(0, 30)])
    buf = synth.device_bernoulli(sizes[-1], 0.5, seed=60, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    lib, st = ppc.lib(), torch.cuda.current_stream().cuda_stream
    if os.path.dirname(out_path):
        os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as out:
        for n in sizes:
            row = {"bytes": n}
            for w in WIDTHS + (0,):
                counts = torch.zeros(max(w, 1), dtype=torch.int64, device=dev)
                if w:
                    call = lambda a, b: ppc.ppc_pospopcnt_timed(w, counts, buf[:n], start_event=a, stop_event=b)
                else:
                    if n % 16384:
                        continue
                    call = lambda a, b: ppc.ppc_read_roofline_timed(sink, buf[:n], start_event=a, stop_event=b)
                for _ in range(3):
                    call(None, None)
                # calls back to back on one stream, each kernel timed by its
                # own dispatch (the loop-carried reuse of buffer and counters
                # of Section 5.1); at least 10 calls and 20 ms of kernel time
                times = []
                t_total = 0.0
                while len(times) < 10 or t_total < 20.0:
                    evs = [(ppc.HipEvent(), ppc.HipEvent()) for _ in range(10)]
                    for a, b in evs:
                        call(a, b)
                    torch.cuda.synchronize()
                    for a, b in evs:
                        times.append(a.elapsed_ms(b))
                        t_total += times[-1]
                    if len(times) >= 2000:
                        break
                med = sorted(times)[len(times) // 2]
                reps = max(10, min(200, int(20.0 / max(med, 1e-3))))
                cp, bp = (counts.data_ptr(), buf.data_ptr())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    if w:
                        lib.ppc_pospopcnt(w, cp, bp, n, st)
                    else:
                        lib.ppc_read_roofline(sink.data_ptr(), bp, n, st)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / reps
                key = ("w%d" % w) if w else "read_roofline"
                row[key + "_us"] = round(med * 1e3, 3)
                row[key + "_GBps"] = round(n / (med * 1e-3) / 1e9, 3)
                row[key + "_wall_us_per_call"] = round(wall * 1e6, 3)
            out.write(json.dumps(row) + "\n")
            out.flush()
            log("sweep %11d B: w16 %9.2f us %9.1f GB/s" % (n, row["w16_us"], row["w16_GBps"]))


def batched_size_sweep(ppc, torch, synth, dev, out_path):
    """The batched forms by array length: for each length L (2^i and 3*2^i
    bytes, 16 B to 16 MiB), N equal arrays of L bytes (N = 1 GiB / L, at
    least 64 and at most 65,536; widths cycling through 8, 16, 32, 64;
    starts 256 bytes apart or more).  Timed: one plan over the N arrays
    (default options: autotuned, graph replay), the allocation-free call over the same
    descriptors, each repeated for at least 10 runs and 20 ms (median), and
    256 plain calls on the first 256 arrays back to back through the raw C
    entry point (mean per call).  GB/s = bytes counted / time."""
    sizes = sorted([1 << i for i in range(4, 25)] + [3 << i for i in range(3, 23)])
    pool = synth.device_bernoulli(1 << 30, 0.5, seed=61, device=dev)
    counts = torch.zeros((65536, 64), dtype=torch.int64, device=dev)
    lib, stream = ppc.lib(), torch.cuda.current_stream()
    base, cb = pool.data_ptr(), counts.data_ptr()

    def median_ms(fn):
        for _ in range(3):
            fn(None, 0)
        torch.cuda.synchronize()
        times = []
        while len(times) < 10 or sum(times) < 20.0:
            times += time_calls(fn, [None], 10, torch)
        return sorted(times)[len(times) // 2]

    if os.path.dirname(out_path):
        os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as out:
        for L in sizes:
            stride = (L + 255) // 256 * 256
            n = int(max(64, min(65536, (1 << 30) // stride)))
            addrs = [base + i * stride for i in range(n)]
            caddr = [cb + i * 512 for i in range(n)]
            widths = [WIDTHS[i % 4] for i in range(n)]
            descs = ppc.make_descs(addrs, [L] * n, caddr, widths)
            plan = ppc.ppc_plan_create(descs, n)
            try:
                info = ppc.ppc_plan_get_info(plan)
                plan_ms = median_ms(lambda b, i: ppc.ppc_plan_run(plan))
            finally:
                ppc.ppc_plan_destroy(plan)
            descs_dev = torch.frombuffer(bytearray(ppc.descs_bytes(descs)), dtype=torch.uint8).to(dev)
            na_ms = median_ms(lambda b, i: ppc.ppc_batch_noalloc(descs_dev, n))
            del descs_dev
            k = min(n, 256)
            st = stream.cuda_stream
            for i in range(k):
                lib.ppc_pospopcnt(widths[i], caddr[i], addrs[i], L, st)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for i in range(k):
                lib.ppc_pospopcnt(widths[i], caddr[i], addrs[i], L, st)
            ev1.record(stream)
            torch.cuda.synchronize()
            plain_ms = ev0.elapsed_time(ev1) / k
            total = n * L
            row = {"array_bytes": L, "arrays": n, "total_bytes": total,
                   "plan_us": round(plan_ms * 1e3, 2), "plan_GBps": round(total / (plan_ms * 1e-3) / 1e9, 1),
                   "noalloc_us": round(na_ms * 1e3, 2), "noalloc_GBps": round(total / (na_ms * 1e-3) / 1e9, 1),
                   "plain_call_us": round(plain_ms * 1e3, 3),
                   "plain_calls_GBps": round(L / (plain_ms * 1e-3) / 1e9, 2),
                   "items": info["n_items"], "tiles_per_item": info["tiles_per_item"], "waves": info["waves"],
                   "tuned": ["given", "measured", "cache"][info["tuned"]]}
            out.write(json.dumps(row) + "\n")
            out.flush()
            log("batched sweep %8d B x %5d: plan %7.1f GB/s, no-alloc %7.1f GB/s, plain calls %8.2f GB/s"
                % (L, n, row["plan_GBps"], row["noalloc_GBps"], row["plain_calls_GBps"]))
    del pool, counts
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--kernel-seconds", type=float, default=1.0,
                    help="accumulated kernel time of the event-timed pass (at least --steps steps)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="length sweep of Section 5.2 (2^i and 3*2^i bytes up to 1.5 GiB) at every "
                         "width, repeated calls on one buffer as in the paper's harness; writes "
                         "JSON lines to --sweep-out and exits")
    ap.add_argument("--sweep-batched", action="store_true",
                    help="the batched form by array length: one plan over many equal arrays per length "
                         "(16 B to 16 MiB, 1 GiB per plan where the array count allows); writes JSON "
                         "lines to --sweep-out and exits")
    ap.add_argument("--sweep-out", default="size_sweep.jsonl",
                    help="JSON-lines file for --sweep (one line per size)")
    ap.add_argument("--ablation", action="store_true",
                    help="time the three accumulation schedules (ppc_pospopcnt_variant 0/1/2) on "
                         "256 MiB at w = 16 and exit (short: also the command to profile them)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="run for rocprofv3 counters on the batched form: the 10,000-array pool filled by "
                         "a few large generator kernels, one plan with the tuned setting (256 tiles per "
                         "item, 1024 waves; no autotuning), 3 runs, then 3 plain 256 MiB device copies "
                         "(counter calibration)")
    ap.add_argument("--profile", action="store_true",
                    help="run for rocprofv3: the plain loop (warm-up + steps), the read roofline as "
                         "often, and 3 plain 256 MiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_16370_amd as ppc
    import synth

    ppc.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("device: %s" % torch.cuda.get_device_name(dev))
    if args.sweep:
        size_sweep(ppc, torch, synth, dev, args.sweep_out)
        return
    if args.sweep_batched:
        batched_size_sweep(ppc, torch, synth, dev, args.sweep_out)
        return
    if args.profile_batched:
        spec = synth.batch_spec(10_000, seed=3)
        n = len(spec["lengths"])
        pool = torch.empty(spec["pool_bytes"] + 128, dtype=torch.uint8, device=dev)
        synth.device_bernoulli(spec["pool_bytes"] + 128, 0.5, seed=3, device=dev, out=pool)
        counts_b = torch.zeros((n, 64), dtype=torch.int64, device=dev)
        base, cbase = pool.data_ptr(), counts_b.data_ptr()
        descs = ppc.make_descs([base + int(o) for o in spec["offsets"]], spec["lengths"],
                               [cbase + i * 512 for i in range(n)], spec["widths"])
        plan = ppc.ppc_plan_create(descs, n, ppc.ppc_plan_opts(256, 1024, 0, 1, 0))
        try:
            for _ in range(3):
                ppc.ppc_plan_run(plan)
            dst = torch.empty(CALL_BYTES, dtype=torch.uint8, device=dev)
            for i in range(3):
                dst.copy_(pool[i * CALL_BYTES:(i + 1) * CALL_BYTES])
            torch.cuda.synchronize()
        finally:
            ppc.ppc_plan_destroy(plan)
        log("profile-batched run done: %d arrays, %d bytes per plan run" % (n, int(spec["lengths"].sum())))
        return
    if args.ablation:
        abufs = [synth.device_bernoulli(CALL_BYTES, 0.5, seed=30 + i, device=dev) for i in range(4)]
        c16 = torch.zeros(16, dtype=torch.int64, device=dev)
        res = {}
        for v in (0, 1, 2):
            # back-to-back calls over the rotating buffers, host clock between
            # two synchronisations (the same for every variant)
            for i in range(4):
                ppc.ppc_pospopcnt_variant(v, 16, c16, abufs[i % 4])
            torch.cuda.synchronize()
            reps = 40
            t0 = time.perf_counter()
            for i in range(reps):
                ppc.ppc_pospopcnt_variant(v, 16, c16, abufs[i % 4])
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / reps * 1e6
            res["variant%d" % v] = {"us_per_call": round(us, 2), "GBps": round(CALL_BYTES / (us * 1e-6) / 1e9, 1)}
            log("variant %d: %.2f us per call, %.1f GB/s" % (v, us, CALL_BYTES / (us * 1e-6) / 1e9))
        print(json.dumps({"ablation_256MiB_w16": res}), flush=True)
        return

    bufs = [synth.device_bernoulli(CALL_BYTES, 0.5, seed=10 + i, device=dev) for i in range(4)]
    counts = {w: torch.zeros(w, dtype=torch.int64, device=dev) for w in WIDTHS}
    torch.cuda.synchronize()
    log("inputs resident: 4 x 256 MiB")

    if args.profile:
        # the bench's own plain loop (warm-up steps, then `steps` steps of one
        # call per width), then the read roofline the same number of times,
        # then three plain 256 MiB device copies (counter calibration)
        sink = torch.zeros(1, dtype=torch.int64, device=dev)
        dst = torch.empty(CALL_BYTES, dtype=torch.uint8, device=dev)
        for i in range(args.warmup + args.steps):
            for j, w in enumerate(WIDTHS):
                ppc.ppc_pospopcnt(w, counts[w], bufs[(i + j) % 4])
        for i in range(args.warmup + args.steps):
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

    # whole-job timing: K steps of plain calls between two synchronisations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_calls(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_bytes = args.steps * len(WIDTHS) * CALL_BYTES
    value = total_bytes / wall / 1e9

    # back-to-back kernel timing (the roofline figure): the same rotation of
    # K steps again, one HIP event pair on the launch stream around each
    # pass, repeated for at least `--kernel-seconds` of GPU time.  The
    # per-launch interval is what a kernel costs when launches follow each
    # other on one stream.
    stream = torch.cuda.current_stream()
    lib, sp = ppc.lib(), stream.cuda_stream
    cptr = {w: counts[w].data_ptr() for w in WIDTHS}
    bptr = [b.data_ptr() for b in bufs]
    b2b_ms, b2b_launches = 0.0, 0
    b2b_w = {w: [] for w in WIDTHS}
    while b2b_launches < args.steps * len(WIDTHS) or b2b_ms < args.kernel_seconds * 1e3:
        for j, w in enumerate(WIDTHS):  # one width at a time: per-width intervals
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(args.steps):
                lib.ppc_pospopcnt(w, cptr[w], bptr[(i + j) % 4], CALL_BYTES, sp)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            b2b_w[w].append(ms / args.steps)
            b2b_ms += ms
            b2b_launches += args.steps
    b2b_avg_ms = b2b_ms / b2b_launches
    achieved = CALL_BYTES / (b2b_avg_ms * 1e-3) / 1e9
    per_width_b2b = {str(w): round(CALL_BYTES / (sum(v) / len(v) * 1e-3) / 1e9, 1) for w, v in b2b_w.items()}
    log("plain: %.1f GB/s whole-job (%.2f us per call); back to back %.2f us per launch over %d launches "
        "-> %.1f GB/s" % (value, wall / (args.steps * len(WIDTHS)) * 1e6, b2b_avg_ms * 1e3, b2b_launches,
                          achieved))

    # idle-queue kernel timing: every launch carries a HIP event pair that its
    # own dispatch records (kernel start and end), for at least K steps and
    # `--kernel-seconds` of kernel time.  Such events leave the queue idle for
    # ~5 us after each kernel, so every launch starts on an idle queue.
    ev = [(ppc.HipEvent(), ppc.HipEvent()) for _ in range(args.steps * len(WIDTHS))]
    per_call = {w: [] for w in WIDTHS}
    kernel_s, steps_timed = 0.0, 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    while steps_timed < args.steps or kernel_s < args.kernel_seconds:
        for i in range(args.steps):
            for j, w in enumerate(WIDTHS):
                a, b = ev[i * len(WIDTHS) + j]
                ppc.ppc_pospopcnt_timed(w, counts[w], bufs[(steps_timed + i + j) % 4], start_event=a, stop_event=b)
        torch.cuda.synchronize()
        for i in range(args.steps):
            for j, w in enumerate(WIDTHS):
                a, b = ev[i * len(WIDTHS) + j]
                ms = a.elapsed_ms(b)
                per_call[w].append(ms)
                kernel_s += ms * 1e-3
        steps_timed += args.steps
    wall_timed = time.perf_counter() - t1
    all_ms = sorted(x for v in per_call.values() for x in v)
    avg_ms = sum(all_ms) / len(all_ms)
    achieved_idle = CALL_BYTES / (avg_ms * 1e-3) / 1e9
    log("plain, idle-queue launches: kernel avg %.2f us over %d launches -> %.1f GB/s"
        % (avg_ms * 1e3, len(all_ms), achieved_idle))

    # read-only roofline kernel on the same buffers
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    for i in range(args.warmup):
        ppc.ppc_read_roofline(sink, bufs[i % 4])
    rl = dispatch_timed(lambda b, e0, e1: ppc.ppc_read_roofline_timed(sink, b, start_event=e0, stop_event=e1),
                        bufs, 4 * args.steps, torch)
    rl_gbps = CALL_BYTES / (sum(rl) / len(rl) * 1e-3) / 1e9
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(4 * args.steps):
        lib.ppc_read_roofline(sink.data_ptr(), bptr[i % 4], CALL_BYTES, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    rl_b2b_gbps = CALL_BYTES * 4 * args.steps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    log("read roofline: %.1f GB/s idle-queue, %.1f GB/s back to back" % (rl_gbps, rl_b2b_gbps))

    # density does not change the speed (all-integer, data-independent work):
    # every width at p = 0.01, 0.5, 0.99, back to back over 4 rotating
    # buffers of that density, each for at least `--kernel-seconds`
    def b2b_gbps(cbufs, w):
        done_ms, n = 0.0, 0
        cp = counts[w].data_ptr()
        ptrs = [b.data_ptr() for b in cbufs]
        while done_ms < args.kernel_seconds * 1e3 or n < 100:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(100):
                lib.ppc_pospopcnt(w, cp, ptrs[i % len(ptrs)], CALL_BYTES, sp)
            e1.record(stream)
            torch.cuda.synchronize()
            done_ms += e0.elapsed_time(e1)
            n += 100
        return {"GBps": round(CALL_BYTES * n / (done_ms * 1e-3) / 1e9, 1),
                "us_per_launch": round(done_ms / n * 1e3, 2), "launches": n}

    density = {}
    for p in (0.01, 0.5, 0.99):
        dbufs = bufs if p == 0.5 else [synth.device_bernoulli(CALL_BYTES, p, seed=20 + i, device=dev)
                                       for i in range(4)]
        torch.cuda.synchronize()
        density[str(p)] = {str(w): b2b_gbps(dbufs, w) for w in WIDTHS}
        if p != 0.5:
            del dbufs
    log("density matrix (GB/s back to back): " + "; ".join(
        "p=%s: %s" % (p, " ".join("%s" % v[str(w)]["GBps"] for w in WIDTHS)) for p, v in density.items()))

    # the total popcount (the same front end, all 64 positions summed into
    # one counter) on the same buffers, back to back
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    done_ms, n_pc = 0.0, 0
    while done_ms < args.kernel_seconds * 1e3 or n_pc < 100:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(100):
            lib.ppc_popcount(total.data_ptr(), bptr[i % 4], CALL_BYTES, sp)
        e1.record(stream)
        torch.cuda.synchronize()
        done_ms += e0.elapsed_time(e1)
        n_pc += 100
    popcount = {"GBps": round(CALL_BYTES * n_pc / (done_ms * 1e-3) / 1e9, 1),
                "us_per_launch": round(done_ms / n_pc * 1e3, 2), "launches": n_pc}
    log("total popcount, back to back: %.2f us per 256 MiB launch -> %.1f GB/s"
        % (popcount["us_per_launch"], popcount["GBps"]))

    def us_stats(v):
        v = sorted(v)
        return {"avg": round(sum(v) / len(v) * 1e3, 2), "median": round(v[len(v) // 2] * 1e3, 2),
                "min": round(v[0] * 1e3, 2), "max": round(v[-1] * 1e3, 2), "launches": len(v)}

    per_width = {str(w): round(CALL_BYTES / (sum(v) / len(v) * 1e-3) / 1e9, 1)
                 for w, v in per_call.items()}
    per_width_us = {str(w): us_stats(v) for w, v in per_call.items()}

    # one GPU's share of a 256 MiB array split over 8 GPUs: 32 MiB slices of
    # the four buffers, 32 distinct slices in rotation (1 GiB, DRAM-resident)
    slices = [b[k * 32 * MiB:(k + 1) * 32 * MiB] for b in bufs for k in range(8)]
    c16 = torch.zeros(16, dtype=torch.int64, device=dev)
    shard = dispatch_timed(lambda b, e0, e1: ppc.ppc_pospopcnt_timed(16, c16, b, start_event=e0, stop_event=e1),
                           slices, 4 * len(slices), torch)
    shard_us = sum(shard) / len(shard) * 1e3
    del slices

    # config 1: one 2 MiB array of 2^20 uint16 words, random bytes from seed 0
    small = torch.from_numpy(synth.random_bytes(2 * MiB, seed=0)).to(dev)
    for _ in range(10):
        ppc.ppc_pospopcnt(16, c16, small)
    small_ms = sorted(dispatch_timed(lambda b, e0, e1: ppc.ppc_pospopcnt_timed(16, c16, b, start_event=e0,
                                                                                 stop_event=e1),
                                     [small], 200, torch))
    st = sp
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(500):
        lib.ppc_pospopcnt(16, c16.data_ptr(), small.data_ptr(), 2 * MiB, st)
    torch.cuda.synchronize()
    small_wall_us = (time.perf_counter() - t2) / 500 * 1e6
    del small
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
                     "traffic": traffic_from_profiles(),
                     "achieved_idle_queue": round(achieved_idle, 1),
                     "frac_idle_queue": round(achieved_idle / HBM_PEAK_GBPS, 4),
                     "measure": "achieved/frac: launches back to back on one stream, a HIP event pair on that "
                                "stream around each pass of K launches (%d launches, %.2f us per launch); "
                                "achieved_idle_queue/frac_idle_queue: events recorded by each launch's own "
                                "dispatch, every launch starting on an idle queue (%d launches, %.2f us avg)"
                                % (b2b_launches, b2b_avg_ms * 1e3, len(all_ms), avg_ms * 1e3)},
        "kernel_avg_us": round(avg_ms * 1e3, 2),
        "kernel_us": us_stats(all_ms) | {"seconds": round(kernel_s, 3)},
        "kernel_us_per_width": per_width_us,
        "b2b_us_per_launch": round(b2b_avg_ms * 1e3, 2),
        "wall_us_per_call": round(wall / (args.steps * len(WIDTHS)) * 1e6, 2),
        "timing": "value: K steps of plain calls (4 widths each), host clock between two synchronisations; "
                  "roofline.achieved: the same calls back to back, GPU events around each pass, at least "
                  "%.1f s; per_width_GBps and kernel_us_per_width: idle-queue launches (whole-job rate of "
                  "that pass, which leaves the queue idle after every kernel: %.1f GB/s)"
                  % (args.kernel_seconds, steps_timed * len(WIDTHS) * CALL_BYTES / wall_timed / 1e9),
        "per_width_GBps": per_width,
        "per_width_b2b_GBps": per_width_b2b,
        "popcount_256MiB_b2b": popcount,
        "density_GBps_b2b": density,
        "read_roofline_GBps": round(rl_gbps, 1),
        "read_roofline_b2b_GBps": round(rl_b2b_gbps, 1),
        "shard_32MiB_w16": {"kernel_avg_us": round(shard_us, 2),
                            "GBps": round(32 * MiB / (shard_us * 1e-6) / 1e9, 1),
                            "frac": round(32 * MiB / (shard_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                            "note": "one GPU's share of a 256 MiB array split over 8 GPUs; "
                                    "32 distinct 32 MiB slices in rotation"},
        "config1_2MiB_w16": {"kernel_median_us": round(small_ms[len(small_ms) // 2] * 1e3, 2),
                             "kernel_GBps": round(2 * MiB / (small_ms[len(small_ms) // 2] * 1e-3) / 1e9, 1),
                             "wall_us_per_call": round(small_wall_us, 2),
                             "note": "latency-bound: one kernel launch per 2 MiB"},
        "frac_of_read_roofline": round(achieved / rl_b2b_gbps, 4),
        "frac_of_read_roofline_idle_queue": round(achieved_idle / rl_gbps, 4),
    }
    del bufs
    torch.cuda.empty_cache()

    if not args.no_batched:
        log("batched leg: 10,000 arrays")
        result["batched"] = batched_leg(ppc, torch, synth, dev, reps=max(8, args.steps))
        log("batched: %s" % result["batched"])
    if not args.no_served:
        log("served leg: Poisson trace at half of the plain bandwidth")
        result["served"] = served_leg(ppc, torch, synth, dev, achieved)

    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
