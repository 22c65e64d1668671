#!/usr/bin/env python3
"""Throughput of the batched skip-list index on one MI355X.

Workload (default): 2^26 distinct uniform uint64 keys bulk-loaded; batches of
2^22 SEARCH queries with keys uniform over the loaded keys (Zipf(theta) with
--theta).  A step is one pi_execute_batch: ordering, descent, ownership,
apply, counters -- the whole hot path -- over one batch already resident in
HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--theta 0.99] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import re
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "Mqueries/s at 64M uint64 keys + % HBM peak; p50/p99 batch latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _block_from(text, start):
    """Text of the top-level definition that starts at `start` (up to the
    first line that is a lone closing brace)."""
    i = text.index(start)
    j = text.index("\n}\n", i)
    return text[i:j + 3]


def _code_only(text):
    """Source text without comments and with whitespace collapsed, so that a
    comment edit does not count as a kernel change."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def _span(text, start, end):
    """Text from the line holding `start` up to and including `end`."""
    i = text.index(start)
    j = text.index(end, i)
    return text[i:j + len(end)]


def kernel_source_hash():
    """Hash of the code the descent kernel is built and launched from: its
    device header (descent.h) in full; from pi_internal.h the structures it
    reads (IndexDesc, DevState) and the wave64 helpers; from batch.hip the
    kernel itself and its launch functions.  Host code elsewhere does not
    count."""
    csrc = os.path.join(ROOT, "paper_1601_00159_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "descent.h")) as fh:
        h.update(_code_only(fh.read()).encode())
    with open(os.path.join(csrc, "pi_internal.h")) as fh:
        t = fh.read()
    for a, b in (("struct IndexDesc {", "\n};\n"), ("struct DevState {", "\n};\n"),
                 ("// wave64 helpers", "// Height rule")):
        h.update(_code_only(_span(t, a, b)).encode())
    with open(os.path.join(csrc, "batch.hip")) as fh:
        b = fh.read()
    h.update(_code_only(_block_from(b, "template <int MODE, int QPL, int DT>\n__global__")).encode())
    for name in ("launch_descend_q", "launch_descend_b", "launch_descend("):
        m = re.search(r"^[\w:<>]+ " + re.escape(name), b, re.M)  # any return type
        h.update(_code_only(_block_from(b, m.group(0))).encode())
    return h.hexdigest()[:16]


def load_traffic(workload_name):
    """HBM bytes per descent launch from the committed rocprofv3 counter
    summary, or None when the kernel has changed since it was taken."""
    p = os.path.join(ROOT, "profiles", "descend_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash() or d.get("workload") != workload_name:
        return None
    return d.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


class OneCore:
    """Pins this process to one core of those it may use for the duration of
    the CPU-baseline leg (the oracle is single-threaded), then restores the
    affinity."""

    def __enter__(self):
        self.prev = os.sched_getaffinity(0)
        self.core = min(self.prev)
        os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *a):
        os.sched_setaffinity(0, self.prev)


def oracle_rate(orc, b, limit, budget_s, chunk):
    """Queries per second of the oracle over the first `limit` queries of
    batch b, in chunks until `budget_s` seconds of work; each chunk is timed
    by the oracle itself (monotonic clock around its loop)."""
    done, elapsed_ns = 0, 0
    while done < min(limit, len(b)) and elapsed_ns < budget_s * 1e9:
        s_ = slice(done, done + chunk)
        _, _, ns = orc.execute_batch_timed(b.ops[s_], b.keys[s_], b.vals[s_])
        elapsed_ns += ns
        done += b.ops[s_].size
    return done, elapsed_ns / 1e9


def cpu_baseline(w, sample_queries, budget_s=12.0):
    """The CPU oracle (single-threaded Pugh skip list) on a bounded sample of
    the same workload: the full index, the first `sample_queries` queries of
    the first timed batch, in chunks until `budget_s` seconds of work, on one
    pinned core."""
    import numpy as np

    from oracle.skiplist import SkipList

    t0 = time.perf_counter()
    sk = np.sort(w.load_keys)
    order = np.argsort(w.load_keys, kind="stable")
    sv = w.load_vals[order]
    orc = SkipList()
    orc.bulk_load_sorted(sk, sv)
    log(f"oracle built in {time.perf_counter() - t0:.1f}s")
    with OneCore() as pin:
        done, elapsed = oracle_rate(orc, w.batches[0], sample_queries, budget_s, 1 << 18)
    orc.close()
    return {"value": done / elapsed / 1e6, "unit": "Mqueries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} SEARCH queries of one batch against the full {w.load_keys.size}-key index "
                      f"(single-threaded Pugh skip list pinned to core {pin.core}, {elapsed:.1f}s timed inside "
                      f"the oracle; host CPU {cpu_model()}, {os.cpu_count()} logical CPUs)"}


def run_range(args):
    """Range searches (--workload range): batches of --ranges range queries at
    each granularity of --granularity over the loaded keys; each batch is
    count -> read the total -> collect.  One JSON line per granularity."""
    import numpy as np
    import torch

    from paper_1601_00159_amd import workloads as W
    from paper_1601_00159_amd.index import Index, to_device_u64, to_numpy_u64

    dev = torch.device("cuda", 0)
    K, WU = args.steps, args.warmup
    orc = None
    for g in [int(x) for x in args.granularity.split(",")]:
        w = W.range_scan(args.load_log2, args.ranges, g, n_batches=K + WU)
        ix = Index(device=0)
        ix.bulk_load(w.load_keys, w.load_vals)
        lo = [to_device_u64(a, dev) for a, _ in w.batches]
        hi = [to_device_u64(b, dev) for _, b in w.batches]
        results = 0
        lat = []
        coll_ms = 0.0
        torch.cuda.synchronize()
        for i in range(K + WU):
            t0 = time.perf_counter()
            off = ix.range_count(lo[i], hi[i])
            total = int(off[-1].item())
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            k, v = ix.range_collect(lo[i], hi[i], off, total)
            e1.record()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if i >= WU:
                lat.append(dt)
                results += total
                coll_ms += e0.elapsed_time(e1)
        # the last batch against sorted arrays (cheap check)
        order = np.argsort(w.load_keys, kind="stable")
        sk, sv = w.load_keys[order], w.load_vals[order]
        a = np.searchsorted(sk, w.batches[-1][0], side="left")
        b = np.searchsorted(sk, w.batches[-1][1], side="right")
        idx = np.concatenate([np.arange(x, y) for x, y in zip(a.tolist(), b.tolist())])
        ok = bool(np.array_equal(to_numpy_u64(k), sk[idx]) and np.array_equal(to_numpy_u64(v), sv[idx]))
        ix.close()
        tot = sum(lat)
        # the collect call (ordering, locate, compaction) against HBM: each
        # result is read (key, value: 16 B) and written (16 B); each range
        # reads its bounds and offsets (32 B)
        algo = results * 32 + K * args.ranges * 32
        achieved = algo / (coll_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "range collect call",
                "kernel_ms": round(coll_ms / K, 4), "algorithmic_bytes_per_launch": int(algo / K)}
        cpu = None
        if not args.no_cpu_baseline:
            if orc is None:
                orc = range_oracle(w)
            cpu = range_cpu_baseline(w, orc)
        print(json.dumps({
            "metric": "Mranges/s (range search, count + collect)", "value": round(K * args.ranges / tot / 1e6, 3),
            "unit": "Mranges/s", "n_gpus": 1, "steps": K, "warmup": WU, "ms_per_step": round(tot / K * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": w.name, "loaded_keys": int(w.load_keys.size), "ranges_per_batch": args.ranges,
                       "granularity": g, "parallelism": "single GPU"},
            "results_per_s_M": round(results / tot / 1e6, 2), "mean_results_per_range": round(results / K / args.ranges, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
                           "p99": round(float(np.percentile(lat, 99)) * 1e3, 4)},
            "correct_last_batch": ok, "roofline": roof, "cpu_baseline": cpu}), flush=True)
    if orc is not None:
        orc.close()


def range_oracle(w):
    """The CPU oracle holding the range workload's index (built once)."""
    import numpy as np

    from oracle.skiplist import SkipList

    order = np.argsort(w.load_keys, kind="stable")
    orc = SkipList()
    orc.bulk_load_sorted(w.load_keys[order], w.load_vals[order])
    return orc


def range_cpu_baseline(w, orc, budget_s=8.0):
    """The CPU oracle's range search on the same index and the first batch's
    ranges, in chunks until budget_s seconds of work."""
    lo, hi = w.batches[0]
    done, elapsed, chunk = 0, 0.0, 256
    while done < lo.size and elapsed < budget_s:
        t = time.perf_counter()
        orc.range_batch(lo[done:done + chunk], hi[done:done + chunk])
        elapsed += time.perf_counter() - t
        done += min(chunk, lo.size - done)
    return {"value": round(done / elapsed / 1e6, 4), "unit": "Mranges/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} ranges of one batch against the full {w.load_keys.size}-key index "
                      f"(single-threaded Pugh skip list, {elapsed:.1f}s timed)"}


def write_oracle_replay(w):
    """Starts the CPU oracle's replay of every batch of the write workload in
    a thread of its own (its ctypes calls release the interpreter lock): the
    last batch's answers and the final set check the GPU run.  Returns a
    future of (last answers, final keys, final values)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle.skiplist import SkipList

    def replay():
        order = np.argsort(w.load_keys, kind="stable")
        orc = SkipList()
        orc.bulk_load_sorted(w.load_keys[order], w.load_vals[order])
        last = None
        for i, b in enumerate(w.batches):
            last = orc.execute_batch(b.ops, b.keys, b.vals)
            log(f"oracle replay: batch {i + 1} of {len(w.batches)}")
        k, v = orc.export()
        orc.close()
        return last, k, v

    return cf.ThreadPoolExecutor(1).submit(replay)


def write_cpu_baseline(w, budget_s=10.0):
    """The CPU oracle on the write-heavy workload: the full index, the first
    batch's queries in arrival order, in chunks until budget_s seconds, on one
    pinned core."""
    import numpy as np

    from oracle.skiplist import SkipList

    order = np.argsort(w.load_keys, kind="stable")
    orc = SkipList()
    orc.bulk_load_sorted(w.load_keys[order], w.load_vals[order])
    with OneCore() as pin:
        done, elapsed = oracle_rate(orc, w.batches[0], len(w.batches[0]), budget_s, 1 << 16)
    orc.close()
    return {"value": round(done / elapsed / 1e6, 4), "unit": "Mqueries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} queries (40/50/10 S/I/D, Zipf 0.99) of one batch against the full "
                      f"{w.load_keys.size}-key index (single-threaded Pugh skip list pinned to core {pin.core}, "
                      f"{elapsed:.1f}s timed inside the oracle; host CPU {cpu_model()})"}


def run_write(args):
    """Write-heavy skew (--workload write): 2^26 loaded keys, batches of 2^22
    queries 40/50/10 SEARCH/INSERT/DELETE, SEARCH and DELETE keys Zipf 0.99
    over the loaded keys, INSERT keys fresh; threshold rebuilds run inside the
    timed batches."""
    import numpy as np
    import torch

    from paper_1601_00159_amd import workloads as W
    from paper_1601_00159_amd.index import Index, to_device_u64, to_device_u8

    from paper_1601_00159_amd import bytemodel
    from paper_1601_00159_amd.index import to_numpy_u64

    dev = torch.device("cuda", 0)
    K, WU = args.steps, args.warmup
    t0 = time.perf_counter()
    w = W.write_skew(args.load_log2, args.batch_log2, n_batches=K + WU)
    log(f"workload {w.name}: {w.note}; generated in {time.perf_counter() - t0:.1f}s")
    replay = None if args.no_check else write_oracle_replay(w)
    Q = 1 << args.batch_log2
    d = [(to_device_u8(b.ops, dev), to_device_u64(b.keys, dev), to_device_u64(b.vals, dev)) for b in w.batches]
    out_v = torch.empty(Q, dtype=torch.int64, device=dev)
    out_s = torch.empty(Q, dtype=torch.uint8, device=dev)
    ix = Index(device=0, profile=1, rebuild_policy=args.rebuild_policy, order_bits=args.order_bits)
    ix.bulk_load(w.load_keys, w.load_vals)
    for i in range(WU):
        ix.execute_raw(*d[i], out_v, out_s)
    torch.cuda.synchronize()
    ix.profile(reset=True)
    r0 = ix.stats()["repairs"]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for i in range(K):
        evs[i][0].record()
        ix.execute_raw(*d[WU + i], out_v, out_s)
        evs[i][1].record()
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    prof = ix.profile(reset=True)
    st = ix.stats()
    last_v, last_s = to_numpy_u64(out_v), out_s.cpu().numpy()
    ek, ev = ix.export()
    ek, ev = to_numpy_u64(ek), to_numpy_u64(ev)
    ix.close()
    nb = max(prof["batches"], 1)
    # algorithmic bytes of a batch: the whole-batch model of the read path on
    # the index as loaded (the index layer is rebuilt every few batches, so
    # this is close to the levels the batches see), plus per new node 21 B
    # (key, value, flag, link) and its predecessor's link (5 B), per in-place
    # update or delete flag one value or flag write (9 B)
    lb = w.batches[WU]
    bm = bytemodel.descent_bytes(np.sort(w.load_keys), np.sort(lb.keys), lds_from=st["lds_from"])
    new_nodes = st["new_nodes"] / max(st["batches"], 1)
    upd = int((lb.ops != 0).sum()) - new_nodes
    wbytes = bytemodel.batch_bytes(bm, Q) + Q * 8 + new_nodes * (21 + 5) + max(upd, 0) * 9
    wach = wbytes / (total_ms / K / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(wach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(wach / HBM_PEAK_GBS, 4), "traffic": None, "scope": "whole batch (ms_per_step)",
            "algorithmic_bytes_per_batch": int(wbytes), "bytes_per_query": round(wbytes / Q, 2),
            "note": "descent lines counted on the index as loaded"}
    correct = None
    if replay is not None:
        log("waiting for the oracle replay")
        (wv, ws), ok, ov = replay.result()
        correct = bool(np.array_equal(last_v, wv) and np.array_equal(last_s, ws) and np.array_equal(ek, ok)
                       and np.array_equal(ev, ov))
        log(f"last batch and final set against the oracle: {correct}")
    print(json.dumps({
        "metric": "Mqueries/s, write-heavy Zipf batches", "value": round(K * Q / (total_ms / 1e3) / 1e6, 2),
        "unit": "Mqueries/s", "n_gpus": 1, "steps": K, "warmup": WU, "ms_per_step": round(total_ms / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w.name, "loaded_keys": int(w.load_keys.size), "batch_queries": Q,
                   "op_mix": "40/50/10 S/I/D", "key_distribution": "zipf 0.99 (inserts fresh uniform)",
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                       "max": round(float(lat.max()), 4), "per_batch": [round(float(x), 3) for x in lat]},
        "stages_ms_per_batch": {k: round(prof[k] / nb, 4) for k in ("sort_ms", "descend_ms", "own_ms", "link_ms")},
        "rebuild_policy": args.rebuild_policy,
        "rebuilds_in_timed_region": st["repairs"] - r0,
        "index_rebuilds": st["index_rebuilds"],
        "rebuild_ms_total": round(prof["rebuild_ms"], 3),
        "live_nodes_after": st["live_nodes"], "correct_last_batch": correct, "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else write_cpu_baseline(w)}), flush=True)


def serve_cpu_baseline(w, budget_s=8.0):
    """The CPU oracle on the serving stream: the full index, the stream's
    queries in arrival order, in chunks until budget_s seconds, one pinned
    core."""
    import numpy as np

    from oracle.skiplist import SkipList
    from paper_1601_00159_amd.workloads import Batch

    order = np.argsort(w.load_keys, kind="stable")
    orc = SkipList()
    orc.bulk_load_sorted(w.load_keys[order], w.load_vals[order])
    m = min(w.keys.size, 1 << 22)
    with OneCore() as pin:
        done, elapsed = oracle_rate(orc, Batch(w.ops[:m], w.keys[:m], w.vals[:m]), m, budget_s, 1 << 16)
    orc.close()
    return {"value": round(done / elapsed / 1e6, 4), "unit": "Mqueries/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {done} queries of the stream (90/5/5 S/I/D, Zipf 0.8) against the full "
                      f"{w.load_keys.size}-key index (single-threaded Pugh skip list pinned to core {pin.core}, "
                      f"{elapsed:.1f}s timed inside the oracle; host CPU {cpu_model()})"}


def serve_bytes(w, lds_from):
    """Algorithmic bytes of the whole stream: the whole-batch model of the
    read path on a sample of up to 2^22 of its queries (index as loaded),
    scaled to the stream, plus the inserted values read (8 B per query),
    per insert a new node and its predecessor's link (26 B), per delete a
    flag write (1 B)."""
    import numpy as np

    from paper_1601_00159_amd import bytemodel

    m = min(w.keys.size, 1 << 22)
    bm = bytemodel.descent_bytes(np.sort(w.load_keys), np.sort(w.keys[:m]), lds_from=lds_from)
    per_q = bytemodel.batch_bytes(bm, m) / m + 8
    return per_q * w.keys.size + int((w.ops == 1).sum()) * 26 + int((w.ops == 2).sum())


def run_serve(args):
    """Serving loop (--workload serve): 2^25 loaded keys, open-loop Poisson
    arrivals at each rate of --rates for --serve-ms of arrivals, 90/5/5
    S/I/D with Zipf 0.8 keys.  Continuous batching (100 us deadline) with 1,
    2 and 4 micro-batches in flight, each after a warm-up of SEARCH
    batches.  The rate "sat" is saturation: --sat-queries queries that have
    all arrived at time 0, served in micro-batches of up to 2^22 back to back
    (the serving form's ceiling, beside the plain launch of 2^22-query
    batches of the same stream).  One JSON line per rate and mode."""
    import numpy as np
    import torch

    from paper_1601_00159_amd import workloads as W
    from paper_1601_00159_amd.index import Index, to_device_u64, to_device_u8

    for rate_s in args.rates.split(","):
        sat = rate_s == "sat"
        rate = 1e9 if sat else float(rate_s)
        n = args.sat_queries if sat else int(rate * args.serve_ms / 1e3)
        t0 = time.perf_counter()
        w = W.serving(args.load_log2 if args.load_log2 != 26 else 25, rate, n)
        if sat:
            w.arrival_us = np.zeros(n, dtype=np.float64)
            w.name = f"serve-2^{25 if args.load_log2 == 26 else args.load_log2}-saturation"
        log(f"workload {w.name}: {w.note}; generated in {time.perf_counter() - t0:.1f}s")
        if sat:
            # the plain launch of the same stream in 2^22-query batches
            with Index(device=0, lds_budget=args.lds_budget) as ix:
                ix.bulk_load(w.load_keys, w.load_vals)
                m = 1 << 22
                for b in range(0, min(n, 2 * m), m):  # warm-up on SEARCH batches
                    ix.execute(np.zeros(min(m, n - b), dtype=np.uint8), w.keys[b:b + m], w.vals[b:b + m])
                dev_b = [(to_device_u8(w.ops[b:b + m]), to_device_u64(w.keys[b:b + m]), to_device_u64(w.vals[b:b + m]),
                          torch.empty(min(m, n - b), dtype=torch.int64, device="cuda"),
                          torch.empty(min(m, n - b), dtype=torch.uint8, device="cuda")) for b in range(0, n, m)]
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for o, k, v, ov, os_ in dev_b:
                    ix.execute_raw(o, k, v, ov, os_)
                torch.cuda.synchronize()
                plain_s = time.perf_counter() - t1
            log(f"plain launch of the same stream: {n / plain_s / 1e6:.1f} Mq/s ({len(dev_b)} batches)")
        cpu = None if args.no_cpu_baseline else serve_cpu_baseline(w)
        sbytes = None
        modes = (("continuous", 0.0, 1), ("continuous", 0.0, 2), ("continuous", 0.0, 4)) if sat else \
            (("continuous", 100.0, 1), ("continuous", 100.0, 2), ("continuous", 100.0, 4))
        for mode, deadline, inflight in modes:
            with Index(device=0, lds_budget=args.lds_budget) as ix:
                ix.bulk_load(w.load_keys, w.load_vals)
                # warm-up outside the measurement: SEARCH batches of every
                # size class load the kernels and size the workspaces
                for m in (1 << 10, 1 << 16, 1 << 22):
                    m = min(m, n)
                    ix.execute(np.zeros(m, dtype=np.uint8), w.keys[:m], w.vals[:m])
                if inflight > 1:
                    # the buffer sets of overlapped micro-batches, as a server
                    # that has been running has them
                    m = min(n, 2 << 22)
                    ix.serve(np.zeros(m), np.zeros(m, dtype=np.uint8), w.keys[:m], w.vals[:m], deadline_us=0.0,
                             max_batch=1 << 22, max_inflight=inflight)
                torch.cuda.synchronize()
                gv, gs, done, ends = ix.serve(w.arrival_us, w.ops, w.keys, w.vals, deadline_us=deadline,
                                              max_inflight=inflight)
                torch.cuda.synchronize()
                st = ix.stats()
            if sbytes is None and not args.no_bytemodel:
                sbytes = serve_bytes(w, st["lds_from"])
            lat = done - w.arrival_us
            starts = np.concatenate([[0], ends[:-1]])
            blat = done[ends - 1] - w.arrival_us[starts]
            span_s = (done.max() - w.arrival_us[0]) / 1e6
            roof = None
            if sbytes is not None:
                ach = sbytes / span_s / 1e9
                roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                        "scope": "whole stream over the served span (first arrival to last answer)",
                        "algorithmic_bytes": int(sbytes), "bytes_per_query": round(sbytes / n, 2),
                        "note": "descent lines counted on the index as loaded"}
            print(json.dumps({
                "metric": "Mqueries/s served (open-loop arrivals) at p99 latency", "value": round(n / span_s / 1e6, 2),
                "unit": "Mqueries/s", "n_gpus": 1, "steps": int(ends.size), "warmup": 0,
                "ms_per_step": round(span_s * 1e3 / max(ends.size, 1), 4), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
                "config": {"workload": w.name, "loaded_keys": int(w.load_keys.size), "queries": n,
                           "offered_Mqps": "saturation" if sat else rate / 1e6, "op_mix": "90/5/5 S/I/D",
                           "key_distribution": "zipf 0.8", "mode": mode, "deadline_us": deadline,
                           "max_inflight": inflight, "lds_budget": args.lds_budget, "parallelism": "single GPU"},
                "latency_us": {"query_p50": round(float(np.percentile(lat, 50)), 1),
                               "query_p99": round(float(np.percentile(lat, 99)), 1),
                               "batch_p50": round(float(np.percentile(blat, 50)), 1),
                               "batch_p99": round(float(np.percentile(blat, 99)), 1)},
                "micro_batches": int(ends.size), "mean_batch": round(n / max(ends.size, 1), 1),
                "plain_launch_Mqps": round(n / plain_s / 1e6, 2) if sat else None,
                "rebuilds": st["repairs"], "roofline": roof, "cpu_baseline": cpu}), flush=True)


def run_many(args):
    """Many indices (--workload many): --indices independent indices, sizes
    log-uniform in [2^10, 2^22] keys, per-index batches log-uniform in
    [2^8, 2^18] queries, 90/5/5 S/I/D.  One round = one batch on every index.
    Per-index launches (pi_execute_batch one index after another) beside the
    group launch (autotuned fused threshold).  One JSON line per mode."""
    import numpy as np
    import torch

    from paper_1601_00159_amd import workloads as W
    from paper_1601_00159_amd.index import Group, Index, to_device_u64, to_device_u8

    dev = torch.device("cuda", 0)
    rounds = args.steps + args.warmup + 1  # one more round feeds the autotuner
    t0 = time.perf_counter()
    w = W.many_indices(n_indices=args.indices, n_rounds=rounds)
    log(f"workload {w.name}: {w.note}; generated in {time.perf_counter() - t0:.1f}s")
    total_keys = sum(k.size for k, _ in w.loads)
    dev_rounds = []
    for batches in w.rounds:
        dev_rounds.append([(to_device_u8(b.ops, dev), to_device_u64(b.keys, dev), to_device_u64(b.vals, dev),
                            torch.empty(len(b), dtype=torch.int64, device=dev),
                            torch.empty(len(b), dtype=torch.uint8, device=dev)) for b in batches])
    q_per_round = [sum(len(b) for b in batches) for batches in w.rounds]
    for mode in args.many_modes.split(","):
        ixs = [Index(device=0, rebuild_policy=args.many_policy, post_form=args.many_post_form,
                     order_bits=args.order_bits) for _ in w.loads]
        for ix, (k, v) in zip(ixs, w.loads):
            ix.bulk_load(k, v)
        torch.cuda.synchronize()
        threads = 1 if mode == "group-1-thread" else 0
        g = Group(host_threads=threads) if mode.startswith("group") else None
        fused = None
        shape = None
        if g is not None and args.many_fused_max:
            g.close()
            g = Group(fused_max=args.many_fused_max, host_threads=threads)
            fused = args.many_fused_max
            log(f"fused_max fixed at {fused} (no autotuning)")
        elif g is not None:
            fused = g.autotune(ixs, dev_rounds[-1])
            _, tb, tl = g.tuning()
            shape = {"block": tb, "lds_budget": tl}
            log(f"autotuner picked fused_max={fused}, descent block {tb}, LDS budget {tl}")

        def one_round(r):
            if g is not None:
                g.execute(ixs, dev_rounds[r])
            else:
                for ix, b in zip(ixs, dev_rounds[r]):
                    ix.execute_raw(*b)

        for r in range(args.warmup):
            one_round(r)
        torch.cuda.synchronize()
        lat = []
        t_all = time.perf_counter()
        for r in range(args.warmup, args.warmup + args.steps):
            t1 = time.perf_counter()
            m0 = time.monotonic_ns()
            one_round(r)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
            log(f"{mode} round {r}: monotonic_ns {m0} {time.monotonic_ns()}")
        tot = time.perf_counter() - t_all
        nq = sum(q_per_round[args.warmup:args.warmup + args.steps])
        if g is not None:
            g.close()
        for ix in ixs:
            ix.close()
        print(json.dumps({
            "metric": "Mqueries/s over many indices (one batch per index per round)",
            "value": round(nq / tot / 1e6, 2), "unit": "Mqueries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(tot / args.steps * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": w.name, "indices": args.indices, "total_keys": int(total_keys),
                       "queries_per_round": int(np.mean(q_per_round)), "op_mix": "90/5/5 S/I/D", "mode": mode,
                       "fused_max": fused, "rebuild_policy": args.many_policy,
                       "host_threads": (threads or 4) if g is not None else 1,
                       "descent_shape": shape,
                       "parallelism": "single GPU"},
            "latency_ms": {"round_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                           "round_p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
            "roofline": None, "cpu_baseline": None}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 32; 4 rounds for --workload many)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 3; 10 rounds for --workload many, whose per-index batch sizes "
                         "change every round and reach steady-state buffer sizes after several rounds)")
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--load-log2", type=int, default=26)
    ap.add_argument("--batch-log2", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bytemodel", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle replay of --workload write")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--queries-per-lane", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--lds-budget", type=int, default=0)
    ap.add_argument("--descent-block", type=int, default=0)
    ap.add_argument("--order-bits", type=int, default=0, choices=[0, 16, 24, 32],
                    help="width of the ordering's range position (0 = chosen per batch)")
    ap.add_argument("--workload", choices=["search", "range", "write", "serve", "many"], default="search",
                    help="search: the 64M-key SEARCH batches (default); range: range searches; "
                         "write: write-heavy Zipf batches; serve: continuous batching of Poisson arrivals; "
                         "many: one batch on each of many indices per round")
    ap.add_argument("--indices", type=int, default=512, help="indices (--workload many)")
    ap.add_argument("--many-modes", default="per-index,group",
                    help="comma list of per-index, group (4 host threads), group-1-thread (--workload many)")
    ap.add_argument("--many-post-form", type=int, default=0, choices=[0, 1, 2],
                    help="post-descent form of the indices: 0 chosen, 1 one launch, 2 separate (--workload many)")
    ap.add_argument("--many-fused-max", type=int, default=0,
                    help="fused threshold of the group launch (0 = autotuned) (--workload many)")
    ap.add_argument("--many-policy", default="threshold", choices=["threshold", "never", "slices"],
                    help="rebuild policy of the indices (--workload many)")
    ap.add_argument("--rebuild-policy", default="background", choices=["threshold", "background", "never"],
                    help="rebuild policy (--workload write)")
    ap.add_argument("--rates", default="50e6,200e6,500e6", help="offered queries/s (--workload serve)")
    ap.add_argument("--serve-ms", type=float, default=20.0, help="ms of arrivals per rate (--workload serve)")
    ap.add_argument("--sat-queries", type=int, default=1 << 25, help="queries of the saturation run (--workload serve)")
    ap.add_argument("--ranges", type=int, default=8192, help="range queries per batch (--workload range)")
    ap.add_argument("--granularity", default="1,10,100,1000", help="mean keys per range (--workload range)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 4 if args.workload == "many" else 32
    if args.warmup is None:
        args.warmup = 10 if args.workload == "many" else 3
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the index shards by key range "
              "across GPUs, which this build does not run.", file=sys.stderr)
        sys.exit(2)
    if args.workload != "search":
        import torch
        assert torch.cuda.is_available(), "bench needs a GPU"
        return {"range": run_range, "write": run_write, "serve": run_serve, "many": run_many}[args.workload](args)

    import numpy as np
    import torch

    from paper_1601_00159_amd import bytemodel
    from paper_1601_00159_amd import workloads as W
    from paper_1601_00159_amd.index import Index, to_device_u64, to_device_u8

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda", 0)
    K, WU = args.steps, args.warmup
    t0 = time.perf_counter()
    w = W.headline(args.theta, args.load_log2, args.batch_log2, n_batches=K + WU)
    log(f"workload {w.name}: {w.note}; generated in {time.perf_counter() - t0:.1f}s")
    Q = 1 << args.batch_log2

    d_ops = [to_device_u8(b.ops, dev) for b in w.batches]
    d_keys = [to_device_u64(b.keys, dev) for b in w.batches]
    d_vals = [to_device_u64(b.vals, dev) for b in w.batches]
    out_v = torch.empty(Q, dtype=torch.int64, device=dev)
    out_s = torch.empty(Q, dtype=torch.uint8, device=dev)

    if args.calibrate_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the counters read for the index kernels
        nb = args.calibrate_copy_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty(nb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.calibrate_copy_mib} MiB done")

    ix = Index(device=0, profile=1, queries_per_lane=args.queries_per_lane, blocks_per_cu=args.blocks_per_cu,
               lds_budget=args.lds_budget, descent_block=args.descent_block, order_bits=args.order_bits)
    t0 = time.perf_counter()
    ix.bulk_load(w.load_keys, w.load_vals)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    st = ix.stats()
    log(f"bulk load of {st['live_nodes']} keys: {load_s:.2f}s; levels 2..{st['n_levels']}, LDS from {st['lds_from']}")

    for i in range(WU):
        ix.execute_raw(d_ops[i], d_keys[i], d_vals[i], out_v, out_s)
    torch.cuda.synchronize()
    ix.profile(reset=True)

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for i in range(K):
        j = WU + i
        evs[i][0].record()
        ix.execute_raw(d_ops[j], d_keys[j], d_vals[j], out_v, out_s)
        evs[i][1].record()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    prof = ix.profile(reset=True)
    log(f"timed {K} batches: {total_ms:.2f} ms on the GPU clock, {wall * 1e3:.2f} ms wall")

    # answers of the last timed batch against the loaded map (cheap check)
    last = w.batches[WU + K - 1]
    sorted_keys = np.sort(w.load_keys)
    pos = np.searchsorted(sorted_keys, last.keys)
    hit_ok = bool((out_s.cpu().numpy() == 1).all())
    ord_ = np.argsort(w.load_keys, kind="stable")
    want_v = w.load_vals[ord_][pos]
    val_ok = bool(np.array_equal(out_v.cpu().numpy().view(np.uint64), want_v))
    log(f"last batch answers: all present={hit_ok}, values match={val_ok}")

    value = K * Q / (total_ms / 1e3) / 1e6
    desc_ms = prof["descend_ms"] / max(prof["batches"], 1)
    roof = None
    roof_batch = None
    if not args.no_bytemodel:
        t0 = time.perf_counter()
        bm = bytemodel.descent_bytes(sorted_keys, np.sort(w.batches[WU].keys), lds_from=st["lds_from"])
        log(f"byte model: {bm['per_query']:.1f} B/query ({time.perf_counter() - t0:.1f}s)")
        achieved = bm["bytes"] / (desc_ms / 1e3) / 1e9
        traffic = load_traffic(w.name)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_descend", "kernel_ms": round(desc_ms, 4),
                "algorithmic_bytes_per_launch": bm["bytes"], "bytes_per_query": round(bm["per_query"], 2)}
        # the whole batch (ordering, descent, answers) against the batch time
        bb = bytemodel.batch_bytes(bm, Q)
        batch_ach = bb / (total_ms / K / 1e3) / 1e9
        roof_batch = {"bound": "hbm", "achieved": round(batch_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(batch_ach / HBM_PEAK_GBS, 4), "scope": "whole batch (ms_per_step)",
                      "algorithmic_bytes_per_batch": bb, "bytes_per_query": round(bb / Q, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, sample_queries=Q)

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mqueries/s", "n_gpus": 1, "steps": K,
        "warmup": WU, "ms_per_step": round(total_ms / K, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w.name, "loaded_keys": int(w.load_keys.size), "batch_queries": Q,
                   "op_mix": "100% SEARCH", "key_distribution": f"zipf {args.theta}" if args.theta else "uniform",
                   "ordering": (f"{args.order_bits}-bit range position" if args.order_bits else
                                "range position of 16 bits after a batch without updates, else 24 (32 above 2^20 queries)"),
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms_per_batch": {k: round(prof[k] / max(prof["batches"], 1), 4)
                                for k in ("sort_ms", "descend_ms", "own_ms", "link_ms")},
        "correct_last_batch": hit_ok and val_ok,
        "roofline": roof,
        "roofline_batch": roof_batch,
        "cpu_baseline": cpu,
    }
    ix.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
