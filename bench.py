"""Throughput benchmark of the failure-less Aho-Corasick scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload printable_256]

A step is one scan of a device-resident text: every start position walks the trie, the
matches are compacted and written as sorted 64-bit keys, and the match count lands in
device memory. Inputs are in HBM before timing starts; four copies of the text are
rotated so the 256 MiB input cannot sit in the 256 MB Infinity Cache between steps.

Prints ONE JSON line: Gbit/s scanned (value), the roofline of the scan kernel (HBM
bound: algorithmic bytes = text bytes + 8 bytes per match written, over the kernel's
average duration from HIP events on the stream it runs on), and the CPU oracle
(textbook Aho-Corasick, OpenMP) timed on this host's cores as a baseline.
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

HBM_PEAK_GBS = 8000.0
METRIC = "Gbit/s scanned + % HBM peak (1 GPU); p99 packet latency in serving loop"

WORKLOADS = {
    "printable_256": ("256 MiB text (90% printable), 5,000 patterns (log-normal length, "
                      "median 12, 4-64), alphabet 256, one plant per 64 KiB"),
    "uniform_256": "1 MiB uniform text, 100 patterns (4-16 bytes), alphabet 256, 1,000 plants",
    "dna_4": ("1 GiB order-2 Markov DNA text (codes 0-3), 10,000 patterns (8-32), "
              "alphabet 4, one plant per MiB"),
    "serving_256": ("open-loop Poisson requests at 40 Gbit/s offered for 2 s, 32 packets per "
                    "request (64/512/1500/9000 B uniform, random bytes), 50,000 patterns "
                    "(log-normal, median 16, 4-256), alphabet 256"),
    "packets_256": ("65,536 packets (64/576/1500 B at 40/20/40 %, 80 % printable), 20,000 "
                    "patterns (4-128 B, heads from a depth-6 branching-3 tree), alphabet 256"),
}

KERNEL_SOURCES = ["paper_1704_02272_amd/csrc/scan_kernels.h",
                  "paper_1704_02272_amd/csrc/kernels_scan.hip",
                  "paper_1704_02272_amd/csrc/kernels_plain.hip",
                  "paper_1704_02272_amd/csrc/scan_internal.h",
                  "paper_1704_02272_amd/csrc/pfac_impl.h"]


def source_digest() -> str:
    """Digest of the kernel sources' code: comments (from // to the end of a line) and
    blank lines are left out, so a comment edit does not count as a kernel change."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        p = os.path.join(ROOT, rel)
        if not os.path.exists(p):
            continue
        for line in open(p, encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(workload: str, algo: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the kernel sources as they are now (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (algo, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_workload(name: str):
    from paper_1704_02272_amd import workloads as W
    return {"printable_256": W.printable_256, "uniform_256": W.uniform_256,
            "dna_4": W.dna_4, "packets_256": W.packets_256}[name]()


def cpu_baseline(w, budget_s: float):
    """Oracle (textbook Aho-Corasick, all host threads) on the same text, repeated until
    about ``budget_s`` seconds of work; returns Gbit/s and what was run."""
    from oracle import native
    ac = native.AhoCorasick(w.patterns, w.alphabet)
    threads = native.threads()
    n = len(w.text)
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 100:
        t0 = time.perf_counter()
        ac.scan(w.text, threads=threads)
        t_total += time.perf_counter() - t0
        reps += 1
    gbit = 8.0 * n * reps / t_total / 1e9
    # one thread on a leading slice of the same text (about a second of work)
    n1 = min(n, 1 << 26)
    t0 = time.perf_counter()
    ac.scan(w.text[:n1], threads=1)
    t1 = time.perf_counter() - t0
    return {"value": round(gbit, 3), "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "one_thread": {"value": round(8.0 * n1 / t1 / 1e9, 3), "unit": "Gbit/s",
                           "sample": "first %d bytes of the text, one scan" % n1},
            "sample": "whole %s text (%d bytes) x %d scans, %.1f s, textbook Aho-Corasick "
                      "with OpenMP chunks" % (w.name, n, reps, t_total)}


def cpu_model() -> str:
    """The host CPU's model name (as /proc/cpuinfo states it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_launch(args, w):
    """Eager launch pairs against replays of one captured graph of the same packet batch:
    groups of --steps launches on one stream, alternating, each timed for the host's
    enqueue (no synchronization inside the group) and in all (up to the synchronization
    after it). Under a kernel trace the groups show where a replay's extra time goes."""
    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac

    dev = torch.device("cuda:0")
    n = int(w.offsets[-1])
    a = pfac.pfac_build(w.patterns, w.alphabet)
    pfac.pfac_set_tuning(a, span_log2=12, root_depth=1, filter_k=4)
    d = torch.from_numpy(w.data).to(dev)
    offs = torch.from_numpy(w.offsets.view(np.int64)).to(dev)
    count = int(pfac.pfac_scan_batch(a, d, offs).numel())
    keys = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream()
    sizes = torch.tensor([n, w.n_packets], dtype=torch.int64, device=dev)
    g = pfac.pfac_graph_create(a, d, offs, keys, cnt, sizes, stream)
    launch = {"eager": lambda: pfac.pfac_scan_batch_async(a, d, offs, keys, cnt, stream),
              "graph": lambda: g.launch(stream)}
    res = {"eager": [], "graph": []}
    with torch.cuda.stream(stream):
        for _ in range(3):
            for mode in ("eager", "graph"):
                for _ in range(args.warmup):
                    launch[mode]()
                stream.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    launch[mode]()
                t1 = time.perf_counter()
                stream.synchronize()
                t2 = time.perf_counter()
                if int(cnt.item()) != count:
                    raise RuntimeError("match count changed: %d vs %d" % (int(cnt.item()), count))
                res[mode].append({"enqueue_us": round((t1 - t0) / args.steps * 1e6, 2),
                                  "total_us": round((t2 - t0) / args.steps * 1e6, 2)})
                time.sleep(0.01)  # a visible gap between the groups in a trace
    g.close()
    print(json.dumps({"mode": "launch", "workload": "packets_256", "bytes": n, "packets": w.n_packets,
                      "matches": count, "launches_per_group": args.steps, **res}), flush=True)


def bench_packets(args, w):
    """Packet batch: one persistent launch pair per batch (eager, and replayed from a
    captured graph) against one plain launch per packet, all on one stream."""
    import ctypes as C

    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac

    dev = torch.device("cuda:0")
    n = int(w.offsets[-1])
    a = pfac.pfac_build(w.patterns, w.alphabet)
    data = [torch.from_numpy(w.data).to(dev) for _ in range(max(1, args.copies))]
    offs = torch.from_numpy(w.offsets.view(np.int64)).to(dev)
    tuning = None
    if not args.no_tune:
        tuning = pfac.pfac_tune(a, data[0], offs, reps=5)
    first = pfac.pfac_scan_batch(a, data[0], offs)
    count = int(first.numel())
    keys = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream()
    sizes = torch.tensor([n, w.n_packets], dtype=torch.int64, device=dev)

    def timed(fn):
        with torch.cuda.stream(stream):
            for i in range(args.warmup):
                fn(i)
            stream.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
            t0 = time.perf_counter()
            for i in range(args.steps):
                ev[i][0].record(stream)
                fn(i)
                ev[i][1].record(stream)
            stream.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
        if int(cnt.item()) != count:
            raise RuntimeError("match count changed: %d vs %d" % (int(cnt.item()), count))
        return wall * 1e3, [s.elapsed_time(e) for s, e in ev]

    eager_ms, eager_ev = timed(lambda i: pfac.pfac_scan_batch_async(a, data[i % len(data)], offs, keys, cnt,
                                                                     stream))
    graphs = [pfac.pfac_graph_create(a, d, offs, keys, cnt, sizes, stream) for d in data]
    graph_ms, graph_ev = timed(lambda i: graphs[i % len(graphs)].launch(stream))

    # baseline: one plain scan (count, offsets, emit launches) per packet, on one stream
    base = pfac.pfac_build(w.patterns, w.alphabet)
    pfac.pfac_set_tuning(base, algo="plain")
    slot = 16
    bkeys = torch.empty(w.n_packets * slot, dtype=torch.int64, device=dev)
    bcnt = torch.zeros(w.n_packets, dtype=torch.int64, device=dev)
    L = pfac.lib()
    h = C.c_void_p(base.handle)
    sh = C.c_void_p(stream.cuda_stream)
    d0, k0, c0 = data[0].data_ptr(), bkeys.data_ptr(), bcnt.data_ptr()
    lo = [int(x) for x in w.offsets]

    def per_packet():
        for i in range(w.n_packets):
            rc = L.pfac_scan_async(h, C.c_void_p(d0 + lo[i]), lo[i + 1] - lo[i], C.c_void_p(k0 + 8 * slot * i),
                                   slot, C.c_void_p(c0 + 8 * i), sh)
            if rc:
                raise pfac.PfacError(rc, "pfac_scan_async")

    base_steps = max(1, min(args.steps, args.baseline_steps))
    with torch.cuda.stream(stream):
        per_packet()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(base_steps):
            per_packet()
        stream.synchronize()
        base_ms = (time.perf_counter() - t0) * 1e3 / base_steps
    if int(bcnt.sum().item()) != count:
        raise RuntimeError("per-packet scans disagree with the batch: %d vs %d"
                           % (int(bcnt.sum().item()), count))
    gbit = 8.0 * n / (graph_ms / 1e3) / 1e9
    kern_s = float(np.mean(graph_ev)) / 1e3
    alg_bytes = n + 8.0 * (w.n_packets + 1) + 8.0 * count
    achieved = alg_bytes / kern_s / 1e9
    out = {
        "metric": METRIC, "value": round(gbit, 2), "unit": "Gbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded numpy generator; see DESIGN.md input recipe)",
        "config": {"workload": "packets_256", "description": WORKLOADS["packets_256"],
                   "packets": w.n_packets, "bytes": n, "patterns": len(w.patterns),
                   "matches": count, "tuning": tuning, "text_copies_rotated": len(data)},
        "batch": {"graph_ms": round(graph_ms, 4), "eager_ms": round(eager_ms, 4),
                  "graph_event_ms_mean": round(float(np.mean(graph_ev)), 4),
                  "eager_event_ms_mean": round(float(np.mean(eager_ev)), 4),
                  "per_packet_plain_ms": round(base_ms, 3), "per_packet_steps": base_steps,
                  "speedup_graph_vs_per_packet": round(base_ms / graph_ms, 1),
                  "per_packet_gbit_s": round(8.0 * n / (base_ms / 1e3) / 1e9, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("packets_256", "tiled"),
                     "kernel_ms_mean": round(kern_s * 1e3, 4),
                     "algorithmic_bytes_per_launch": int(alg_bytes)},
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import native
        ac = native.AhoCorasick(w.patterns, w.alphabet)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < args.cpu_budget and reps < 50:
            ac.scan_packets(w.data, w.offsets)
            reps += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(8.0 * n * reps / el / 1e9, 3), "unit": "Gbit/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "whole batch x %d, %.1f s, textbook Aho-Corasick per packet, "
                                         "one thread" % (reps, el)}
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Serving loop under an open-loop Poisson stream: requests are submitted at their
    scheduled arrival times (latency counts from the schedule, so a late client shows as
    latency), results are drained by a second thread, and the server's own statistics
    give per-packet p50/p99 latency and the achieved rate."""
    import threading

    import numpy as np

    import paper_1704_02272_amd.pfac as pfac
    from paper_1704_02272_amd import workloads as W

    w = W.serving_256(duration_s=args.serve_seconds, contiguous=True, plant_every=args.plant_every)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    srv = pfac.pfac_server_create(a, slots=args.slots, max_batch_bytes=args.batch_mib << 20,
                                  flags=0 if args.graph else pfac.PFAC_SERVER_EAGER)
    cfg = srv.config()
    ptrs = [(r.data.ctypes.data, r.offsets.ctypes.data, int(r.offsets[-1])) for r in w.requests]
    arr_ns = [int(r.arrival_s * 1e9) for r in w.requests]
    # warm-up: a few requests through every slot
    for i in range(min(64, len(ptrs))):
        srv.submit_raw(ptrs[i][0], ptrs[i][1], w.packets_per_request)
    seen = 0
    while seen < min(64, len(ptrs)):
        seen += len(srv.poll(timeout_us=100000, with_keys=False))
    srv.stats(reset=True)
    done = {"n": 0, "matches": 0, "bad": 0}
    n_total = len(ptrs)
    stop = threading.Event()
    # a sample of requests, evenly spread over the stream, whose keys are kept and
    # checked against the oracle after the run
    n_verify = min(args.verify, n_total)
    verify_idx = set(np.linspace(0, n_total - 1, n_verify).astype(int).tolist()) if n_verify else set()
    ticket_of = {}
    got_keys = {}
    # keys are copied out only for the sampled requests: a ticket is added to
    # verify_tickets before the registered bound moves past it, and any ticket above the
    # bound (a result that beat its own registration) is kept too
    verify_tickets = set()
    registered = {"max": 0}
    # per request: queueing (launch - arrival), service (done - launch), total; filled in
    # place so the drain thread allocates nothing per result
    phases = np.zeros((n_total, 3), dtype=np.float64)

    def want(t):
        return t in verify_tickets or t > registered["max"]

    def drain():
        while done["n"] < n_total and not stop.is_set():
            for r in srv.poll(timeout_us=50000, with_keys=bool(verify_idx), keys_for=want):
                k = done["n"]
                if k < n_total:
                    phases[k, 0] = r["launch_ns"] - r["arrival_ns"]
                    phases[k, 1] = r["done_ns"] - r["launch_ns"]
                    phases[k, 2] = r["done_ns"] - r["arrival_ns"]
                done["n"] += 1
                done["matches"] += r["n_matches"]
                done["bad"] += r["status"] != 0
                if r["keys"] is not None:
                    got_keys[r["ticket"]] = r["keys"]

    # no garbage collection pauses in the client while the stream runs (a pause delays
    # submissions, which the latency, counted from the schedule, would show)
    import gc
    gc.collect()
    gc.disable()
    th = threading.Thread(target=drain, daemon=True)
    th.start()
    t0 = time.monotonic_ns() + 20_000_000
    busy = 0
    i = 0
    while i < n_total:
        now = time.monotonic_ns()
        while i < n_total and t0 + arr_ns[i] <= now:
            rc = srv.submit_raw(ptrs[i][0], ptrs[i][1], w.packets_per_request, t0 + arr_ns[i])
            if rc == pfac.PFAC_EBUSY:
                busy += 1
            elif rc:
                raise pfac.PfacError(rc, "pfac_server_submit")
            else:
                if i in verify_idx:
                    ticket_of[srv.last] = i
                    verify_tickets.add(srv.last)
                registered["max"] = srv.last
            i += 1
        if i < n_total:
            wait = (t0 + arr_ns[i] - time.monotonic_ns()) / 1e9
            if wait > 2e-4:
                time.sleep(wait - 1e-4)
    th.join(timeout=120)
    stop.set()
    gc.enable()
    st = srv.stats()
    srv.close()
    offered = 8.0 * sum(p[2] for p in ptrs) / (arr_ns[-1] / 1e9) / 1e9
    # every request has the same number of packets, so per-request percentiles are the
    # per-packet ones
    ph = phases[: min(done["n"], n_total)] / 1e3
    pct = (lambda col, q: round(float(np.percentile(ph[:, col], q)), 1) if len(ph) else None)
    mism = None
    if verify_idx:
        from oracle import native
        ac = native.AhoCorasick(w.patterns, w.alphabet)
        kept = {i: got_keys.get(t) for t, i in ticket_of.items()}
        missing = np.zeros(1, np.uint64) - np.uint64(1)
        mism = sum(not np.array_equal(kept[i] if kept.get(i) is not None else missing,
                                      ac.scan_packets(w.requests[i].data, w.requests[i].offsets))
                   for i in sorted(kept))
    out = {
        "metric": METRIC, "value": round(st["bytes_per_s"] * 8 / 1e9, 3), "unit": "Gbit/s", "n_gpus": 1,
        "steps": n_total, "warmup": 64, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded numpy generator; see DESIGN.md input recipe)",
        "config": {"workload": "serving_256", "description": WORKLOADS["serving_256"],
                   "requests": n_total, "patterns": len(w.patterns), "server": cfg,
                   "plant_every": args.plant_every, "slot_launch": "graph" if args.graph else "eager"},
        "serving": {"offered_gbit_s": round(offered, 3), "achieved_gbit_s": round(st["bytes_per_s"] * 8 / 1e9, 3),
                    "p50_us": round(st["p50_ns"] / 1e3, 1), "p99_us": round(st["p99_ns"] / 1e3, 1),
                    "max_us": round(st["max_ns"] / 1e3, 1), "requests_done": done["n"],
                    "rejected_busy": busy, "failed": done["bad"], "batches": st["batches"],
                    "mean_batch_kib": round(st["mean_batch_bytes"] / 1024, 1), "matches": done["matches"],
                    "queue_us": {"p50": pct(0, 50), "p99": pct(0, 99), "max": pct(0, 100)},
                    "service_us": {"p50": pct(1, 50), "p99": pct(1, 99), "max": pct(1, 100)},
                    "verified_requests": len(ticket_of), "verify_mismatches": mism},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def equal_length_patterns(alphabet: int, count: int, length: int, seed: int):
    """``count`` distinct random patterns of ``length`` symbols over 0..alphabet-1 (the
    synthetic pattern sets of Section 4.1)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pats = set()
    while len(pats) < count:
        block = rng.integers(0, alphabet, size=(count - len(pats), length)).astype(np.uint8)
        pats.update(row.tobytes() for row in block)
    return sorted(pats)[:count]


def bench_sizes(args):
    """Trie sizes of Section 4.1 (Figs. 4 and 5): 20-symbol random patterns at
    alphabets 4 and 52, for several pattern counts. Bitmapped trie (Section 3.1) and its
    compressed form (Section 3.2) from the library; an array trie (one 4-byte child
    pointer per symbol per node) and a binary trie (symbols as ceil(log2 alphabet)-bit
    codes, two 4-byte child pointers per node) as the textbook baselines the figures
    plot. No GPU."""
    import math

    import paper_1704_02272_amd.pfac as pfac
    rows = []
    for alphabet in (4, 52):
        bits = max(1, math.ceil(math.log2(alphabet)))
        for count in (10, 100, 1000, 10000, 100000):
            pats = equal_length_patterns(alphabet, count, 20, seed=alphabet * 1000 + count)
            info = {lv: pfac.pfac_table_info(pfac.pfac_build(pats, alphabet, merge_levels=lv)) for lv in (0, 1, 3, 255)}
            q = info[0]["n_nodes"]
            bin_prefixes = set()
            for p in pats:
                code = "".join(format(c, "0%db" % bits) for c in p)
                bin_prefixes.update(code[:i] for i in range(1, len(code) + 1))
            row = {"alphabet": alphabet, "patterns": count, "length": 20,
                   "array_trie_bytes": q * 4 * alphabet,
                   "binary_trie_bytes": (1 + len(bin_prefixes)) * 8,
                   "bitmapped_nodes": q, "bitmapped_bytes": info[0]["paper_table_bytes"]}
            for lv in (1, 3, 255):
                row["reduced%d_nodes" % lv] = info[lv]["reduced_nodes"]
                row["reduced%d_bytes" % lv] = info[lv]["reduced_paper_bytes"]
                row["reduced%d_saving" % lv] = round(1 - info[lv]["reduced_nodes"] / q, 4)
                row["device%d_records" % lv] = info[lv]["table_records"]
            row["device0_table_bytes"] = info[0]["device_table_bytes"]
            row["device3_table_bytes"] = info[3]["device_table_bytes"]
            rows.append(row)
    for alphabet in (4, 52):
        sel = [r for r in rows if r["alphabet"] == alphabet]
        for lv in (1, 3, 255):
            rows.append({"alphabet": alphabet, "mean_saving_levels_%d" % lv:
                         round(sum(r["reduced%d_saving" % lv] for r in sel) / len(sel), 4)})
    print(json.dumps({"mode": "sizes", "rows": rows}), flush=True)


def bench_prefix(args):
    """Prefix-length study (Section 4.2, Fig. 3 shape): for alphabets 4, 8, ..., 52 (and
    256), 100 random 20-symbol patterns planted once each into five seeded texts of
    uniform symbols. The library's prefix-depth histogram gives, for every prefix length
    k, how many starts a trie truncated after k levels (Section 2.4) lets through; those
    beyond the full matches are false positives. Reported per alphabet: the smallest k
    with no false positive in a file (mean over the files), the false-positive rate at
    several k, and the uniform-text estimate n * P * |Sigma|^-k of the false positives.
    The histogram of the first file of each alphabet is checked against the oracle on a
    1 MiB slice."""
    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac
    from oracle import prefix as oprefix

    dev = torch.device("cuda:0")
    n = args.sweep_mib << 20
    L, P, cap = 20, 100, 24
    rows = []
    for alphabet in list(range(4, 53, 4)) + [256]:
        pats = equal_length_patterns(alphabet, P, L, seed=alphabet * 7919 + P)
        a = pfac.pfac_build(pats, alphabet)
        kstar, fp_at = [], {k: [] for k in (3, 4, 5, 6, 8, 10, 12, 14, 16)}
        for f in range(args.sweep_files):
            rng = np.random.default_rng(20_000 + alphabet * 10 + f)
            host = rng.integers(0, alphabet, size=n, dtype=np.uint8)
            for j, p in enumerate(pats):  # each pattern once
                o = int(rng.integers(0, n - L))
                host[o:o + L] = np.frombuffer(p, np.uint8)
            text = torch.from_numpy(host).to(dev)
            h = pfac.pfac_prefix_histogram(a, text, cap).cpu().tolist()
            if f == 0:
                sl = host[: 1 << 20]
                if pfac.pfac_prefix_histogram(a, text[: 1 << 20], cap).cpu().tolist() != \
                        oprefix.depth_histogram(pats, sl, cap):
                    raise RuntimeError("prefix histogram differs from the oracle at alphabet %d" % alphabet)
            full = sum(h[L:])
            fp = [sum(h[k:]) - full for k in range(cap + 1)]
            kstar.append(next(k for k in range(1, L + 1) if fp[k] == 0))
            for k in fp_at:
                fp_at[k].append(fp[k] / n)
            del text
        rows.append({"alphabet": alphabet, "patterns": P, "length": L, "full_matches_per_file": full,
                     "k_no_false_positive_mean": round(float(np.mean(kstar)), 2),
                     "k_no_false_positive_per_file": kstar,
                     "false_positive_rate": {str(k): float("%.3g" % np.mean(v)) for k, v in fp_at.items()},
                     "uniform_estimate_fp_at_k": {str(k): float("%.3g" % (n * P * float(alphabet) ** -k))
                                                  for k in fp_at}})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"mode": "prefix", "text_mib": args.sweep_mib, "files": args.sweep_files,
                      "rows": rows}), flush=True)


def bench_sweep(args):
    """Throughput over alphabets and pattern counts (Section 4.3, Figs. 7-9 shape): for
    every alphabet in 4, 8, ..., 52 and 256 and every count in 1, 10, 100, 1,000 of
    20-symbol random patterns, scan five seeded 100 MiB texts of uniform symbols
    (Section 4: five synthetic files, 100 runs each, the mean reported) with the plain
    and the compressed (three merged levels) table. Each configuration is first checked
    against the oracle on a 4 MiB slice. Also the oracle itself (all host threads) at
    alphabet 52 with 100 patterns on 100 and 200 MiB texts (Fig. 9)."""
    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac
    from oracle import native

    dev = torch.device("cuda:0")
    n = args.sweep_mib << 20
    reps = args.steps
    alphabets = list(range(4, 53, 4)) + [256]
    counts = [1, 10, 100, 1000]
    stream = torch.cuda.current_stream()
    import ctypes
    scan_async = pfac.lib().pfac_scan_async
    rows = []
    for alphabet in alphabets:
        texts = []
        for f in range(args.sweep_files):
            rng = np.random.default_rng(10_000 + alphabet * 10 + f)
            texts.append(torch.from_numpy(rng.integers(0, alphabet, size=n, dtype=np.uint8)).to(dev))
        for count in counts:
            pats = equal_length_patterns(alphabet, count, 20, seed=alphabet * 7919 + count)
            row = {"alphabet": alphabet, "patterns": count}
            for levels in (0, 3):
                a = pfac.pfac_build(pats, alphabet, merge_levels=levels)
                sl = texts[0][: 4 << 20]
                got = pfac.keys_to_numpy(pfac.pfac_scan(a, sl))
                want = native.AhoCorasick(pats, alphabet).scan(sl.cpu().numpy())
                if not np.array_equal(got, want):
                    raise RuntimeError("sweep parity failed at alphabet %d, %d patterns, levels %d"
                                       % (alphabet, count, levels))
                keys = torch.empty(max(1 << 16, int(len(want)) * 64), dtype=torch.int64, device=dev)
                cnt = torch.zeros(1, dtype=torch.int64, device=dev)
                per_file = []
                for t in texts:
                    call = (a.handle, ctypes.c_void_p(t.data_ptr()), t.numel(), ctypes.c_void_p(keys.data_ptr()),
                            keys.numel(), ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
                    for _ in range(2):
                        scan_async(*call)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    bad = 0
                    for _ in range(reps):
                        bad |= scan_async(*call)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    if bad:
                        raise RuntimeError("pfac_scan_async failed in the sweep")
                    if int(cnt.item()) > keys.numel():
                        raise RuntimeError("sweep key buffer too small")
                    per_file.append(e0.elapsed_time(e1) / reps)
                ms = float(np.mean(per_file))
                tag = "plain" if levels == 0 else "reduced3"
                row[tag + "_gbit_s"] = round(8.0 * n / (ms / 1e3) / 1e9, 1)
                row[tag + "_ms"] = round(ms, 4)
                row[tag + "_hbm_frac"] = round(n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            row["matches_4mib_slice"] = int(len(want))
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
        del texts
    # Fig. 9: the oracle on the host at alphabet 52, 100 patterns, 100 and 200 MiB
    cpu = []
    if not args.no_cpu:
        pats = equal_length_patterns(52, 100, 20, seed=52 * 7919 + 100)
        ac = native.AhoCorasick(pats, 52)
        for mib in (100, 200):
            t = np.random.default_rng(52).integers(0, 52, size=mib << 20, dtype=np.uint8)
            t0 = time.perf_counter()
            ac.scan(t, threads=native.threads())
            el = time.perf_counter() - t0
            cpu.append({"mib": mib, "gbit_s": round(8.0 * (mib << 20) / el / 1e9, 3), "threads": native.threads()})
    print(json.dumps({"mode": "sweep", "text_mib": args.sweep_mib, "files": args.sweep_files, "reps": reps,
                      "pattern_length": 20, "rows": rows, "cpu_oracle_alphabet52_100pats": cpu,
                      "cpu_model": cpu_model()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="printable_256", choices=sorted(WORKLOADS))
    ap.add_argument("--algo", default="auto", choices=["auto", "plain", "tiled"])
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--lane-bytes", type=int, default=0, choices=[0, 16, 32],
                    help="scan: positions per thread and step (0: the library's default)")
    ap.add_argument("--span-log2", type=int, default=0,
                    help="scan: log2 of the span length, 11..16 (0: chosen from the text size)")
    ap.add_argument("--streams", type=int, default=1, help="scan: streams the scans alternate over")
    ap.add_argument("--no-pipelined", dest="pipelined", action="store_false",
                    help="scan: skip the extra two-stream measurement")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="packets: skip the autotuner")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="serving: seconds of offered load")
    ap.add_argument("--slots", type=int, default=4, help="serving: batch slots")
    ap.add_argument("--batch-mib", type=int, default=8, help="serving: MiB per batch")
    ap.add_argument("--plant-every", type=int, default=0, help="serving: planted variant")
    ap.add_argument("--graph", action="store_true",
                    help="serving: slots replay captured graphs instead of enqueueing eager launch pairs")
    ap.add_argument("--verify", type=int, default=256,
                    help="serving: requests (evenly spread) whose keys are checked against the oracle")
    ap.add_argument("--sweep-mib", type=int, default=100, help="sweep: MiB per text")
    ap.add_argument("--sweep-files", type=int, default=5, help="sweep: seeded texts per alphabet")
    ap.add_argument("--baseline-steps", type=int, default=3,
                    help="packets: timed passes of the per-packet baseline")
    ap.add_argument("--mode", default="scan", choices=["scan", "copy", "host", "sizes", "sweep", "prefix", "launch"],
                    help="copy: a plain device-to-device copy of the workload's text, the "
                         "reference that scales the HBM byte counters of the scan; host: the "
                         "text starts in host memory (pinned, then pageable) and crosses PCIe "
                         "inside the timed region; sizes: the trie-size study of Section 4.1 (no GPU); "
                         "sweep: throughput over alphabets and pattern counts (Section 4.3); "
                         "launch (packets_256): eager launch pairs against graph replays of one "
                         "batch, host enqueue time and total time per launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "sizes":
        bench_sizes(args)
        return

    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "prefix":
        bench_prefix(args)
        return
    if args.mode == "sweep":
        bench_sweep(args)
        return
    if args.workload == "serving_256":
        bench_serving(args)
        return
    w = make_workload(args.workload)
    if args.workload == "packets_256":
        if args.mode == "launch":
            bench_launch(args, w)
        else:
            bench_packets(args, w)
        return
    n = len(w.text)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    info = pfac.pfac_table_info(a)
    if args.algo != "auto" or args.lane_bytes or args.span_log2:
        pfac.pfac_set_tuning(a, algo=args.algo, lane_bytes=args.lane_bytes, span_log2=args.span_log2)
    if args.mode == "host":
        pinned = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        pinned.numpy()[:] = w.text
        res = {}
        for name, buf in (("pinned", pinned.numpy()), ("pageable", w.text)):
            pfac.pfac_scan_host(a, buf)  # warm-up: device copy, staging buffers
            times = []
            for _ in range(max(1, args.steps)):
                t0 = time.perf_counter()
                m = pfac.pfac_scan_host(a, buf)
                times.append(time.perf_counter() - t0)
            res[name] = {"ms": round(1e3 * float(np.median(times)), 3),
                         "gbit_s": round(8.0 * n / float(np.median(times)) / 1e9, 2), "matches": len(m)}
        print(json.dumps({"mode": "host", "workload": args.workload, "bytes": n, "steps": args.steps,
                          "chunk_bytes": 64 << 20, "end_to_end": res}), flush=True)
        return
    texts = [torch.from_numpy(w.text).to(dev) for _ in range(max(1, args.copies))]
    if args.mode == "copy":
        dst = torch.empty_like(texts[0])
        for i in range(args.warmup + args.steps):
            dst.copy_(texts[i % len(texts)])
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_per_copy": n, "copies": args.warmup + args.steps}))
        return
    # size the key buffer with one blocking scan
    first = pfac.pfac_scan(a, texts[0])
    count = int(first.numel())
    import ctypes
    scan_async = pfac.lib().pfac_scan_async

    def timed_scans(S):
        """K scans round-robin over S streams (each with its own key buffer and the
        library's scratch for that stream; with S > 1 one scan's placement runs beside
        the next one's count kernel, and every scan is still done inside the timed
        region). Returns (wall seconds, event milliseconds) for the K scans.

        Two HIP events on the first scan stream bracket the K back-to-back scans (a timing
        event per scan would put its own barrier between the scans); the other streams wait
        for the first event, and the first stream waits for all of them before the second.
        The C entry point is called with its arguments marshalled once, so the host keeps
        ahead of the device even on a loaded host."""
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
        keys = [torch.empty(max(count, 1), dtype=torch.int64, device=dev) for _ in range(S)]
        cnts = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(S)]
        stream = streams[0]
        for i in range(max(args.warmup, S)):
            pfac.pfac_scan_async(a, texts[i % len(texts)], keys[i % S], cnts[i % S], streams[i % S])
        torch.cuda.synchronize()
        call_args = [(a.handle, ctypes.c_void_p(texts[i % len(texts)].data_ptr()), texts[i % len(texts)].numel(),
                      ctypes.c_void_p(keys[i % S].data_ptr()), keys[i % S].numel(),
                      ctypes.c_void_p(cnts[i % S].data_ptr()), ctypes.c_void_p(streams[i % S].cuda_stream))
                     for i in range(len(texts) * S)]
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for st in streams[1:]:
            st.wait_event(ev0)
        bad = 0
        for i in range(args.steps):
            bad |= scan_async(*call_args[i % len(call_args)])
        for st in streams[1:]:
            e = torch.cuda.Event()
            e.record(st)
            stream.wait_event(e)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if bad:
            raise RuntimeError("pfac_scan_async failed in the timed loop (status bits %d)" % bad)
        for c in cnts:
            if int(c.item()) != count:
                raise RuntimeError("match count changed between runs: %d vs %d" % (int(c.item()), count))
        return wall, ev0.elapsed_time(ev1)

    S = max(1, args.streams)
    wall, ev_ms = timed_scans(S)
    kern_ms_mean = ev_ms / args.steps
    ms_step = wall * 1e3 / args.steps
    gbit = 8.0 * n / (ms_step / 1e3) / 1e9
    avg_kern_s = kern_ms_mean / 1e3
    alg_bytes = n + 8.0 * count
    achieved = alg_bytes / avg_kern_s / 1e9
    algo = pfac.pfac_get_tuning(a)["algo"]
    traffic = load_traffic(args.workload, algo)
    out = {
        "metric": METRIC,
        "value": round(gbit, 2),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded numpy generator; see DESIGN.md input recipe)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "text_bytes": n, "patterns": len(w.patterns), "alphabet": w.alphabet,
                   "matches": count, "algo": algo, "text_copies_rotated": len(texts), "streams": S,
                   "trie_nodes": info["n_nodes"], "lane_bytes": pfac.pfac_get_tuning(a)["lane_bytes"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel_ms_mean": round(kern_ms_mean, 4),
                     "algorithmic_bytes_per_launch": int(alg_bytes)},
        "hbm_frac_of_peak": round(achieved / HBM_PEAK_GBS, 4),
        "pipelined": None,
        "cpu_baseline": None,
    }
    if S == 1 and args.pipelined:
        # the same K scans alternating over two streams: the rate of a scanner that keeps
        # two buffers in flight (one scan's placement beside the next one's count kernel)
        w2, e2 = timed_scans(2)
        out["pipelined"] = {"streams": 2, "value": round(8.0 * n / (w2 / args.steps) / 1e9, 2),
                            "ms_per_step": round(w2 * 1e3 / args.steps, 4),
                            "event_ms_per_scan": round(e2 / args.steps, 4),
                            "hbm_frac": round(alg_bytes / (e2 / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
