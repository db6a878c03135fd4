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
}

KERNEL_SOURCES = ["paper_1704_02272_amd/csrc/kernels_scan.hip",
                  "paper_1704_02272_amd/csrc/kernels_plain.hip"]


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        p = os.path.join(ROOT, rel)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
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
            "dna_4": W.dna_4}[name]()


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
    return {"value": round(gbit, 3), "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "sample": "whole %s text (%d bytes) x %d scans, %.1f s, textbook Aho-Corasick "
                      "with OpenMP chunks" % (w.name, n, reps, t_total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="printable_256", choices=sorted(WORKLOADS))
    ap.add_argument("--algo", default="auto", choices=["auto", "plain", "tiled"])
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="scan", choices=["scan", "copy"],
                    help="copy: a plain device-to-device copy of the workload's text, the "
                         "reference that scales the HBM byte counters of the scan")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1704_02272_amd.pfac as pfac

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = make_workload(args.workload)
    n = len(w.text)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    info = pfac.pfac_table_info(a)
    if args.algo != "auto":
        pfac.pfac_set_tuning(a, algo=args.algo)
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
    keys = torch.empty(max(count, 1), dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        pfac.pfac_scan_async(a, texts[i % len(texts)], keys, cnt, stream)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        pfac.pfac_scan_async(a, texts[i % len(texts)], keys, cnt, stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(cnt.item()) != count:
        raise RuntimeError("match count changed between runs: %d vs %d" % (int(cnt.item()), count))
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = wall * 1e3 / args.steps
    gbit = 8.0 * n / (ms_step / 1e3) / 1e9
    avg_kern_s = float(np.mean(kern_ms)) / 1e3
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
                   "matches": count, "algo": algo, "text_copies_rotated": len(texts),
                   "trie_nodes": info["n_nodes"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel_ms_mean": round(float(np.mean(kern_ms)), 4),
                     "kernel_ms_median": round(float(np.median(kern_ms)), 4),
                     "algorithmic_bytes_per_launch": int(alg_bytes)},
        "hbm_frac_of_peak": round(achieved / HBM_PEAK_GBS, 4),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
