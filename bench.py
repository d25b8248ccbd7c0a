#!/usr/bin/env python
"""Throughput of the Aho-Corasick scan on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-batch] [--no-cpu] [--no-serve]

Workload (dna_dense): 268,435,456 DNA bases, GC content 0.4, 1 % of the text
in poly-A runs of 50-500 bases; 10,000 patterns (A^8..A^16, 7,000 cut from
the text with lengths 10-30, 2,991 random from the background).  The text
sits in HBM as letters when the timed region starts.

One step runs the whole GPU path once: letters -> 2-bit packed text
(encoder), then the scan: count pass, tile offsets, work list, emit pass,
which writes every (pattern id, end position) match in (end, id) order (no
separate sort exists to run).  The dictionary is compiled once, before
timing (the paper's stage 1); its host time is reported as build_ms.

Printed: one JSON line on stdout.  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scan throughput (Gbases/s) + % HBM/LDS roofline, bit-exact; batched vs plain speedup"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
CUS, CLOCK_GHZ = 256, 2.4      # MI355X compute units, peak engine clock


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("scan.hip", "batch.inc", "internal.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_1403_7294_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, only if
    they were taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(f"{kernel}:{workload}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


# nominal LDS lookup peak: 32 banks x 4 B per clock per CU, conflict-free
LDS_LOOKUP_PEAK = 32 * CUS * CLOCK_GHZ * 1e9


def scan_roofline(n, matches, ms, text_bytes_per_base, kernel_sum_us, traffic=None):
    """The scan's place under its roofs:
    bases/s divided by min(HBM peak / HBM bytes per base, LDS lookup peak /
    one lookup per base).  HBM bytes per base are the algorithmic ones: the
    text read once plus 8 bytes per match written."""
    bpb = text_bytes_per_base + 8.0 * matches / n
    bases_s = n / (ms * 1e-3)
    hbm_roof = HBM_PEAK_GBS * 1e9 / bpb
    lds_roof = LDS_LOOKUP_PEAK
    bound = "hbm" if hbm_roof <= lds_roof else "lds"
    achieved = bases_s * bpb / 1e9
    out = {"bound": bound, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(bases_s / min(hbm_roof, lds_roof), 4), "traffic": traffic,
           "scope": "the scan: every kernel from the packed text in HBM to all matches "
                    "written, one launch sequence", "scan_us": round(ms * 1e3, 2),
           "kernel_sum_us": round(kernel_sum_us, 2),
           "bytes_per_base": round(bpb, 4), "bases_per_s": round(bases_s, 1),
           "hbm_roof_bases_per_s": round(hbm_roof, 1), "lds_roof_bases_per_s": lds_roof,
           "frac_hbm": round(bases_s / hbm_roof, 4), "frac_lds": round(bases_s / lds_roof, 4)}
    if bound == "lds":
        out.update(achieved=round(bases_s / 1e9, 2), peak=round(lds_roof / 1e9, 1),
                   unit="G lookups/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the partitioned / failure-less / two-symbol comparisons")
    ap.add_argument("--no-protein", action="store_true", help="skip the protein workload")
    ap.add_argument("--no-small", action="store_true", help="skip the dna_small graph loop")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the microbenchmarks of the HBM, LDS and gather ceilings")
    ap.add_argument("--serve-requests", type=int, default=10_000,
                    help="requests timed at the fixed arrival rate")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing)")
    ap.add_argument("--profile-leg", choices=["protein", "batch", "dna_small", "serve"],
                    default=None,
                    help="run only this workload's leg and print its JSON (for kernel traces "
                         "of one workload under rocprofv3); no benchmark line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device 5 times: the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this benchmark runs on a single MI355X "
              "(multi-GPU sharding of the scan is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1403_7294_amd as ac
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 1 << 30,
                          "bytes_written": 1 << 30, "launches": 5}), flush=True)
        return

    if args.profile_leg:
        leg = {"protein": lambda: bench_protein(args, torch, ac, W, dev, stream),
               "batch": lambda: bench_batch(args, torch, ac, W, dev, stream),
               "dna_small": lambda: bench_small_graph(args, torch, ac, W, dev, stream),
               "serve": lambda: bench_serve(args, torch, ac, W)}
        print(json.dumps({args.profile_leg: leg[args.profile_leg]()}), flush=True)
        return

    t0 = time.time()
    inst = W.dna_dense(scale=args.scale)
    n = len(inst.text)
    log(f"[bench] generated dna_dense: {n} bases, {inst.patterns.count} patterns "
        f"({time.time() - t0:.1f} s)")
    d = ac.ac_build(inst.patterns, sigma=4)
    info = d.info
    log(f"[bench] built: {info.states} states, table {info.table_bytes / 2**20:.2f} MiB, "
        f"build {info.build_ms:.1f} ms")

    letters = torch.from_numpy(W.to_ascii(inst.text, W.DNA)).to(dev)
    packed = torch.empty((n + 3) // 4, dtype=torch.uint8, device=dev)
    bad = torch.zeros(1, dtype=torch.int64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    fmt = ac.AC_TEXT_2BIT
    ws = torch.empty(ac.ac_scan_workspace_size(d, n, fmt), dtype=torch.uint8, device=dev)

    def encode():
        ac.ac_encode(letters, ac.AC_ALPHA_DNA, fmt, packed, bad)

    # size the output exactly with a counting pass (capacity 0)
    encode()
    dummy = torch.empty((1, 2), dtype=torch.int32, device=dev)
    ac.ac_scan(d, packed, n, fmt, dummy, 0, count, workspace_dev=ws)
    torch.cuda.synchronize()
    total = int(count.item())
    out = torch.empty((max(1, total), 2), dtype=torch.int32, device=dev)
    log(f"[bench] matches: {total} ({total * 8 / 2**30:.2f} GiB of output)")

    def scan():
        ac.ac_scan(d, packed, n, fmt, out, total, count, workspace_dev=ws)

    def step():
        encode()
        scan()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # per-kernel pass (not the timed steps): every kernel between HIP events
    # on its stream, for the per-kernel table and to find the dominant one
    ac.ac_timing_enable(True)
    ac.ac_timing_read(reset=True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ktimes = ac.ac_timing_read(reset=True)
    ac.ac_timing_enable(False)
    dom_name = max(("count", "emit_dense", "emit", "encode"),
                   key=lambda k: ktimes[k][0] / max(1, ktimes[k][1]))
    # the timed steps: only the dominant kernel keeps its event pair (each
    # pair adds a little time to the stream), so its duration is measured
    # live in the same region as the step
    ac.ac_timing_enable(True, kinds=[ac.KERNEL_NAMES.index(dom_name)])
    ac.ac_timing_read(reset=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    step_ms = ev0.elapsed_time(ev1) / args.steps
    live = ac.ac_timing_read(reset=True)[dom_name]
    ac.ac_timing_enable(False)
    log(f"[bench] step {step_ms:.3f} ms; {dom_name} {live[0] / max(1, live[1]) * 1e3:.1f} us "
        "live; per-kernel pass: " +
        ", ".join(f"{k} {v[0] / max(1, v[1]) * 1e3:.1f} us" for k, v in ktimes.items() if v[1]))
    assert int(bad.item()) == 0 and int(count.item()) == total

    # scan only (packed text already in HBM), untimed by the kernel timer
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        scan()
    ev1.record(stream)
    torch.cuda.synchronize()
    scan_ms = ev0.elapsed_time(ev1) / args.steps

    # --------------------------------------------------------- rooflines
    avg = {k: v[0] / v[1] for k, v in ktimes.items() if v[1]}
    # matches written by each emit kernel: segments of AC_SEGMENT symbols
    # with >= AC_DENSE_SEGMENT_MATCHES matches are the dense kernel's
    ends = out[:, 1].cpu().numpy().view(np.uint32)
    per_seg = np.bincount(ends // ac.AC_SEGMENT)
    dense_m = int(per_seg[per_seg >= ac.AC_DENSE_SEGMENT_MATCHES].sum())
    sparse_m = total - dense_m
    del ends, per_seg

    def hbm(name, nbytes, note):
        t = avg.get(name)
        if not t:
            return None
        return {"bound": "hbm", "achieved": nbytes / (t * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "algorithmic_bytes": nbytes, "avg_us": t * 1e3, "per_unit": note}

    rooflines = {
        # letters read, packed text written
        "encode": hbm("encode", n + (n + 3) // 4, "1.25 B per base"),
        # one dependent table lookup per base; from HBM only the packed text
        "count": hbm("count", (n + 3) // 4, "0.25 B per base (+1 table lookup per base)"),
        # 8 B per match written (+ 16 B of text per listed segment, ignored)
        "emit": hbm("emit", 8 * sparse_m, "8 B per match in sparse segments"),
        "emit_dense": hbm("emit_dense", 8 * dense_m, "8 B per match in dense segments"),
    }
    rooflines = {k: v for k, v in rooflines.items() if v}
    rooflines["count"]["lookups_per_s"] = n / (avg["count"] * 1e-3)
    # nominal LDS lookup peak: 32 banks x 4 B per clock per CU, conflict-free
    lds_lookup_peak = 32 * CUS * CLOCK_GHZ * 1e9
    rooflines["count"]["lds_lookup_peak_per_s"] = lds_lookup_peak
    rooflines["count"]["lookup_frac"] = rooflines["count"]["lookups_per_s"] / lds_lookup_peak
    # the dominant kernel's figures, from its duration in the timed steps
    dom = dom_name
    live_ms = live[0] / max(1, live[1])
    r = dict(rooflines[dom])
    dominant = {"kernel": dom, "avg_us": round(live_ms * 1e3, 2),
                "achieved": round(r["algorithmic_bytes"] / (live_ms * 1e-3) / 1e9, 1),
                "peak": r["peak"], "unit": r["unit"],
                "frac": round(r["algorithmic_bytes"] / (live_ms * 1e-3) / 1e9 / r["peak"], 4),
                "traffic": measured_traffic(dom, "dna_dense")}
    if dom == "count":
        dominant["lookups_per_s"] = round(n / (live_ms * 1e-3), 1)
        dominant["lookup_frac"] = round(n / (live_ms * 1e-3) / lds_lookup_peak, 4)
    # the scan's roofline: bases/s against the lower of the HBM roof at the
    # scan's algorithmic bytes per base (packed text read + 8 B per match)
    # and the LDS roof at one table lookup per base
    roofline = scan_roofline(n, total, scan_ms, text_bytes_per_base=0.25,
                             kernel_sum_us=sum(avg[k] for k in avg) * 1e3 - avg.get("encode", 0) * 1e3,
                             traffic=measured_traffic("scan", "dna_dense"))

    cus, lds = ac.ac_device_info()
    lds_limit = lds - 512
    if info.table_bytes + 1024 <= lds_limit:
        placement = "LDS (whole table)"
    else:
        rows = min(info.hot_states, lds_limit // (info.sigma * 2))
        placement = (f"hybrid: {rows} most likely rows in LDS as 16-bit ids, "
                     f"the rest from L2" if rows else "global (L1/L2)")

    # whole-step HBM roofline: letters read + packed write + packed read +
    # 8 B per match written
    step_bytes = n + 2 * ((n + 3) // 4) + 8.0 * total
    result = {
        "metric": METRIC,
        "value": round(n / (step_ms * 1e-3) / 1e9, 3),
        "unit": "Gbases/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "dna_dense: 268,435,456 DNA bases as letters in HBM, packed to "
                               "2 bits in the step, GC 0.4, 1% poly-A runs of 50-500; 10,000 "
                               "patterns (A^8..A^16, 7,000 cut 10-30, 2,991 random 10-30)",
                   "bases": n, "patterns": inst.patterns.count, "states": info.states,
                   "table_mib": round(info.table_bytes / 2**20, 3), "matches": total,
                   "text_format": "2-bit", "placement": placement},
        "roofline": roofline,
        "dominant_kernel": dominant,
        "step_hbm_roofline": {"algorithmic_bytes": step_bytes,
                              "achieved_gbs": round(step_bytes / (step_ms * 1e-3) / 1e9, 1),
                              "frac": round(step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "scan_only": {"ms": round(scan_ms, 4), "gbases_s": round(n / (scan_ms * 1e-3) / 1e9, 3)},
        "matches_per_s": round(total / (step_ms * 1e-3), 1),
        "matches_dense_segments": dense_m,
        "kernel_us": {k: round(v * 1e3, 2) for k, v in avg.items()},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in rooflines.items()},
        "build_ms": round(info.build_ms, 2),
    }

    # --------------------------------------------------------- CPU oracle
    if not args.no_cpu:
        import oracle
        m = oracle.Machine(inst.patterns, 4)
        times = []
        with pinned_to_one_core() as core:
            for _ in range(3):
                t = time.perf_counter()
                pid, end = m.scan(inst.text)
                times.append(time.perf_counter() - t)
                if len(times) < 3:
                    del pid, end
        cpu_s = float(np.median(times))
        want = oracle.keys(pid, end)
        got = ac.match_keys(out)
        exact = bool(len(want) == total and np.array_equal(got, want))
        log(f"[bench] oracle: {cpu_s:.2f} s for {n} bases (median of 3, core {core}); "
            f"bit-exact: {exact}")
        result["bit_exact"] = exact
        result["cpu_baseline"] = {"value": round(n / cpu_s / 1e9, 4), "unit": "Gbases/s",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"the whole dna_dense text ({n} bases), scan only "
                                            f"(build excluded), median of 3 runs, one thread "
                                            f"pinned to host core {core}",
                                  "host_cpu": host_cpu(),
                                  "speedup_gpu_step": round(result["value"] / (n / cpu_s / 1e9), 1)}
        del pid, end, want, got
        # the paper's own parallel design on the host's cores (context only)
        result["paper_design_cpu"] = bench_split_cpu(oracle, inst, result)

    # --------------------------------------------------------- batched vs plain
    if not args.no_batch:
        result["batched"] = bench_batch(args, torch, ac, W, dev, stream)

    # --------------------------------------------------------- variants
    if not args.no_variants:
        result["variants"] = bench_variants(args, torch, ac, W, inst, d, packed, out, total,
                                            scan_ms)

    # --------------------------------------------------------- other configs
    if not args.no_protein:
        result["protein"] = bench_protein(args, torch, ac, W, dev, stream)
    if not args.no_small:
        result["dna_small_graph"] = bench_small_graph(args, torch, ac, W, dev, stream)
    if not args.no_peaks:
        result["measured_peaks"] = bench_peaks(torch, result)

    # --------------------------------------------------------- build vs scan
    result["build_vs_scan"] = bench_build(args, ac, W, inst, step_ms)

    # --------------------------------------------------------- serving
    if not args.no_serve:
        result["serve"] = bench_serve(args, torch, ac, W)

    del out
    print(json.dumps(result), flush=True)


class pinned_to_one_core:
    """Run the enclosed CPU work on one host core (the first one this process
    may use), then restore the process's affinity."""

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        self.core = min(self.saved)
        os.sched_setaffinity(0, {self.core})
        return self.core

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)
        return False


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "os_cpu_count": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


def bench_split_cpu(oracle, inst, result):
    """The paper's second parallel design (pattern slices, one machine and one
    POSIX thread each, every thread reading the whole text) on N = 1 and
    N = all usable host cores, over a 12 MiB-base prefix of the dna_dense
    text (the paper's Fig. 5 input size) with the full dictionary.  Timed as
    the paper timed it (build + scan) and scan only; the N-thread speed-up
    is quoted beside the paper's 9x (context, not a target)."""
    text = inst.text[:12 << 20]
    cores = len(os.sched_getaffinity(0))
    rows = []
    for parts in sorted({1, cores}):
        r = oracle.split_run(inst.patterns, 4, text, parts)
        rows.append({"threads": parts, "matches": int(r["counts"].sum()),
                     "build_scan_s": round(r["wall_build_scan_s"], 4),
                     "scan_only_s": round(r["wall_scan_s"], 4),
                     "build_s_max_thread": round(float(r["build_s"].max()), 4),
                     "gbases_s_build_scan": round(len(text) / r["wall_build_scan_s"] / 1e9, 4),
                     "gbases_s_scan_only": round(len(text) / r["wall_scan_s"] / 1e9, 4)})
    one, alln = rows[0], rows[-1]
    res = {"design": "pattern list cut into N slices, one goto/failure machine and one "
                     "POSIX thread per slice, every thread scans the whole text",
           "sample": f"{len(text)} bases (prefix of dna_dense), 10,000 patterns",
           "cores": cores, "host_cpu": host_cpu(), "runs": rows,
           "speedup_n_over_1_build_scan": round(one["build_scan_s"] / alln["build_scan_s"], 2),
           "speedup_n_over_1_scan_only": round(one["scan_only_s"] / alln["scan_only_s"], 2),
           "paper_speedup_context": "9x: 16 threads of an 8-core Xeon X7560 over one thread "
                                    "(abstract; section V words it as over a Pentium 4), "
                                    "build + scan, the paper's own data",
           "gpu_step_over_n_thread_scan_only": round(result["value"] / alln["gbases_s_scan_only"], 1)}
    log(f"[bench] paper design on CPU: {cores} threads, build+scan speed-up "
        f"{res['speedup_n_over_1_build_scan']}x, scan-only {res['speedup_n_over_1_scan_only']}x")
    return res


def bench_protein(args, torch, ac, W, dev, stream):
    """The protein workload: 67,108,864 residues (20 letters, skewed
    background) as letters in HBM, 5,000 patterns of 5-12 cut from the text.
    A step encodes the letters to byte codes and scans; the scan is also
    timed alone, and its output compared with the oracle's."""
    inst = W.protein(scale=args.scale)
    n = len(inst.text)
    d = ac.ac_build(inst.patterns, sigma=20)
    fmt = ac.AC_TEXT_U8
    letters = torch.from_numpy(W.to_ascii(inst.text, W.PROTEIN)).to(dev)
    codes = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(ac.ac_scan_workspace_size(d, n, fmt), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    ac.ac_encode(letters, ac.AC_ALPHA_PROTEIN, fmt, codes)
    dummy = torch.empty((1, 2), dtype=torch.int32, device=dev)
    ac.ac_scan(d, codes, n, fmt, dummy, 0, count, workspace_dev=ws)
    torch.cuda.synchronize()
    total = int(count.item())
    out = torch.empty((max(1, total), 2), dtype=torch.int32, device=dev)

    def scan():
        ac.ac_scan(d, codes, n, fmt, out, total, count, workspace_dev=ws)

    def step():
        ac.ac_encode(letters, ac.AC_ALPHA_PROTEIN, fmt, codes)
        scan()

    def timeit(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    step_ms = timeit(step, args.steps)
    scan_ms = timeit(scan, args.steps)
    ac.ac_timing_enable(True)
    ac.ac_timing_read(reset=True)
    for _ in range(args.steps):
        scan()
    torch.cuda.synchronize()
    kt = ac.ac_timing_read(reset=True)
    ac.ac_timing_enable(False)
    kus = {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt.items() if v[1]}
    import oracle
    want = oracle.Machine(inst.patterns, 20).scan_keys(inst.text)
    exact = bool(total == len(want) and np.array_equal(ac.match_keys(out), want))
    roof = scan_roofline(n, total, scan_ms, text_bytes_per_base=1.0,
                         kernel_sum_us=sum(kus.values()),
                         traffic=measured_traffic("scan", "protein"))
    log(f"[bench] protein: step {step_ms:.3f} ms, scan {scan_ms:.3f} ms "
        f"({n / scan_ms / 1e6:.1f} Gres/s), {total} matches, bit-exact {exact}; kernels {kus}")
    info = d.info
    return {"workload": "protein: 67,108,864 residues as letters in HBM (20 letters, skewed "
                        "background, max 10 %, min 1.3 %), 5,000 patterns of 5-12 cut from "
                        "the text; byte codes",
            "residues": n, "patterns": inst.patterns.count, "states": info.states,
            "table_mib": round(info.table_bytes / 2**20, 3), "matches": total,
            "step_ms": round(step_ms, 4), "gbases_s_step": round(n / (step_ms * 1e-3) / 1e9, 3),
            "scan_ms": round(scan_ms, 4), "gbases_s_scan": round(n / (scan_ms * 1e-3) / 1e9, 3),
            "kernel_us": kus, "roofline": roof, "bit_exact": exact}


def bench_small_graph(args, torch, ac, W, dev, stream):
    """dna_small (1,048,576 bases as byte codes, 100 patterns): one scan takes
    a few microseconds of GPU work, so it is timed as 100 scans captured in
    one hipGraph and replayed, and also as single calls."""
    inst = W.dna_small()
    n = len(inst.text)
    d = ac.ac_build(inst.patterns, sigma=4)
    fmt = ac.AC_TEXT_U8
    codes = torch.from_numpy(inst.text.copy()).to(dev)
    ws = torch.empty(ac.ac_scan_workspace_size(d, n, fmt), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out, total = ac.scan(d, codes, fmt, n=n)
    out = torch.full((total + 8, 2), -1, dtype=torch.int32, device=dev)
    iters = 100
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        ac.ac_scan(d, codes, n, fmt, out, total, count, workspace_dev=ws, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(iters):
                ac.ac_scan(d, codes, n, fmt, out, total, count, workspace_dev=ws, stream=s)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record(stream)
    for _ in range(reps):
        g.replay()
    b.record(stream)
    torch.cuda.synchronize()
    per_scan_ms = a.elapsed_time(b) / (reps * iters)
    import oracle
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    exact = bool(int(count.item()) == len(want) and
                 np.array_equal(ac.match_keys(out[:len(want)]), want))
    call_ms = _timed(torch, lambda: ac.ac_scan(d, codes, n, fmt, out, total, count,
                                               workspace_dev=ws), 50)
    log(f"[bench] dna_small: {per_scan_ms * 1e3:.2f} us per scan in a graph of {iters} "
        f"({n / per_scan_ms / 1e6:.1f} Gbases/s); {call_ms * 1e3:.1f} us per call")
    return {"workload": "dna_small: 1,048,576 uniform DNA bases as byte codes, 100 patterns of "
                        "8-16 (50 cut, 50 random)", "matches": total,
            "graph_iterations": iters, "us_per_scan_graph": round(per_scan_ms * 1e3, 3),
            "gbases_s_graph": round(n / (per_scan_ms * 1e-3) / 1e9, 3),
            "us_per_call_wall": round(call_ms * 1e3, 2),
            "gbases_s_call_wall": round(n / (call_ms * 1e-3) / 1e9, 3), "bit_exact": exact}


def bench_peaks(torch, result):
    """Measured ceilings (the roofline denominators) beside the published
    ones, and the scan's fractions of the measured ones."""
    from paper_1403_7294_amd import microbench
    m = microbench.measure(torch)
    m["nominal"] = {"hbm_gbs": HBM_PEAK_GBS, "lds_lookups_per_s": LDS_LOOKUP_PEAK}
    r = result["roofline"]
    best_hbm = max(m["hbm_copy_gbs"], m["hbm_write_gbs"], m["hbm_read_gbs"])
    m["scan_frac_of_measured_hbm"] = round(r["bases_per_s"] * r["bytes_per_base"] / 1e9 /
                                           best_hbm, 4)
    m["scan_frac_of_measured_write"] = round(r["bases_per_s"] * r["bytes_per_base"] / 1e9 /
                                             m["hbm_write_gbs"], 4)
    log(f"[bench] measured peaks: {m}")
    return m


def bench_batch(args, torch, ac, W, dev, stream):
    t0 = time.time()
    insts = W.batch(scale=args.scale)
    dicts = [ac.ac_build(i.patterns, sigma=4) for i in insts]
    fmt = ac.AC_TEXT_2BIT
    texts = []
    for i in insts:
        letters = torch.from_numpy(W.to_ascii(i.text, W.DNA)).to(dev)
        p = torch.empty((len(i.text) + 3) // 4, dtype=torch.uint8, device=dev)
        ac.ac_encode(letters, ac.AC_ALPHA_DNA, fmt, p)
        texts.append(p)
    bases = sum(len(i.text) for i in insts)
    counts = torch.zeros(len(insts), dtype=torch.int64, device=dev)
    # exact output sizes from a counting run of the plain form
    dummy = torch.empty((1, 2), dtype=torch.int32, device=dev)
    for k, (dct, t, i) in enumerate(zip(dicts, texts, insts)):
        ac.ac_scan(dct, t, len(i.text), fmt, dummy, 0, counts[k:k + 1])
    torch.cuda.synchronize()
    caps = counts.cpu().numpy().astype(np.int64)
    outs = [torch.empty((max(1, int(c)), 2), dtype=torch.int32, device=dev) for c in caps]
    wss = [torch.empty(ac.ac_scan_workspace_size(dct, len(i.text), fmt), dtype=torch.uint8,
                       device=dev) for dct, i in zip(dicts, insts)]
    log(f"[bench] batch: {len(insts)} instances, {bases} bases, {int(caps.sum())} matches "
        f"(setup {time.time() - t0:.1f} s)")

    def plain():
        for k, (dct, t, i) in enumerate(zip(dicts, texts, insts)):
            ac.ac_scan(dct, t, len(i.text), fmt, outs[k], int(caps[k]), counts[k:k + 1],
                       workspace_dev=wss[k])

    items = [(dct, t, len(i.text), fmt, outs[k], int(caps[k]), counts[k:k + 1])
             for k, (dct, t, i) in enumerate(zip(dicts, texts, insts))]
    plan = ac.ac_batch_create(items)

    def batched():
        ac.ac_batch_run(plan)

    def timeit(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, args.steps // 2)
    plain_ms = timeit(plain, reps)
    plain_keys = [ac.match_keys(o[:int(c)]) for o, c in zip(outs, caps)]
    batch_ms = timeit(batched, reps)
    same = all(np.array_equal(ac.match_keys(o[:int(c)]), k)
               for o, c, k in zip(outs, caps, plain_keys))
    # the batched launches captured once in a graph and replayed
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ac.ac_batch_run(plan, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            ac.ac_batch_run(plan, stream=s)
    graph_ms = timeit(g.replay, reps)
    same_graph = all(np.array_equal(ac.match_keys(o[:int(c)]), k)
                     for o, c, k in zip(outs, caps, plain_keys))
    # the same batch with the two-symbol table where it fits LDS
    two = {"placement": ac.AC_PLACE_LDS2, "chains": 1}
    plan2 = ac.ac_batch_create(items, tune=two)
    two_ms = timeit(lambda: ac.ac_batch_run(plan2), reps)
    plan2.close()
    same_two = all(np.array_equal(ac.match_keys(o[:int(c)]), k)
                   for o, c, k in zip(outs, caps, plain_keys))
    # the launch shape picked by the autotuner for this batch
    from paper_1403_7294_amd import tune as actune
    best = actune.autotune_batch(items)
    plan3 = ac.ac_batch_create(items, tune=best)
    tuned_ms = timeit(lambda: ac.ac_batch_run(plan3), reps)
    plan3.close()
    same_tuned = all(np.array_equal(ac.match_keys(o[:int(c)]), k)
                     for o, c, k in zip(outs, caps, plain_keys))
    log(f"[bench] batch: plain {plain_ms:.3f} ms, batched {batch_ms:.3f} ms, "
        f"graph {graph_ms:.3f} ms, autotuned {tuned_ms:.3f} ms ({best}), "
        f"identical {same and same_graph and same_tuned}")
    plan.close()
    return {"workload": "batch: 512 DNA instances, text log-uniform 4 Ki-4 Mi bases, "
                        "10-2,000 patterns of 8-24 each, 2-bit text",
            "instances": len(insts), "bases": bases, "matches": int(caps.sum()),
            "plain_ms": round(plain_ms, 3), "batched_ms": round(batch_ms, 3),
            "graph_ms": round(graph_ms, 3),
            "plain_gbases_s": round(bases / (plain_ms * 1e-3) / 1e9, 3),
            "batched_gbases_s": round(bases / (batch_ms * 1e-3) / 1e9, 3),
            "speedup_batched_vs_plain": round(plain_ms / batch_ms, 2),
            "speedup_graph_vs_plain": round(plain_ms / graph_ms, 2),
            "two_symbol_batched_ms": round(two_ms, 3),
            "autotuned_ms": round(tuned_ms, 3), "autotuned_shape": best,
            "autotuned_gbases_s": round(bases / (tuned_ms * 1e-3) / 1e9, 3),
            "identical_to_plain": bool(same and same_graph and same_two and same_tuned)}


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps * 1e3


def bench_variants(args, torch, ac, W, inst, d, packed, out, total, scan_ms):
    """The other forms of stage 2 on the same workloads, each checked equal to
    the main scan's output: the paper's second design (one machine per
    pattern slice, each table in LDS, merged by a stable sort), the
    failure-less kernel (one thread per start position, then a sort), and the
    two-symbol table on an LDS-resident dictionary.  Wall-clock per call
    (the partitioned and failure-less forms synchronise once per call)."""
    fmt = ac.AC_TEXT_2BIT
    n = len(inst.text)
    res = {"dna_dense_scan_ms": round(scan_ms, 4)}
    out2 = torch.empty_like(out)
    cnt = torch.zeros(1, dtype=torch.int64, device=out.device)
    part = ac.ac_build_partitioned(inst.patterns, sigma=4)
    ms = _timed(torch, lambda: ac.ac_scan(part, packed, n, fmt, out2, total, cnt), 3)
    res["partitioned"] = {"parts": len(ac.ac_dict_parts(part)), "ms": round(ms, 3),
                          "identical": bool(torch.equal(out2, out))}
    part.close()
    out2.fill_(0)
    ms = _timed(torch, lambda: ac.ac_scan_pfac(d, packed, n, fmt, out2, total, cnt), 3)
    res["failure_less"] = {"ms": round(ms, 3), "identical": bool(torch.equal(out2, out))}
    del out2
    # an LDS-resident dictionary (dna_small) over its own 1 Mi-base text
    sm = W.dna_small()
    ds = ac.ac_build(sm.patterns, sigma=4)
    letters = torch.from_numpy(W.to_ascii(sm.text, W.DNA)).to(out.device)
    ps = torch.empty((len(sm.text) + 3) // 4, dtype=torch.uint8, device=out.device)
    ac.ac_encode(letters, ac.AC_ALPHA_DNA, fmt, ps)
    ref, tot = ac.scan(ds, ps, fmt, n=len(sm.text))
    o = torch.empty_like(ref)
    small = {}
    for name, fn in [
            ("lds", lambda: ac.ac_scan(ds, ps, len(sm.text), fmt, o, tot, cnt)),
            ("lds_two_symbol", lambda: ac.ac_scan(ds, ps, len(sm.text), fmt, o, tot, cnt,
                                                  tune={"placement": ac.AC_PLACE_LDS2})),
            ("failure_less", lambda: ac.ac_scan_pfac(ds, ps, len(sm.text), fmt, o, tot, cnt))]:
        ms = _timed(torch, fn, 20)
        small[name] = {"ms": round(ms, 4), "identical": bool(torch.equal(o, ref))}
    res["dna_small"] = small
    log("[bench] variants: partitioned %(p)s ms (%(k)d parts), failure-less %(f)s ms; dna_small %(s)s"
        % {"p": res["partitioned"]["ms"], "k": res["partitioned"]["parts"],
           "f": res["failure_less"]["ms"], "s": {k: v["ms"] for k, v in small.items()}})
    return res


def bench_build(args, ac, W, inst, step_ms):
    """Host build time (stage 1) against scan time (stage 2): the paper finds
    machine construction dominating on its CPUs.  Parallel (level by level,
    up to 16 threads) and one-thread builds of the same tables."""
    rows = []
    sets = [("dna_dense", inst.patterns)] + [
        (f"serve dictionary {k}", p) for k, p in enumerate(W.serve(requests=1).dictionaries)]
    for name, pats in sets:
        par = min(ac.ac_build(pats, sigma=4, host_only=True).info.build_ms for _ in range(2))
        ser = min(ac.ac_build(pats, sigma=4, host_only=True, serial=True).info.build_ms
                  for _ in range(2))
        d = ac.ac_build(pats, sigma=4, host_only=True)
        rows.append({"dictionary": name, "patterns": int(pats.count), "states": d.info.states,
                     "build_ms": round(par, 2), "build_ms_one_thread": round(ser, 2)})
    log("[bench] build: " + ", ".join(f"{r['dictionary']} {r['build_ms']} ms" for r in rows))
    return {"dictionaries": rows, "dna_dense_step_ms": round(step_ms, 4),
            "dna_dense_build_over_step": round(rows[0]["build_ms"] / step_ms, 2)}


def bench_serve(args, torch, ac, W):
    """Continuous batching under Poisson arrivals: the saturated request
    rate R_sat (all requests queued at once), then latency percentiles at a
    fixed arrival rate of 0.7 R_sat."""
    from paper_1403_7294_amd.serve import Server, run_poisson
    t0 = time.time()
    # enough requests that filling and draining the server's pipeline (about
    # 20 ms) is a small part of the saturated run
    n_sat = 6000
    wl = W.serve(scale=args.scale, requests=n_sat + args.serve_requests)
    letters = [W.to_ascii(t, W.DNA) for t in wl.texts]
    srv = Server(wl.dictionaries, budget_bytes=8 << 30)
    log(f"[bench] serve: {len(letters)} requests, {sum(len(t) for t in letters)} bases, "
        f"8 dictionaries (setup {time.time() - t0:.1f} s)")
    # warm-up (a saturated run of its own: the first server of a process
    # runs its batches markedly slower), then saturation: everything queued
    # at once
    for f in [srv.submit(letters[k], int(wl.dict_of[k])) for k in range(2000)]:
        f.result()
    srv.close()
    srv = Server(wl.dictionaries, budget_bytes=8 << 30)
    futs = [srv.submit(letters[k], int(wl.dict_of[k])) for k in range(n_sat)]
    sat_res = [f.result() for f in futs]
    sat = srv.close()
    r_sat = n_sat / sat.wall_s
    # the same requests alone, for equality (a sample)
    same = True
    for k in range(0, n_sat, n_sat // 25):
        dev = torch.from_numpy(wl.texts[k].copy()).cuda()
        out, total = ac.scan(srv.dicts[int(wl.dict_of[k])], dev, ac.AC_TEXT_U8)
        same &= bool(np.array_equal(ac.match_keys(out), sat_res[k]))
    rate = 0.7 * r_sat
    srv = Server(wl.dictionaries, budget_bytes=8 << 30)
    futs = run_poisson(srv, letters[n_sat:], wl.dict_of[n_sat:], wl.gaps[n_sat:], rate)
    for f in futs:
        f.result()
    st = srv.close()
    s = st.summary()
    log(f"[bench] serve: R_sat {r_sat:.0f} req/s ({sat.bases / sat.wall_s / 1e9:.2f} Gbases/s); "
        f"at {rate:.0f} req/s: p50 {s['p50_ms']} ms, p99 {s['p99_ms']} ms")
    return {"workload": "serve: requests of log-uniform 1 K-1 M DNA letters, 8 dictionaries of "
                        "1,000-50,000 random 10-30-mers, Poisson arrivals",
            "saturated_requests_per_s": round(r_sat, 1),
            "saturated_gbases_s": round(sat.bases / sat.wall_s / 1e9, 3),
            "arrival_rate_per_s": round(rate, 1), **s,
            "sample_equals_alone": same}


if __name__ == "__main__":
    main()
