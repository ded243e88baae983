#!/usr/bin/env python3
"""Benchmark of the Schulze hot path on one MI355X.

A step is one pass of the whole path over one election whose ballots are
already resident in HBM: pairwise counts -> widest-path closure -> winners
-> ranking.  The default workload is m=4096 candidates, n=60000 voters drawn
from Mallows(0.97) with 30% of the ballots cut to their top-100, uint16
counters.

Printed (one JSON line): throughput as m^3 max-min updates per second of the
whole step (Gop/s), per-kernel times from HIP events recorded on the launch
stream inside the timed region, the roofline of the dominant kernel and of
the closure, and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: 256 CUs x 64 lanes x 2.4 GHz 32-bit VALU lane-ops,
# 8 TB/s HBM3E.
VALU_LANE_OPS = 256 * 64 * 2.4e9
HBM_BYTES = 8.0e12

WORKLOADS = ("mid", "small", "large", "learned", "batch", "paper")


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch recorded in profiles/traffic.txt, or None when no
    record exists or the kernel's source changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, wl, src, sha, fetch, write = line.split()[:6]
        if k != kernel or wl != workload_name:
            continue
        h = hashlib.sha256()
        for part in src.split("+"):  # the kernel's source files, hashed in order
            with open(os.path.join(ROOT, part), "rb") as f:
                h.update(f.read())
        if not h.hexdigest().startswith(sha):
            return None
        return float(fetch) + float(write)
    return None


def valu_probe(ctx):
    """Measured integer VALU issue rate (the peak the "alu" rooflines divide
    by is the published one; this puts the chip's delivered rate beside it)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    wg, trips = 8 * cus, 8000
    ctx.valu_probe(wg, trips)  # warm-up
    best = None
    for _ in range(3):
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        ops = ctx.valu_probe(wg, trips)
        end.record()
        torch.cuda.synchronize()
        t = start.elapsed_time(end) * 1e-3
        best = t if best is None else min(best, t)
    rate = ops / best
    return {"achieved": rate / 1e12, "peak": VALU_LANE_OPS / 1e12, "unit": "T lane-ops/s",
            "frac": rate / VALU_LANE_OPS,
            "what": "packed uint16 max/min/add/sub, 8 independent chains per lane, 8 waves per SIMD"}


def host_cpu():
    """The host CPU the oracle ran on: model name and logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=WORKLOADS, default="mid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-voters", type=int, default=30000)
    ap.add_argument("--batch-elections", type=int, default=4096)
    ap.add_argument("--no-per-election", action="store_true",
                    help="batch workload: skip the pass of per-election calls (profiling runs)")
    ap.add_argument("--closure-schedule", choices=("auto", "phased"), default="auto")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy a 1 GiB buffer once (a known-size reference "
                         "for hardware byte counters)")
    return ap.parse_args()


def make_workload(name):
    import workload
    return {"mid": workload.plain_mid, "small": workload.plain_small, "large": workload.plain_large,
            "learned": workload.plain_learned, "paper": workload.plain_paper}[name]()


def bench_learned(args):
    """Exact winners through the learned proposal versus the full closure, on
    m=32768 candidates, n=200000 top-30 Plackett-Luce Zipf(1.0) ballots."""
    import numpy as np
    import torch

    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.proposer import load_checkpoint

    dev = torch.device("cuda", 0)
    wl = make_workload("learned")
    m, n = wl.m, wl.n
    ckpt = os.path.join(ROOT, "paper_2505_12976_amd", "data", "proposer.npz")
    params = torch.from_numpy(load_checkpoint(ckpt)["params"]).to(dev)
    ctx = sz.Context(0)
    ballots = torch.from_numpy(wl.ballots).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = ctx.pairwise(ballots, m, dtype="i32")
    torch.cuda.synchronize()
    t_count = time.perf_counter() - t0
    print(f"[bench] count {t_count * 1e3:.1f} ms", file=sys.stderr, flush=True)

    def full():
        p = ctx.closure(d)
        w, nw = ctx.winners(p)
        torch.cuda.synchronize()
        return w

    def learned():
        w, nw, st = ctx.winners_learned(d, float(n), params)
        torch.cuda.synchronize()
        return w, st

    learned()  # warm-up
    t_learned = []
    ctx.reset_timing()
    ctx.set_timing(True)
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        w_l, st = learned()
        t_learned.append(time.perf_counter() - t0)
    ctx.set_timing(False)
    print(f"[bench] learned {np.median(t_learned) * 1e3:.2f} ms", file=sys.stderr, flush=True)
    # per-kernel times of the learned path (HIP events on the launch stream)
    kern = {}
    for nm in ("weights", "feature_rows", "features", "mlp_prepare", "mlp_forward", "propose", "widest", "verdict",
               "fill"):
        launches, total = ctx.kernel_time(nm)
        if launches:
            kern[nm] = {"launches_per_call": launches / len(t_learned), "ms_per_call": total / len(t_learned),
                        "avg_launch_ms": total / launches}
    # dominant kernel: the pass that reads d and writes w, w^T and the
    # per-candidate statistics (HBM-bound): d read once, w and w^T written once
    es = 4
    w_bytes = 3 * es * m * m
    roof = None
    if "feature_rows" in kern:
        ach = w_bytes / (kern["feature_rows"]["avg_launch_ms"] / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "feature_rows (weights, transposed weights, statistics)",
                "achieved": ach, "peak": HBM_BYTES / 1e9, "unit": "GB/s",
                "frac": ach * 1e9 / HBM_BYTES, "traffic": None, "algorithmic_bytes": w_bytes}
    if "widest" in kern:
        kern["widest"]["note"] = "one launch per direction runs all sweeps to the fixpoint"
    t_full = []
    for _ in range(2):
        t0 = time.perf_counter()
        w_f = full()
        t_full.append(time.perf_counter() - t0)
        print(f"[bench] full closure {t_full[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # the label-propagation winners algorithm of Section 4 on the same counts
    def propagate():
        w, nw, st = ctx.winners_propagate(d)
        torch.cuda.synchronize()
        return w, st

    propagate()  # warm-up
    t_prop = []
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        w_p, st_p = propagate()
        t_prop.append(time.perf_counter() - t0)
    print(f"[bench] label propagation {np.median(t_prop) * 1e3:.2f} ms, {st_p}", file=sys.stderr, flush=True)
    # the closure without value ranking (int32 arithmetic throughout)
    ctx.set_value_ranking(False)
    t0 = time.perf_counter()
    w_i = full()
    t_full_i32 = time.perf_counter() - t0
    ctx.set_value_ranking(True)
    print(f"[bench] full closure, int32 values {t_full_i32 * 1e3:.1f} ms", file=sys.stderr, flush=True)
    w_f_np = w_f.cpu().numpy()
    exact = bool((w_l.cpu().numpy() == w_f_np).all())
    exact_prop = bool((w_p.cpu().numpy() == w_f_np).all())
    exact_i32 = bool((w_i.cpu().numpy() == w_f_np).all())
    tl, tf = float(np.median(t_learned)), float(min(t_full))
    tp = float(np.median(t_prop))
    out = {
        "metric": "learned-verify vs full-closure speedup",
        "value": tf / tl,
        "unit": "x",
        "n_gpus": 1,
        "steps": len(t_learned),
        "higher_is_better": True,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": wl.name, "m": m, "n": n, "recipe": wl.recipe},
        "ms_learned": tl * 1e3,
        "ms_full_closure_and_winners": tf * 1e3,
        "ms_count": t_count * 1e3,
        "closure_gops": m ** 3 / tf / 1e9,
        "ms_full_closure_int32_values": t_full_i32 * 1e3,
        "ms_label_propagation": tp * 1e3,
        "kernels_learned": kern,
        "roofline": roof,
        "label_propagation_stats": st_p,
        "exact": exact,
        "exact_label_propagation": exact_prop,
        "exact_int32_closure": exact_i32,
        "winners": np.nonzero(w_l.cpu().numpy())[0].tolist(),
        "learned_stats": st,
    }
    out["valu_probe"] = valu_probe(ctx)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """4096 independent elections (m ~ U{8..512}, n ~ U{50..20000}, full
    Mallows rankings with phi ~ U[0.5, 1]) in one persistent launch replayed
    from a captured HIP graph, against one pass of per-election calls
    (pairwise, closure, winners, ranking for each election in turn)."""
    import numpy as np
    import torch

    import paper_2505_12976_amd as sz
    import workload
    from paper_2505_12976_amd.batch import Packed, alloc_outputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    E = args.batch_elections
    t0 = time.time()
    flat, desc, (ms, ns, phis) = workload.batch_mallows(1004, E)
    print(f"[bench] batch of {E} elections generated in {time.time() - t0:.1f}s "
          f"({flat.nbytes / 1e9:.1f} GB of ballots)", file=sys.stderr, flush=True)
    packed = Packed(flat, desc, int(np.sum(ms * ms)), int(np.sum(ms)))
    ctx = sz.Context(0)
    ballots = torch.from_numpy(flat).to(dev)
    del flat
    t0 = time.time()
    tune_ms = ctx.batch_autotune(16, int(ms.max()))
    names = ["registers", "tiled32", "tiled64", "tiled128"]
    tuned = [ctx.batch_get_closure(16, 32 * (b + 1)) for b in range(tune_ms.shape[0])]
    print(f"[bench] autotuned closure schedules in {time.time() - t0:.1f}s: {tuned}", file=sys.stderr, flush=True)
    plan = ctx.batch_plan(desc, "u16", "winning_votes")
    outs = alloc_outputs(packed, dev)

    def run():
        ctx.batch_run(plan, ballots, outs["d"], outs["is_winner"], p=outs["p"], n_winners=outs["n_winners"],
                      beaten_by=outs["beaten_by"], order=outs["order"], graph=True)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    if ctx.device_error() != 0:
        raise RuntimeError("device error during warmup")
    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ctx.set_timing(False)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    launches, total = ctx.kernel_time("batch")
    kernel_ms = total / max(launches, 1)
    print(f"[bench] batch: {ms_per_step:.2f} ms per step (graph {kernel_ms:.2f} ms)", file=sys.stderr, flush=True)

    # per-election launches: the same outputs, election by election
    d_ref = torch.empty_like(outs["d"])
    p_ref = torch.empty_like(outs["p"])
    w_ref = torch.empty_like(outs["is_winner"])
    o_ref = torch.empty_like(outs["order"])
    bb_ref = torch.empty_like(outs["beaten_by"])

    def per_election():
        for e, (bo, n, L, m, mo, vo) in enumerate(desc):
            b = ballots[bo:bo + n * L].view(n, L)
            d = ctx.pairwise(b, m, dtype="i32", out=d_ref[mo:mo + m * m].view(m, m))
            p = ctx.closure(d, "winning_votes", out=p_ref[mo:mo + m * m].view(m, m))
            w, _ = ctx.winners(p)
            order, beaten = ctx.ranking(p)
            w_ref[vo:vo + m].copy_(w)
            o_ref[vo:vo + m].copy_(order)
            bb_ref[vo:vo + m].copy_(beaten)

    t_per, exact = None, None
    if not args.no_per_election:
        per_election()  # warm-up (workspace growth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_election()
        torch.cuda.synchronize()
        t_per = time.perf_counter() - t0
        exact = bool(torch.equal(d_ref, outs["d"]) and torch.equal(p_ref, outs["p"]) and
                     torch.equal(w_ref, outs["is_winner"]) and torch.equal(o_ref, outs["order"]) and
                     torch.equal(bb_ref, outs["beaten_by"]))
        print(f"[bench] per-election calls: {t_per * 1e3:.1f} ms, identical outputs: {exact}", file=sys.stderr,
              flush=True)
    if ctx.device_error() != 0:
        raise RuntimeError("device error")

    # algorithmic work: one VALU lane-op per (voter, candidate pair) of the count,
    # one per packed max-min update of the closure (padded sizes actually run)
    count_ops = float(np.sum(ns * ms * (ms - 1) / 2))
    closure_ops = float(np.sum(ms.astype(np.float64) ** 3))
    work = count_ops + closure_ops
    roof = {"bound": "alu", "kernel": "batch", "achieved": work / (kernel_ms / 1e3) / 1e12,
            "peak": VALU_LANE_OPS / 1e12, "unit": "Tops/s",
            "traffic": measured_traffic("batch", "batch_mallows_E%d" % E)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {
        "metric": "closure Gop/s (max-min) + elections/sec; learned-verify vs full-closure speedup",
        "value": E / (ms_per_step / 1e3),
        "unit": "elections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "batch_mallows_E%d" % E, "elections": E, "m": "U{8..512}", "n": "U{50..20000}",
                   "phi": "U[0.5,1.0]", "seed": 1004, "weight_mode": "winning_votes", "parallelism": "single GPU",
                   "launch": "one persistent kernel per step, replayed from a captured HIP graph"},
        "elections_per_s_per_election_calls": E / t_per if t_per else None,
        "speedup_vs_per_election_calls": t_per / (ms_per_step / 1e3) if t_per else None,
        "ms_per_election_calls_pass": t_per * 1e3 if t_per else None,
        "identical_to_per_election_calls": exact,
        "graph_ms": kernel_ms,
        "count_comparisons": count_ops,
        "closure_updates": closure_ops,
        "closure_schedule_by_bucket": tuned,
        "roofline": roof,
    }
    out["valu_probe"] = valu_probe(ctx)
    ctx.close()
    if not args.no_cpu_baseline:
        import oracle
        print("[bench] timing the CPU oracle on a sample of elections", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        k = 0
        while k < E and time.perf_counter() - t0 < 20.0:
            b = workload.batch_election(1004, k, int(ms[k]), int(ns[k]), float(phis[k]))
            oracle.schulze(b, int(ms[k]))
            k += 1
        t_cpu = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        out["cpu_baseline"] = {"value": k / t_cpu, "unit": "elections/s", "cores": cores, "kind": "oracle",
                               **host_cpu(),
                               "sample": f"the first {k} of the {E} elections, whole path per election "
                                         f"({t_cpu:.1f} s; ballot generation excluded)"}
    print(json.dumps(out), flush=True)


def cpu_baseline(wl, sample_voters):
    """Oracle on a bounded sample: the count over the first `sample_voters`
    ballots (scaled to all n), then weights, closure and ranking at full m."""
    import numpy as np

    import oracle
    ns = min(sample_voters, wl.n)
    sample = wl.ballots[:ns]
    t0 = time.perf_counter()
    d = oracle.pairwise(sample, wl.m)
    t_count = (time.perf_counter() - t0) * (wl.n / ns)
    t0 = time.perf_counter()
    w = oracle.weights(d, oracle.WINNING_VOTES)
    p = oracle.closure(w)
    oracle.rank(p)
    t_rest = time.perf_counter() - t0
    t_step = t_count + t_rest
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    # one thread, as the paper times its sequential baseline: count over a
    # smaller sample, closure at m1 = min(m, 2048) extrapolated by (m / m1)^3
    prev = oracle.set_threads(1)
    try:
        ns1 = min(max(1, sample_voters // 10), wl.n)
        t0 = time.perf_counter()
        oracle.pairwise(wl.ballots[:ns1], wl.m)
        t_count1 = (time.perf_counter() - t0) * (wl.n / ns1)
        m1 = min(wl.m, 2048)
        w1 = np.ascontiguousarray(w[:m1, :m1])
        t0 = time.perf_counter()
        oracle.closure(w1)
        t_close1 = (time.perf_counter() - t0) * (wl.m / m1) ** 3
    finally:
        oracle.set_threads(prev)
    t_step1 = t_count1 + t_close1
    return {
        "value": wl.m ** 3 / t_step / 1e9,
        "unit": "Gop/s",
        "cores": cores,
        **host_cpu(),
        "kind": "oracle",
        "sample": (f"count over the first {ns} of {wl.n} ballots scaled by n/{ns} "
                   f"({t_count:.1f} s scaled); weights+closure+ranking at full m={wl.m} ({t_rest:.1f} s)"),
        "seconds_per_step": t_step,
        "single_thread": {
            "value": wl.m ** 3 / t_step1 / 1e9, "unit": "Gop/s", "cores": 1,
            "seconds_per_step": t_step1, "extrapolated": True,
            "sample": (f"count over the first {ns1} ballots scaled by n/{ns1} ({t_count1:.1f} s scaled); "
                       f"closure of the leading {m1} x {m1} block of w scaled by (m/{m1})^3 ({t_close1:.1f} s)"),
        },
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return

    import numpy as np
    import torch

    import paper_2505_12976_amd as sz

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}), flush=True)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    t0 = time.time()
    wl = make_workload(args.workload)
    print(f"[bench] workload {wl.name} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    m, n = wl.m, wl.n
    ballots = torch.from_numpy(wl.ballots).to(dev)
    ctx = sz.Context(0)
    ctx.set_closure_schedule(args.closure_schedule)
    dcode = wl.d_dtype
    tdtype = torch.uint16 if dcode == "u16" else torch.int32
    d = torch.empty((m, m), dtype=tdtype, device=dev)
    p = torch.empty((m, m), dtype=tdtype, device=dev)

    def step():
        ctx.pairwise(ballots, m, dtype=dcode, out=d)
        ctx.closure(d, "winning_votes", out=p)
        ctx.winners(p)
        ctx.ranking(p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if ctx.device_error() != 0:
        raise RuntimeError("device error during warmup")
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ctx.set_timing(False)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    names = ["ballot_scan", "route", "ballot_scatter", "count_dense", "count_trunc", "count_sparse", "count_finish",
             "weights",
             "fw_diag", "fw_panel", "fw_rest", "fw_persist", "fw_store", "value_rank", "beaten_by", "rank_sort",
             "winners", "fill"]
    kern = {}
    for nm in names:
        launches, total = ctx.kernel_time(nm)
        if launches:
            kern[nm] = {"launches_per_step": launches / args.steps, "ms_per_step": total / args.steps,
                        "avg_launch_ms": total / launches}
    closure_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in
                     ("weights", "fw_diag", "fw_panel", "fw_rest", "fw_persist", "fw_store", "value_rank"))
    count_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in
                   ("ballot_scan", "route", "ballot_scatter", "count_dense", "count_trunc", "count_sparse",
                    "count_finish"))
    dominant = max(kern, key=lambda k: kern[k]["ms_per_step"])

    # algorithmic work of the two main kernels
    n_full = int(np.count_nonzero((wl.ballots != (0xFFFF if wl.ballots.dtype == np.uint16 else -1)).sum(axis=1)
                                  >= m - 1)) if wl.ballots.shape[1] >= m - 1 else 0
    roof = None
    # an int32 closure whose weights were ranked runs its updates in packed uint16
    # (six ranking launches per step: mark, block sums, scan, word ranks, apply, store)
    ranked = dcode == "i32" and kern.get("value_rank", {}).get("launches_per_step", 0) == 6
    closure_bits = 16 if (dcode == "u16" or ranked) else 32
    if dominant == "count_dense":
        # one comparison per (full ranking, unordered pair): one VALU lane-op each
        work = n_full * m * (m - 1) / 2
        avg = kern["count_dense"]["avg_launch_ms"] / 1e3
        roof = {"bound": "alu", "kernel": "count_dense", "achieved": work / avg / 1e12,
                "peak": VALU_LANE_OPS / 1e12, "unit": "Tops/s",
                "traffic": measured_traffic("count_dense", wl.name)}
    elif dominant in ("fw_rest", "fw_panel", "fw_diag", "fw_persist"):
        ops_per_update = 1 if closure_bits == 16 else 2
        work = m ** 3 * ops_per_update
        roof = {"bound": "alu", "kernel": "closure", "achieved": work / (closure_ms / 1e3) / 1e12,
                "peak": VALU_LANE_OPS / 1e12, "unit": "Tops/s",
                "traffic": measured_traffic("fw_persist", wl.name)}
    else:
        avg = kern[dominant]["avg_launch_ms"] / 1e3
        roof = {"bound": "hbm", "kernel": dominant, "achieved": None, "peak": HBM_BYTES / 1e9,
                "unit": "GB/s", "traffic": None}
    if roof.get("achieved") is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    ops_per_update = 1 if closure_bits == 16 else 2
    closure_roof = {"bound": "alu", "achieved": m ** 3 * ops_per_update / (closure_ms / 1e3) / 1e12,
                    "peak": VALU_LANE_OPS / 1e12, "unit": "Tops/s",
                    "updates_per_s": m ** 3 / (closure_ms / 1e3)}
    closure_roof["frac"] = closure_roof["achieved"] / closure_roof["peak"]
    closure_roof["traffic"] = measured_traffic("fw_persist", wl.name)
    closure_roof["value_bits"] = closure_bits
    closure_roof["value_ranked"] = ranked

    out = {
        "metric": "closure Gop/s (max-min) + elections/sec; learned-verify vs full-closure speedup",
        "value": m ** 3 / (ms_per_step / 1e3) / 1e9,
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dcode,
        "data": "synthetic",
        "config": {"workload": wl.name, "m": m, "n": n, "recipe": wl.recipe, "weight_mode": "winning_votes",
                   "parallelism": "single GPU",
                   "closure_schedule": args.closure_schedule},
        "elections_per_s": 1e3 / ms_per_step,
        "closure_ms": closure_ms,
        "closure_gops": m ** 3 / (closure_ms / 1e3) / 1e9,
        "count_ms": count_ms,
        "kernels": kern,
        "roofline": roof,
        "roofline_closure": closure_roof,
    }
    if args.workload == "paper":
        # the paper's own algorithm (winners only) on the same counts, and its
        # published single-core timings at this shape, for context
        ctx.winners_propagate(d)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st = ctx.winners_propagate(d)
        torch.cuda.synchronize()
        out["label_propagation_ms"] = (time.perf_counter() - t0) * 1e3
        out["label_propagation_stats"] = st
        out["paper_context"] = {"closure_and_ranking_single_core_min": 221,
                                "winners_only_single_core_min": 64,
                                "shape": "Global150 chart data: m=14187, n=15553, top-150",
                                "note": "the paper's own hardware and data; not a target"}
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * src.element_size()
        del src, dst
    out["valu_probe"] = valu_probe(ctx)
    ctx.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_voters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
