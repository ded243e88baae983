#!/usr/bin/env python3
"""Benchmark of the Schulze hot path on one MI355X.

Default run (no --workload): one JSON line whose headline is the widest-path
closure rate on the m=16384 workload (n=10^6 top-20 Plackett-Luce Zipf(1.1)
ballots, int32 counts).  A step is one pass of the whole single-election
path over ballots already resident in HBM: pairwise counts -> closure ->
winners -> ranking.  `value` is m^3 max-min updates divided by the closure's
time per step (Gop/s); the line also carries the step time, per-kernel times
from HIP events recorded on the launch stream inside the timed region, the
closure kernel's roofline against the integer VALU peak, the count's HBM
fraction, the CPU oracle on a bounded sample, and an equality check against
the oracle's stored results.  Two more workloads ride along as keys of their
own, each with its roofline and CPU baseline:
  "batch"    4096 independent elections in one persistent launch (elections/s),
  "learned"  exact winners by learned proposal + widest-path verification at
             m=32768 against the full closure on the same GPU (speedup).
--workload picks a single workload instead; --parts limits the default run.
"""
import argparse
import hashlib
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
METRIC = "closure Gop/s (max-min) + elections/sec; learned-verify vs full-closure speedup"

WORKLOADS = ("default", "mid", "small", "large", "learned", "batch", "paper")
PARTS = ("headline", "learned", "batch")
GOLD = os.path.join(ROOT, "tests", "golden")


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch recorded in profiles/traffic.txt, or None when no
    record exists or the kernel's source changed since it was measured."""
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


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()


def digest(a, rows=1024):
    """SHA-256 of an integer array as int64 little-endian, row-major."""
    import numpy as np
    h = hashlib.sha256()
    if a.ndim < 2:
        h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
        return h.hexdigest()
    for i in range(0, a.shape[0], rows):
        h.update(np.ascontiguousarray(a[i:i + rows], dtype="<i8").tobytes())
    return h.hexdigest()


def golden(name):
    path = os.path.join(GOLD, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=WORKLOADS, default="default")
    ap.add_argument("--parts", default=",".join(PARTS),
                    help="default workload: comma-separated parts to run (headline, learned, batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip comparing outputs with the oracle's stored results")
    ap.add_argument("--batch-elections", type=int, default=4096)
    ap.add_argument("--no-per-election", action="store_true",
                    help="batch workload: skip the pass of per-election calls (profiling runs)")
    ap.add_argument("--learned-path-only", action="store_true",
                    help="learned workload: time the learned path only, no full closures or label propagation "
                         "(profiling runs)")
    ap.add_argument("--closure-schedule", choices=("auto", "phased"), default="auto")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy a 1 GiB buffer once (a known-size reference "
                         "for hardware byte counters)")
    return ap.parse_args()


def make_workload(name):
    import workload
    return {"mid": workload.plain_mid, "small": workload.plain_small, "large": workload.plain_large,
            "learned": workload.plain_learned, "paper": workload.plain_paper}[name]()


# --------------------------------------------------------------------------- CPU baselines

def cpu_baseline_single(wl, count_voters=30000, block=2048, count_voters_1t=3000, block_1t=1024):
    """The oracle on a bounded sample of one election: the count over the
    first ballots (scaled to n by the O(n k m) count), the closure of the
    leading block x block corner of that sample's weights (scaled by
    (m / block)^3, the plain loop's cost), and ranking; all threads, then
    one thread (the paper times its sequential baseline on one core)."""
    import numpy as np

    import oracle
    m, n = wl.m, wl.n
    out = {"unit": "Gop/s", "cores": oracle_threads(), "kind": "oracle", **host_cpu(), "extrapolated": m > block}

    def leg(nv, blk):
        nv = min(nv, n)
        t0 = time.perf_counter()
        d = oracle.pairwise(wl.ballots[:nv], m)
        t_count = (time.perf_counter() - t0) * (n / nv)
        b = min(blk, m)
        w = np.ascontiguousarray(oracle.weights(d, oracle.WINNING_VOTES)[:b, :b])
        del d
        t0 = time.perf_counter()
        p = oracle.closure(w)
        oracle.rank(p)
        t_blk = time.perf_counter() - t0
        t_close = t_blk * (m / b) ** 3
        return nv, b, t_count, t_blk, t_close

    nv, b, t_count, t_blk, t_close = leg(count_voters, block)
    out["value"] = m ** 3 / t_close / 1e9
    out["seconds_per_step"] = t_count + t_close
    out["sample"] = (f"count over the first {nv} of {n} ballots ({t_count:.1f} s scaled to n); closure + ranking "
                     f"of the leading {b} x {b} block of the weights ({t_blk:.1f} s), scaled by (m/{b})^3 "
                     f"to {t_close:.0f} s; value = m^3 / scaled closure time")
    prev = oracle.set_threads(1)
    try:
        nv1, b1, t_count1, t_blk1, t_close1 = leg(count_voters_1t, block_1t)
    finally:
        oracle.set_threads(prev)
    out["single_thread"] = {
        "value": m ** 3 / t_close1 / 1e9, "unit": "Gop/s", "cores": 1, "extrapolated": True,
        "seconds_per_step": t_count1 + t_close1,
        "sample": (f"count over the first {nv1} ballots ({t_count1:.1f} s scaled); closure + ranking of the "
                   f"leading {b1} x {b1} block ({t_blk1:.1f} s) scaled by (m/{b1})^3"),
    }
    return out


def cpu_baseline_learned(wl, count_voters=4000, block=2048):
    """The oracle's own exact route to the winner set of the m=32768 election
    on a bounded sample: the count over the first ballots (scaled to n),
    weights, one single-source and one single-target widest path (dense
    Dijkstra, the check the GPU's verify makes), and the closure of the
    leading block of the weights scaled by (m/block)^3 for the full-closure
    route."""
    import numpy as np

    import oracle
    m, n = wl.m, wl.n
    nv = min(count_voters, n)
    t0 = time.perf_counter()
    d = oracle.pairwise(wl.ballots[:nv], m)
    t_count = (time.perf_counter() - t0) * (n / nv)
    t0 = time.perf_counter()
    w = oracle.weights(d, oracle.WINNING_VOTES)
    t_w = time.perf_counter() - t0
    del d
    c = int(np.argmax((w > 0).sum(axis=1)))
    t0 = time.perf_counter()
    oracle.widest_from(w, c)
    oracle.widest_to(w, c)
    t_verify = time.perf_counter() - t0
    blk = np.ascontiguousarray(w[:block, :block])
    del w
    t0 = time.perf_counter()
    oracle.closure(blk)
    t_blk = time.perf_counter() - t0
    t_close = t_blk * (m / block) ** 3
    t_route = t_count + t_w + t_verify
    return {"value": t_route, "unit": "s/election", "cores": oracle_threads(), "kind": "oracle", **host_cpu(),
            "extrapolated": True,
            "full_closure_route_s": t_count + t_w + t_close,
            "sample": (f"count over the first {nv} of {n} ballots ({t_count:.1f} s scaled to n), weights "
                       f"({t_w:.1f} s), widest paths from and to one candidate ({t_verify:.1f} s): the oracle's "
                       f"exact check of one proposal; full-closure route: closure of the leading {block} x "
                       f"{block} block ({t_blk:.1f} s) scaled by (m/{block})^3 = {t_close:.0f} s")}


# --------------------------------------------------------------------------- single election

CLOSURE_KERNELS = ("weights", "fw_diag", "fw_panel", "fw_rest", "fw_persist", "fw_store", "value_rank")
COUNT_KERNELS = ("ballot_scan", "route", "ballot_scatter", "count_dense", "count_trunc", "count_sparse",
                 "count_finish")
STEP_KERNELS = COUNT_KERNELS + CLOSURE_KERNELS + ("beaten_by", "rank_sort", "winners", "fill")


def bench_single(args, wl):
    """The whole single-election path, `args.steps` timed steps."""
    import numpy as np
    import torch

    import paper_2505_12976_amd as sz

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    m, n = wl.m, wl.n
    ballots = torch.from_numpy(wl.ballots).to(dev)
    ctx = sz.Context(0)
    ctx.set_closure_schedule(args.closure_schedule)
    dcode = wl.d_dtype
    tdtype = torch.uint16 if dcode == "u16" else torch.int32
    d = torch.empty((m, m), dtype=tdtype, device=dev)
    p = torch.empty((m, m), dtype=tdtype, device=dev)
    is_w = torch.empty(m, dtype=torch.uint8, device=dev)
    order = torch.empty(m, dtype=torch.int32, device=dev)

    def step():
        ctx.pairwise(ballots, m, dtype=dcode, out=d)
        ctx.closure(d, "winning_votes", out=p)
        w, _ = ctx.winners(p)
        o, _ = ctx.ranking(p)
        return w, o

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if ctx.device_error() != 0:
        raise RuntimeError("device error during warmup")
    say(f"{wl.name}: warmup done ({args.warmup} steps)")
    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        w_out, o_out = step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ctx.set_timing(False)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    say(f"{wl.name}: timed {args.steps} steps, {ms_per_step:.3f} ms/step")
    if ctx.device_error() != 0:
        raise RuntimeError("device error")

    kern = {}
    for nm in STEP_KERNELS:
        launches, total = ctx.kernel_time(nm)
        if launches:
            kern[nm] = {"launches_per_step": launches / args.steps, "ms_per_step": total / args.steps,
                        "avg_launch_ms": total / launches}
    closure_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in CLOSURE_KERNELS)
    count_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in COUNT_KERNELS)
    bits = ctx.closure_value_bits()
    ranked = dcode == "i32" and bits == 16
    # the persistent closure kernel: uint16 (or ranks) 1 lane-op per update
    # (v_pk_min_u16 + v_pk_max_u16 on two columns); int32 1.5 (v_min_i32 on
    # two k, one v_max3_i32).  An int32 closure queues both variants gated by
    # the device's ranking decision; the one not taken returns at once, so the
    # kernel time per closure is the sum of both launches.
    ops_per_update = 1.0 if bits == 16 else 1.5
    persist_ms = kern.get("fw_persist", {}).get("ms_per_step", 0.0)
    roof = None
    if persist_ms > 0:
        ach = m ** 3 * ops_per_update / (persist_ms / 1e3) / 1e12
        roof = {"bound": "alu", "kernel": "k_fw_persist (%s, %d-bit values)" % ("value ranks" if ranked else dcode,
                                                                                 bits),
                "achieved": ach, "peak": VALU_LANE_OPS / 1e12, "unit": "Tops/s", "frac": ach / (VALU_LANE_OPS / 1e12),
                "traffic": measured_traffic("fw_persist", wl.name),
                "kernel_ms_per_closure": persist_ms, "updates_per_s": m ** 3 / (persist_ms / 1e3),
                "lane_ops_per_update": ops_per_update,
                "work": f"m^3 = {m ** 3:.3e} max-min updates x {ops_per_update} lane-ops"}
    out = {
        "metric": METRIC,
        "value": m ** 3 / (closure_ms / 1e3) / 1e9 if closure_ms > 0 else None,
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
                   "parallelism": "single GPU", "closure_schedule": args.closure_schedule,
                   "closure_values": "%d-bit%s" % (bits, " ranks of the int32 weights" if ranked else "")},
        "value_is": "m^3 / closure time per step (weights + value ranking + persistent kernel + store)",
        "step_gops": m ** 3 / (ms_per_step / 1e3) / 1e9,
        "elections_per_s": 1e3 / ms_per_step,
        "closure_ms": closure_ms,
        "count_ms": count_ms,
        "kernels": kern,
        "roofline": roof,
    }
    if dcode == "i32" and "count_sparse" in kern and wl.ballots.shape[1] < m - 1:
        # sparse count: ballots read once (n x L int ids) + d written once
        alg = wl.ballots.nbytes + 4 * m * m
        ach = alg / (count_ms / 1e3)
        out["roofline_count"] = {"bound": "hbm", "kernel": "count (scan, route, bucketed pairs, finish)",
                                 "achieved": ach / 1e9, "peak": HBM_BYTES / 1e9, "unit": "GB/s",
                                 "frac": ach / HBM_BYTES, "algorithmic_bytes": alg, "ms_per_step": count_ms,
                                 "traffic": measured_traffic("count", wl.name)}
    if not args.no_oracle_check:
        gold = golden(wl.name)
        if gold is not None:
            say(f"{wl.name}: comparing with the oracle's stored results")
            torch.cuda.synchronize()
            chk = {"d": digest(d.cpu().numpy()) == gold["d_sha256"]}
            if "p_sha256" in gold:
                chk["p"] = digest(p.cpu().numpy()) == gold["p_sha256"]
            chk["winners"] = np.nonzero(w_out.cpu().numpy())[0].tolist() == gold["winners"]
            if "order" in gold:
                chk["order"] = o_out.cpu().numpy().tolist() == gold["order"]
            out["equal_to_oracle"] = chk
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * src.element_size()
        del src, dst
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
    out["valu_probe"] = valu_probe(ctx)
    ctx.close()
    del d, p, ballots
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        say(f"{wl.name}: timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline_single(wl)
    return out


# --------------------------------------------------------------------------- learned

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
    d = torch.empty((m, m), dtype=torch.int32, device=dev)
    steps = max(args.steps, 1)
    ctx.pairwise(ballots, m, dtype="i32", out=d)  # warm-up (workspace)
    torch.cuda.synchronize()
    t_count = []
    for _ in range(3):
        t0 = time.perf_counter()
        ctx.pairwise(ballots, m, dtype="i32", out=d)
        torch.cuda.synchronize()
        t_count.append(time.perf_counter() - t0)
    t_count = float(np.median(t_count))
    say(f"learned: count {t_count * 1e3:.2f} ms")

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
    for _ in range(steps):
        t0 = time.perf_counter()
        w_l, st = learned()
        t_learned.append(time.perf_counter() - t0)
    ctx.set_timing(False)
    say(f"learned: learned path {np.median(t_learned) * 1e3:.2f} ms")
    kern = {}
    for nm in ("weights", "feature_rows", "features", "mlp_prepare", "mlp_forward", "propose", "widest", "verdict",
               "fill"):
        launches, total = ctx.kernel_time(nm)
        if launches:
            kern[nm] = {"launches_per_call": launches / steps, "ms_per_call": total / steps,
                        "avg_launch_ms": total / launches}
    if "widest" in kern:
        kern["widest"]["note"] = ("one cooperative launch (after a plain init launch) runs the sweeps of both "
                                  "directions to the fixpoint, forming the weights from d")
    # dominant kernel: the pass that reads d (int32) once for the
    # per-candidate statistics (HBM-bound; nothing of m^2 size is written)
    es = 4
    alg = es * m * m
    roof = None
    if "feature_rows" in kern:
        ach = alg / (kern["feature_rows"]["avg_launch_ms"] / 1e3)
        roof = {"bound": "hbm", "kernel": "k_feature_rows (per-candidate statistics)",
                "achieved": ach / 1e9, "peak": HBM_BYTES / 1e9, "unit": "GB/s", "frac": ach / HBM_BYTES,
                "traffic": measured_traffic("feature_rows", wl.name), "algorithmic_bytes": alg,
                "work": "d read once: 4 m^2 bytes"}
    if args.learned_path_only:
        ctx.close()
        return {"metric": "learned path only (profiling run)", "ms_learned": float(np.median(t_learned)) * 1e3,
                "ms_count": t_count * 1e3, "kernels_learned": kern, "roofline": roof, "learned_stats": st}
    ctx.reset_timing()
    full()  # warm-up (workspace)
    t_full = []
    for _ in range(2):
        t0 = time.perf_counter()
        w_f = full()
        t_full.append(time.perf_counter() - t0)
    say(f"learned: full closure + winners {min(t_full) * 1e3:.1f} ms")

    # the label-propagation winners algorithm of Section 4 on the same counts
    def propagate():
        w, nw, st = ctx.winners_propagate(d)
        torch.cuda.synchronize()
        return w, st

    propagate()  # warm-up
    t_prop = []
    for _ in range(steps):
        t0 = time.perf_counter()
        w_p, st_p = propagate()
        t_prop.append(time.perf_counter() - t0)
    say(f"learned: label propagation {np.median(t_prop) * 1e3:.2f} ms")
    # the closure without value ranking (int32 arithmetic throughout)
    ctx.set_value_ranking(False)
    t0 = time.perf_counter()
    w_i = full()
    t_full_i32 = time.perf_counter() - t0
    ctx.set_value_ranking(True)
    say(f"learned: full closure, int32 values {t_full_i32 * 1e3:.1f} ms")
    w_f_np = w_f.cpu().numpy()
    tl, tf, tp = float(np.median(t_learned)), float(min(t_full)), float(np.median(t_prop))
    out = {
        "metric": "learned-verify vs full-closure speedup",
        "value": tf / tl,
        "unit": "x",
        "value_is": "(full closure + winners) / (learned path: weights, features, network, verify, climbs, "
                    "tied checks), counts already computed",
        "speedup_with_count": (t_count + tf) / (t_count + tl),
        "steps": steps,
        "dtype": "i32",
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
        "learned_stats": st,
        "winners": np.nonzero(w_l.cpu().numpy())[0].tolist(),
        "equal_to_full_closure": {"learned": bool((w_l.cpu().numpy() == w_f_np).all()),
                                  "label_propagation": bool((w_p.cpu().numpy() == w_f_np).all()),
                                  "int32_closure": bool((w_i.cpu().numpy() == w_f_np).all())},
    }
    if not args.no_oracle_check:
        gold = golden(wl.name)
        if gold is not None:
            out["equal_to_oracle"] = {"d": digest(d.cpu().numpy()) == gold["d_sha256"],
                                      "winners": out["winners"] == gold["winners"]}
    ctx.close()
    del d, ballots
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        say("learned: timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline_learned(wl)
    return out


# --------------------------------------------------------------------------- batch

def bench_batch(args):
    """4096 independent elections (m ~ U{8..512}, n ~ U{50..20000}, full
    Mallows rankings with phi ~ U[0.5, 1]) in one persistent launch replayed
    from a captured HIP graph, against one pass of per-election calls
    (pairwise, closure, winners, ranking for each election in turn)."""
    import numpy as np
    import torch

    import paper_2505_12976_amd as sz
    import workload
    from paper_2505_12976_amd.batch import Packed, alloc_outputs, tuned_closures

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    E = args.batch_elections
    t0 = time.time()
    flat, desc, (ms, ns, phis) = workload.batch_mallows(
        1004, E, progress=lambda k: say(f"batch: {k} of {E} elections generated ({time.time() - t0:.0f} s)"))
    say(f"batch: {E} elections generated in {time.time() - t0:.1f}s ({flat.nbytes / 1e9:.1f} GB of ballots)")
    packed = Packed(flat, desc, int(np.sum(ms * ms)), int(np.sum(ms)))
    ctx = sz.Context(0)
    ballots = torch.from_numpy(flat).to(dev)
    del flat
    t0 = time.time()
    tuned, from_file = tuned_closures(ctx, 16, int(ms.max()))
    say(f"batch: closure schedules {'read from the tuning file' if from_file else 'autotuned'} "
        f"in {time.time() - t0:.1f}s: {tuned}")
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
    steps = max(args.steps, 1)
    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ctx.set_timing(False)
    ms_per_step = (t_end - t_start) * 1e3 / steps
    launches, total = ctx.kernel_time("batch")
    kernel_ms = total / max(launches, 1)
    say(f"batch: {ms_per_step:.2f} ms per step (graph {kernel_ms:.2f} ms)")

    # per-election launches: the same outputs, election by election
    t_per, same = None, None
    if not args.no_per_election:
        d_ref = torch.empty_like(outs["d"])
        p_ref = torch.empty_like(outs["p"])
        w_ref = torch.empty_like(outs["is_winner"])
        o_ref = torch.empty_like(outs["order"])
        bb_ref = torch.empty_like(outs["beaten_by"])

        def per_election():
            for e, (bo, n, L, m, mo, vo) in enumerate(desc):
                b = ballots[bo:bo + n * L].view(n, L)
                dd = ctx.pairwise(b, m, dtype="i32", out=d_ref[mo:mo + m * m].view(m, m))
                pp = ctx.closure(dd, "winning_votes", out=p_ref[mo:mo + m * m].view(m, m))
                w, _ = ctx.winners(pp)
                order, beaten = ctx.ranking(pp)
                w_ref[vo:vo + m].copy_(w)
                o_ref[vo:vo + m].copy_(order)
                bb_ref[vo:vo + m].copy_(beaten)

        per_election()  # warm-up (workspace growth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_election()
        torch.cuda.synchronize()
        t_per = time.perf_counter() - t0
        same = bool(torch.equal(d_ref, outs["d"]) and torch.equal(p_ref, outs["p"]) and
                    torch.equal(w_ref, outs["is_winner"]) and torch.equal(o_ref, outs["order"]) and
                    torch.equal(bb_ref, outs["beaten_by"]))
        say(f"batch: per-election calls {t_per * 1e3:.1f} ms, identical outputs: {same}")
        del d_ref, p_ref, w_ref, o_ref, bb_ref
    if ctx.device_error() != 0:
        raise RuntimeError("device error")
    oracle_equal = None
    gold = None if args.no_oracle_check else golden("batch_mallows_E%d" % E)
    if gold is not None:
        say("batch: comparing every election with the oracle's stored digests")
        d_all, p_all = outs["d"].cpu().numpy(), outs["p"].cpu().numpy()
        w_all = outs["is_winner"].cpu().numpy().astype(np.int64)
        bb_all, o_all = outs["beaten_by"].cpu().numpy(), outs["order"].cpu().numpy()
        nw_all = outs["n_winners"].cpu().numpy()
        bad = 0
        for e, (bo, n, L, m, mo, vo) in enumerate(desc):
            h = hashlib.sha256()
            for a in (bb_all[vo:vo + m], w_all[vo:vo + m], o_all[vo:vo + m]):
                h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
            got = [digest(d_all[mo:mo + m * m])[:32], digest(p_all[mo:mo + m * m])[:32], h.hexdigest()[:32],
                   int(nw_all[e])]
            bad += got != gold["elections"][e]
        oracle_equal = {"elections": E, "differing": int(bad)}
        del d_all, p_all
    # algorithmic work: one VALU lane-op per (voter, candidate pair) of the count,
    # one per packed max-min update of the closure
    count_ops = float(np.sum(ns * ms * (ms - 1) / 2))
    closure_ops = float(np.sum(ms.astype(np.float64) ** 3))
    work = count_ops + closure_ops
    ach = work / (kernel_ms / 1e3) / 1e12
    roof = {"bound": "alu", "kernel": "k_batch (graph replay)", "achieved": ach, "peak": VALU_LANE_OPS / 1e12,
            "unit": "Tops/s", "frac": ach / (VALU_LANE_OPS / 1e12),
            "traffic": measured_traffic("batch", "batch_mallows_E%d" % E),
            "work": "1 lane-op per (voter, unordered pair) of the count + 1 per packed max-min update"}
    out = {
        "metric": "elections/sec",
        "value": E / (ms_per_step / 1e3),
        "unit": "elections/s",
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "dtype": "i32",
        "config": {"workload": "batch_mallows_E%d" % E, "elections": E, "m": "U{8..512}", "n": "U{50..20000}",
                   "phi": "U[0.5,1.0]", "seed": 1004, "weight_mode": "winning_votes",
                   "launch": "one persistent kernel per step, replayed from a captured HIP graph"},
        "elections_per_s_per_election_calls": E / t_per if t_per else None,
        "speedup_vs_per_election_calls": t_per / (ms_per_step / 1e3) if t_per else None,
        "ms_per_election_calls_pass": t_per * 1e3 if t_per else None,
        "identical_to_per_election_calls": same,
        "equal_to_oracle": oracle_equal,
        "graph_ms": kernel_ms,
        "count_comparisons": count_ops,
        "closure_updates": closure_ops,
        "closure_schedule_by_bucket": tuned,
        "closure_schedules_from_tuning_file": from_file,
        "roofline": roof,
    }
    plan.destroy()
    ctx.close()
    del ballots, outs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle
        say("batch: timing the CPU oracle on a sample of elections")
        t0 = time.perf_counter()
        k = 0
        while k < E and time.perf_counter() - t0 < 10.0:
            b = workload.batch_election(1004, k, int(ms[k]), int(ns[k]), float(phis[k]))
            oracle.schulze(b, int(ms[k]))
            k += 1
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": k / t_cpu, "unit": "elections/s", "cores": oracle_threads(),
                               "kind": "oracle", **host_cpu(),
                               "sample": f"the first {k} of the {E} elections, whole path per election "
                                         f"({t_cpu:.1f} s; ballot generation excluded)"}
    return out


# --------------------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; runs on more than one GPU are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}), flush=True)
        sys.exit(1)
    if args.workload == "learned":
        out = bench_learned(args)
        out.update({"n_gpus": 1, "higher_is_better": True, "data": "synthetic"})
    elif args.workload == "batch":
        out = bench_batch(args)
        out.update({"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "data": "synthetic"})
    elif args.workload in ("mid", "small", "paper", "large"):
        t0 = time.time()
        wl = make_workload(args.workload)
        say(f"workload {wl.name} generated in {time.time() - t0:.1f}s")
        out = bench_single(args, wl)
    else:
        parts = [p for p in args.parts.split(",") if p]
        bad = [p for p in parts if p not in PARTS]
        if bad or "headline" not in parts:
            print(json.dumps({"error": f"--parts must include headline and only {PARTS}"}), flush=True)
            sys.exit(2)
        t0 = time.time()
        wl = make_workload("large")
        say(f"workload {wl.name} generated in {time.time() - t0:.1f}s")
        out = bench_single(args, wl)
        if "learned" in parts:
            out["learned"] = bench_learned(args)
        if "batch" in parts:
            out["batch"] = bench_batch(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
