"""What the trained proposer gains over plain proposals, measured on the
whole exact learned path.

For each election and each proposer (the network; Borda, the vertex order
Section 4 suggests; Copeland; the Section 4 initialisation filter followed
by Borda) the library's schulze_winners_learned runs end to end (weights,
features, scores, verification, climbs, tied checks, fallback) and is timed;
the winner sets of all proposers must agree (the verification makes them
exact).  Results are split by whether the election has a Condorcet winner.

    python -m paper_2505_12976_amd.proposer_gain --out gpurun_out/proposer_gain.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PROPOSERS = ("network", "borda", "copeland", "filter+borda")


def run_election(ctx, params, ballots, m, n, repeats=1):
    """{proposer: {ms, first_hit, verify_calls, climbs, fallback}} and the
    Condorcet flag for one election; raises if the winner sets differ."""
    import torch
    b = torch.from_numpy(np.ascontiguousarray(ballots)).cuda()
    d = ctx.pairwise(b, m, dtype="u16" if n <= 65535 else "i32")
    feat = ctx.features(d, float(n))
    cope = np.rint(feat[:, 0].cpu().numpy() * max(m - 1, 1)).astype(np.int64)
    condorcet = bool(m > 1 and (cope == m - 1).any())
    out, ref = {}, None
    try:
        for prop in PROPOSERS:
            ctx.set_proposer(prop)
            ctx.winners_learned(d, float(n), params)  # warm-up
            best = None
            for _ in range(repeats):
                t0 = time.perf_counter()
                w, nw, st = ctx.winners_learned(d, float(n), params)
                torch.cuda.synchronize()  # the winner set is written by the call's last queued launch
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            win = w.cpu().numpy().astype(bool)
            if ref is None:
                ref = win
            elif not np.array_equal(ref, win):
                raise AssertionError(f"{prop}: winner set differs from the network's")
            out[prop] = {"ms": best * 1e3, "first_hit": st["first_hit"], "verify_calls": st["verify_calls"],
                         "climbs": st["climbs"], "fallback": st["fallback"]}
    finally:
        ctx.set_proposer("network")
    return out, condorcet, ref


def summarise(rows):
    """rows: list of (per-proposer dict, condorcet flag) -> strata summary."""
    strata = {"all": rows, "condorcet": [r for r in rows if r[1]], "no_condorcet": [r for r in rows if not r[1]]}
    out = {}
    for key, lst in strata.items():
        s = {"elections": len(lst)}
        for prop in PROPOSERS:
            if not lst:
                s[prop] = None
                continue
            vals = [r[0][prop] for r in lst]
            s[prop] = {"first_hit_rate": float(np.mean([v["first_hit"] for v in vals])),
                       "mean_verify_calls": float(np.mean([v["verify_calls"] for v in vals])),
                       "mean_climbs": float(np.mean([v["climbs"] for v in vals])),
                       "fallbacks": int(np.sum([v["fallback"] for v in vals])),
                       "mean_ms": float(np.mean([v["ms"] for v in vals])),
                       "total_ms": float(np.sum([v["ms"] for v in vals]))}
        out[key] = s
    return out


def study(ctx, params, no_condorcet=500, heldout=600, big=32, log=None):
    """The held-out training mixture (seed 3005), elections near impartial
    culture until `no_condorcet` of them lack a Condorcet winner (seed 3105),
    and `big` elections of the m=32768 workload's shape (seed 3005)."""
    import workload
    rows_mix, rows_nc, rows_big = [], [], []
    for el in workload.training_mixture(3005, heldout):
        r, cw, _ = run_election(ctx, params, el["ballots"], el["m"], el["n"])
        rows_mix.append((r, cw))
        if log and len(rows_mix) % 200 == 0:
            log(f"held-out mixture: {len(rows_mix)} elections")
    if log:
        log(f"held-out mixture: {len(rows_mix)} elections")
    seen = 0
    for el in workload.near_impartial_mixture(3105, 10 * no_condorcet):
        r, cw, _ = run_election(ctx, params, el["ballots"], el["m"], el["n"])
        seen += 1
        if not cw:
            rows_nc.append((r, cw))
        if log and seen % 200 == 0:
            log(f"near-impartial: {seen} elections, {len(rows_nc)} without a Condorcet winner")
        if len(rows_nc) >= no_condorcet:
            break
    if log:
        log(f"near-impartial: {len(rows_nc)} elections without a Condorcet winner")
    for e in range(big):
        b = workload.pl_zipf(3005, 200_000, 32768, 1.0, 30, election=e)
        r, cw, _ = run_election(ctx, params, b, 32768, 200_000, repeats=3)
        rows_big.append((r, cw))
        if log:
            log(f"m=32768 election {e}: " + ", ".join(f"{p} {r[p]['ms']:.2f} ms" for p in PROPOSERS))
    return {"heldout_mixture": summarise(rows_mix), "no_condorcet_near_impartial": summarise(rows_nc),
            "plzipf_m32768_n200000_top30_x%d" % big: summarise(rows_big)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-condorcet", type=int, default=500)
    ap.add_argument("--heldout", type=int, default=600)
    ap.add_argument("--big", type=int, default=32)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.proposer import load_checkpoint
    ckpt = os.path.join(ROOT, "paper_2505_12976_amd", "data", "proposer.npz")
    params = torch.from_numpy(load_checkpoint(ckpt)["params"]).cuda()
    ctx = sz.Context(0)
    t0 = time.time()
    res = study(ctx, params, args.no_condorcet, args.heldout, args.big,
                log=lambda msg: print(f"[gain] {msg} ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True))
    ctx.close()
    line = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
