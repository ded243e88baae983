"""Write the stored expected results for the full-size workloads.

Calls only the CPU oracle (``oracle``) and the input generators
(``workload``); nothing here touches the GPU library.  For each workload it
stores SHA-256 digests of d and p (int64, little-endian, row-major), per-row
sums of d and p (to locate a mismatch), beaten_by, the winner set and the
ranking.

    python tests/golden/make_golden.py mid      # m=4096 workload
    python tests/golden/make_golden.py large    # m=16384 workload (about an hour)
    python tests/golden/make_golden.py learned  # m=32768 workload: winners certified
                                                # by widest paths (a few minutes)
    python tests/golden/make_golden.py batch    # all 4096 batch elections (minutes)

At m=32768 the plain closure is out of reach on the CPU (3.5e13 updates), so
the winner set is certified the way Section 3 shows membership in NL:
single-source and single-target widest paths from one candidate decide
whether anyone beats it.  Beats is a strict partial order, so moving to a
beater until none is left ends at a winner; every winner is tied with every
other, so the winner set is that candidate plus the tied candidates that
pass the same check.  Rows and columns of p for those candidates and for a
seeded sample are stored as digests.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(a: np.ndarray, rows_per_chunk: int = 1024) -> str:
    """SHA-256 of the array as int64, little-endian, row-major (hashed in
    row chunks, which gives the same digest as hashing it whole)."""
    h = hashlib.sha256()
    a = np.asarray(a)
    if a.ndim < 2:
        h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
        return h.hexdigest()
    for i in range(0, a.shape[0], rows_per_chunk):
        h.update(np.ascontiguousarray(a[i:i + rows_per_chunk], dtype="<i8").tobytes())
    return h.hexdigest()


def certify_winners(w: np.ndarray, start: int, max_tied: int = 4096):
    """Winner set from single-source/target widest paths only (see above).
    Returns (winners, the first winner found, its tied candidates, climb path,
    {candidate: (row digest, column digest)} for every candidate checked)."""
    m = w.shape[0]
    checked = {}

    def check(c):
        pf = oracle.widest_from(w, c)   # p(c, x)
        pt = oracle.widest_to(w, c)     # p(x, c)
        checked[c] = (digest(pf), digest(pt))
        return pf, pt

    c, path = start, [start]
    while True:
        pf, pt = check(c)
        beaters = np.nonzero(pt > pf)[0]
        if len(beaters) == 0:
            break
        c = int(beaters[np.argmax(pt[beaters] - pf[beaters])])
        path.append(c)
        assert len(path) <= m, "beats must be acyclic"
    ids = np.arange(m)
    tied = [int(t) for t in np.nonzero((pf == pt) & (ids != c))[0]]
    assert len(tied) <= max_tied, f"{len(tied)} candidates tied with the winner"
    winners = [c]
    for t in tied:
        tf, tt = check(t)
        if not (tt > tf).any():
            winners.append(t)
    return sorted(winners), c, tied, path, checked


def run(name: str) -> None:
    t0 = time.time()
    wl = {"mid": workload.plain_mid, "large": workload.plain_large}[name]()
    print(f"[{name}] generated {wl.ballots.shape} in {time.time() - t0:.1f}s", flush=True)
    t = time.time()
    d = oracle.pairwise(wl.ballots, wl.m)
    print(f"[{name}] count {time.time() - t:.1f}s", flush=True)
    w = oracle.weights(d, oracle.WINNING_VOTES)
    t = time.time()
    p = oracle.closure(w)
    print(f"[{name}] closure {time.time() - t:.1f}s", flush=True)
    beaten, win, order = oracle.rank(p)
    out = {
        "workload": wl.name,
        "recipe": wl.recipe,
        "m": wl.m,
        "n": wl.n,
        "weight_mode": "winning_votes",
        "ballots_sha256": hashlib.sha256(np.ascontiguousarray(wl.ballots).tobytes()).hexdigest(),
        "d_sha256": digest(d),
        "p_sha256": digest(p),
        "d_row_sums": [int(x) for x in d.sum(axis=1)],
        "p_row_sums": [int(x) for x in p.sum(axis=1)],
        "d_max": int(d.max()),
        "beaten_by": [int(x) for x in beaten],
        "winners": [int(x) for x in np.nonzero(win)[0]],
        "order": [int(x) for x in order],
        "generated_by": "tests/golden/make_golden.py (oracle only)",
    }
    path = os.path.join(HERE, f"{wl.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"[{name}] wrote {path} in {time.time() - t0:.1f}s total", flush=True)


def run_learned() -> None:
    t0 = time.time()
    wl = workload.plain_learned()
    m = wl.m
    print(f"[learned] generated {wl.ballots.shape} in {time.time() - t0:.1f}s", flush=True)
    t = time.time()
    d = oracle.pairwise(wl.ballots, m)
    print(f"[learned] count {time.time() - t:.1f}s", flush=True)
    d_sha, d_rows, d_max = digest(d), [int(x) for x in d.sum(axis=1)], int(d.max())
    w = oracle.weights(d, oracle.WINNING_VOTES)
    # start the climb at the candidate with the most pairwise wins (any start
    # gives the same certified set; this one needs few steps)
    wins = (w > 0).sum(axis=1)
    del d
    start = int(np.argmax(wins))
    t = time.time()
    winners, first, tied, path, checked = certify_winners(w, start)
    print(f"[learned] winners {winners} (climb {path}, {len(tied)} tied) in {time.time() - t:.1f}s", flush=True)
    # a seeded sample of further rows and columns of p
    rng = np.random.default_rng(5005)
    sample = sorted(set(int(x) for x in rng.choice(m, 8, replace=False)) | {0, m - 1})
    for c in sample:
        if c not in checked:
            checked[c] = (digest(oracle.widest_from(w, c)), digest(oracle.widest_to(w, c)))
    out = {
        "workload": wl.name,
        "recipe": wl.recipe,
        "m": m,
        "n": wl.n,
        "weight_mode": "winning_votes",
        "ballots_sha256": hashlib.sha256(np.ascontiguousarray(wl.ballots).tobytes()).hexdigest(),
        "d_sha256": d_sha,
        "d_row_sums": d_rows,
        "d_max": d_max,
        "winners": winners,
        "first_winner": first,
        "climb": path,
        "tied_with_first_winner": tied,
        "p_rows_cols": {str(c): {"row_sha256": r, "col_sha256": cc} for c, (r, cc) in sorted(checked.items())},
        "certified_by": "single-source/target widest paths (oracle.widest_from/_to), Section 3",
        "generated_by": "tests/golden/make_golden.py (oracle only)",
    }
    path = os.path.join(HERE, f"{wl.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"[learned] wrote {path} in {time.time() - t0:.1f}s total", flush=True)


def election_digests(res: dict) -> dict:
    """Per-election digests: d, p, and the ranking outputs together."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(res["beaten_by"], dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(res["is_winner"], dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(res["order"], dtype="<i8").tobytes())
    return {"d": digest(res["d"])[:32], "p": digest(res["p"])[:32], "rank": h.hexdigest()[:32]}


def run_batch(count: int = 4096, seed: int = 1004) -> None:
    t0 = time.time()
    ms, ns, phis = workload.batch_params(seed, count)
    els = []
    for e in range(count):
        b = workload.batch_election(seed, e, int(ms[e]), int(ns[e]), float(phis[e]))
        res = oracle.schulze(b, int(ms[e]), oracle.WINNING_VOTES)
        dg = election_digests(res)
        els.append([dg["d"], dg["p"], dg["rank"], int(res["is_winner"].sum())])
        if e % 256 == 255:
            print(f"[batch] {e + 1} elections in {time.time() - t0:.1f}s", flush=True)
    out = {
        "workload": f"batch_mallows_E{count}",
        "recipe": f"{count} elections: m ~ U{{8..512}}, n ~ U{{50..20000}}, full Mallows(phi ~ U[0.5, 1]) "
                  f"rankings, seed {seed}",
        "count": count,
        "weight_mode": "winning_votes",
        "m": [int(x) for x in ms],
        "n": [int(x) for x in ns],
        "digest": "per election [d, p, (beaten_by, is_winner, order)]: first 32 hex digits of the SHA-256 of "
                  "the int64 little-endian arrays, plus the number of winners",
        "elections": els,
        "generated_by": "tests/golden/make_golden.py (oracle only)",
    }
    path = os.path.join(HERE, f"batch_mallows_E{count}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"[batch] wrote {path} in {time.time() - t0:.1f}s total", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["mid"]:
        if arg == "learned":
            run_learned()
        elif arg == "batch":
            run_batch()
        else:
            run(arg)
