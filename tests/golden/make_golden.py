"""Write the stored expected results for the full-size workloads.

Calls only the CPU oracle (``oracle``) and the input generators
(``workload``); nothing here touches the GPU library.  For each workload it
stores SHA-256 digests of d and p (int64, little-endian, row-major), per-row
sums of d and p (to locate a mismatch), beaten_by, the winner set and the
ranking.

    python tests/golden/make_golden.py mid      # m=4096 workload
    python tests/golden/make_golden.py large    # m=16384 workload (about an hour)
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


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


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


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["mid"]:
        run(arg)
