"""Train the winner proposer on elections labelled by the exact GPU path.

    python -m paper_2505_12976_amd.train_proposer --train 20000 --heldout 2000 \
        --out paper_2505_12976_amd/data/proposer.npz

Training elections come from ``workload.training_mixture`` (m ~ U{256..2048},
n = rho m with rho ~ U[3, 12], half Plackett-Luce Zipf top-k, half Mallows
top-k).  Each election's label is its Schulze winner set from the library
(counts -> closure -> winners); its input is the library's feature matrix.
After training, the held-out elections (another seed) compare the first
proposal's hit rate of the network with Borda, Copeland and the
initialisation filter followed by Borda, split by whether a Condorcet winner
exists.  Prints one JSON line with the summary.
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


def label_election(ctx, ballots: np.ndarray, m: int, n: int):
    """(features (m,16) CUDA f32, winner mask (m,) CUDA u8) from ballots."""
    import torch
    b = torch.from_numpy(np.ascontiguousarray(ballots)).cuda()
    d = ctx.pairwise(b, m, dtype="u16" if n <= 65535 else "i32")
    p = ctx.closure(d)
    win, _ = ctx.winners(p)
    feat = ctx.features(d, float(n))
    return feat, win


def evaluate(ctx, params, elections) -> dict:
    """Hit rates of the first proposal for several proposers."""
    from paper_2505_12976_amd.proposer import filtered_argmax
    import torch
    pt = torch.from_numpy(np.asarray(params, dtype=np.float32)).cuda()
    rows = {"all": [], "condorcet": [], "no_condorcet": []}
    for feat, win in elections:
        f = feat.cpu().numpy()
        w = win.cpu().numpy().astype(bool)
        s = ctx.mlp_forward(pt, feat).cpu().numpy()
        m = f.shape[0]
        cope = np.rint(f[:, 0] * max(m - 1, 1)).astype(np.int64)
        has_cw = bool((cope == m - 1).any()) and m > 1
        hits = {
            "network": w[filtered_argmax(s, f)],
            "borda": w[int(np.argmax(f[:, 2]))],
            "copeland": w[int(np.argmax(f[:, 0]))],
            "filter+borda": w[filtered_argmax(f[:, 2], f)],
        }
        for key in ("all", "condorcet" if has_cw else "no_condorcet"):
            rows[key].append(hits)
    out = {}
    for key, lst in rows.items():
        out[key] = {"elections": len(lst)}
        for name in ("network", "borda", "copeland", "filter+borda"):
            out[key][name] = float(np.mean([h[name] for h in lst])) if lst else None
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--heldout", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=2005)
    ap.add_argument("--heldout-seed", type=int, default=3005)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2505_12976_amd", "data", "proposer.npz"))
    args = ap.parse_args(argv)

    import workload
    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.proposer import Trainer

    def log(msg):
        print(f"[train] {msg}", file=sys.stderr, flush=True)

    ctx = sz.Context(0)
    trainer = Trainer(ctx, seed=args.seed)
    t0 = time.time()
    for el in workload.training_mixture(args.seed, args.train):
        feat, win = label_election(ctx, el["ballots"], el["m"], el["n"])
        trainer.add(feat, win)
        if (el["election"] + 1) % 1000 == 0:
            log(f"labelled {el['election'] + 1} elections ({time.time() - t0:.0f}s)")
    t_label = time.time() - t0
    t0 = time.time()
    history = trainer.fit(epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    t_fit = time.time() - t0
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    meta = {"train_elections": args.train, "seed": args.seed, "epochs": args.epochs, "batch": args.batch,
            "lr": args.lr, "recipe": "workload.training_mixture(seed, count)"}
    trainer.save(args.out, meta)
    held = []
    for el in workload.training_mixture(args.heldout_seed, args.heldout):
        held.append(label_election(ctx, el["ballots"], el["m"], el["n"]))
    res = evaluate(ctx, trainer.params.cpu().numpy(), held)
    print(json.dumps({"train_elections": args.train, "rows": int(trainer.offsets_host[-1]),
                      "label_seconds": t_label, "fit_seconds": t_fit, "loss_per_epoch": history,
                      "steps": trainer.step, "heldout": res, "checkpoint": os.path.relpath(args.out, ROOT)}),
          flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
