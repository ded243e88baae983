"""What the trained proposer gains over the method's own cheap proposals:
first-proposal hit rates on held-out elections (a seed the network never
saw), against Borda (the paper's vertex-id order, Section 4), Copeland and
the initialisation filter followed by Borda."""
import os

import pytest

import workload
from tests.test_gpu_learned import CKPT
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu


def test_trained_network_beats_borda_and_matches_copeland():
    import torch
    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.proposer import load_checkpoint
    from paper_2505_12976_amd.train_proposer import evaluate, label_election
    if not os.path.exists(CKPT):
        pytest.skip("no trained checkpoint")
    ctx = sz.Context(0)
    try:
        held = [label_election(ctx, el["ballots"], el["m"], el["n"])
                for el in workload.training_mixture(4005, 600)]
        res = evaluate(ctx, load_checkpoint(CKPT)["params"], held)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    log(f"[result] hit rates {res}")
    a = res["all"]
    assert a["network"] >= a["borda"] + 0.02
    assert a["network"] >= a["copeland"] - 0.005


def test_network_gain_on_elections_without_condorcet_winner():
    """The whole exact learned path with each proposer on 500 near-impartial
    elections that have no Condorcet winner (seed 3105), stratified, and on
    four elections of the m=32768, n=200000 top-30 shape: every proposer
    reaches the same winner set (the verification makes them exact), and on
    the elections without a Condorcet winner the network's first proposal
    wins clearly more often than Copeland's or Borda's and needs fewer exact
    checks."""
    import torch
    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.proposer import load_checkpoint
    from paper_2505_12976_amd.proposer_gain import run_election, summarise
    if not os.path.exists(CKPT):
        pytest.skip("no trained checkpoint")
    ctx = sz.Context(0)
    try:
        params = torch.from_numpy(load_checkpoint(CKPT)["params"]).cuda()
        rows = []
        for el in workload.near_impartial_mixture(3105, 5000):
            r, cw, _ = run_election(ctx, params, el["ballots"], el["m"], el["n"])  # raises if winner sets differ
            if not cw:
                rows.append((r, cw))
            if len(rows) >= 500:
                break
        big = []
        for e in range(4):
            b = workload.pl_zipf(3005, 200_000, 32768, 1.0, 30, election=e)
            r, cw, _ = run_election(ctx, params, b, 32768, 200_000)
            big.append((r, cw))
        torch.cuda.synchronize()
    finally:
        ctx.close()
    s = summarise(rows)["no_condorcet"]
    log(f"[result] no Condorcet winner, {s['elections']} elections: " +
        ", ".join(f"{p} hit {s[p]['first_hit_rate']:.3f} checks {s[p]['mean_verify_calls']:.3f}"
                  for p in ("network", "copeland", "borda", "filter+borda")))
    assert s["elections"] == 500
    assert s["network"]["first_hit_rate"] >= s["copeland"]["first_hit_rate"] + 0.08
    assert s["network"]["first_hit_rate"] >= s["borda"]["first_hit_rate"] + 0.15
    assert s["network"]["mean_verify_calls"] < s["copeland"]["mean_verify_calls"]
    assert all(r[0][p]["fallback"] == 0 for r in rows + big for p in r[0])
    assert all(r[0][p]["first_hit"] for r in big for p in r[0])  # Condorcet elections: every proposer hits
