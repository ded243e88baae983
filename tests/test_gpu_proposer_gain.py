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
