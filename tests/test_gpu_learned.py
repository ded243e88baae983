"""The learned path returns exactly the Schulze winner set, whatever the
network proposes: compared with the oracle's winners, for random and trained
parameters, with climbs, tied winners and the closure fallback forced."""
import os

import numpy as np
import pytest

import oracle
import workload
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu

CKPT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2505_12976_amd", "data",
                    "proposer.npz")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def params_list():
    from paper_2505_12976_amd.proposer import init_params, load_checkpoint
    ps = [("random", init_params(5)), ("negated", -init_params(6))]
    if os.path.exists(CKPT):
        ps.append(("trained", load_checkpoint(CKPT)["params"]))
    return ps


def elections():
    yield "mallows-topk", workload.mallows_topk(1, 900, 300, 0.95, 20), 300
    yield "plzipf", workload.pl_zipf(2, 2000, 500, 1.0, 25), 500
    yield "mallows-trunc", workload.mallows(3, 401, 130, 0.9, trunc_mod=3, trunc_lt=1, trunc_k=10), 130
    yield "uniform-ties", workload.uniform_ballots(4, 30, 60, min_len=0), 60
    yield "one-candidate", np.zeros((5, 1), dtype=np.uint16), 1
    yield "opposed", np.stack([workload.permutation(5, 0, 40), workload.permutation(5, 0, 40)[::-1]] * 3
                              ).astype(np.uint16), 40


@pytest.mark.parametrize("which", ["random", "negated", "trained"])
def test_learned_winners_are_exact(ctx, which):
    import torch
    plist = dict(params_list())
    if which not in plist:
        pytest.skip("no trained checkpoint")
    pt = torch.from_numpy(np.asarray(plist[which], dtype=np.float32)).cuda()
    for name, b, m in elections():
        log(f"[case] learned {which} {name} m={m}")
        want = oracle.schulze(b, m)["is_winner"]
        d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype="i32")
        for max_climb, max_tied in ((8, 64), (0, 64), (8, 0)):
            w, nw, st = ctx.winners_learned(d, float(b.shape[0]), pt, max_climb=max_climb, max_tied=max_tied)
            got = w.cpu().numpy().astype(bool)
            assert (got == want).all(), (which, name, max_climb, max_tied, st)
            assert int(nw.cpu()[0]) == int(want.sum()) == st["n_winners"]
            assert st["first_hit"] == int(want[st["proposal"]])
            if st["fallback"] == 0:
                assert want[st["proposal"]] or st["climbs"] > 0


def test_learned_matches_closure_on_mid_workload(ctx):
    """m=4096: the exact check agrees with the stored oracle winners."""
    import json
    import torch
    from tests.test_gpu_parity import GOLD
    wl = workload.plain_mid()
    path = os.path.join(GOLD, wl.name + ".json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle results")
    gold = json.load(open(path))
    d = ctx.pairwise(torch.from_numpy(wl.ballots).cuda(), wl.m, dtype="u16")
    for which, p in params_list():
        pt = torch.from_numpy(np.asarray(p, dtype=np.float32)).cuda()
        w, nw, st = ctx.winners_learned(d, float(wl.n), pt)
        log(f"[case] learned mid workload {which}: {st}")
        assert np.nonzero(w.cpu().numpy())[0].tolist() == gold["winners"]


@pytest.mark.parametrize("proposer", ["borda", "copeland", "filter+borda"])
def test_learned_winners_with_plain_proposers(ctx, proposer):
    """Borda, Copeland or filtered Borda in place of the network: the same
    exact winner sets (the proposal only decides where the search starts)."""
    import torch
    try:
        ctx.set_proposer(proposer)
        for name, b, m in elections():
            log(f"[case] learned proposer={proposer} {name} m={m}")
            want = oracle.schulze(b, m)["is_winner"]
            d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype="i32")
            for max_climb, max_tied in ((8, 64), (0, 64), (8, 0)):
                w, nw, st = ctx.winners_learned(d, float(b.shape[0]), None, max_climb=max_climb,
                                                max_tied=max_tied)
                got = w.cpu().numpy().astype(bool)
                assert np.array_equal(got, want), (proposer, name, max_climb, max_tied, st)
                assert int(nw.cpu()[0]) == int(want.sum())
    finally:
        ctx.set_proposer("network")
    import paper_2505_12976_amd as sz
    assert ctx._lib.schulze_set_proposer(ctx._h, 7) == sz.EINVAL


@pytest.mark.parametrize("mode", ["winning_votes", "margin"])
def test_learned_winners_by_count_width_and_mode(ctx, mode):
    """int32 counts take the signed-weight form of the exact check (one
    matrix S = w - w^T, both directions reading its rows), 16-bit counts the
    w and w^T form: both give the oracle's winners under either weight rule,
    and, as the proposals and every verdict agree, the same search (same
    proposal, climbs and number of checks)."""
    import torch
    from paper_2505_12976_amd.proposer import init_params
    om = oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES
    for which, p in (("random", init_params(7)), ("negated", -init_params(8))):
        pt = torch.from_numpy(np.asarray(p, dtype=np.float32)).cuda()
        for name, b, m in elections():
            log(f"[case] learned {mode} {which} {name} m={m}")
            want = oracle.schulze(b, m, om)["is_winner"]
            for max_climb, max_tied in ((8, 64), (0, 64), (8, 0)):
                stats = {}
                for dtype in ("u16", "i32"):
                    d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype=dtype)
                    w, nw, st = ctx.winners_learned(d, float(b.shape[0]), pt, mode=mode, max_climb=max_climb,
                                                    max_tied=max_tied)
                    got = w.cpu().numpy().astype(bool)
                    assert np.array_equal(got, want), (mode, which, name, dtype, max_climb, max_tied, st)
                    assert int(nw.cpu()[0]) == int(want.sum()) == st["n_winners"]
                    stats[dtype] = st
                assert stats["u16"] == stats["i32"], (mode, which, name, max_climb, max_tied, stats)
