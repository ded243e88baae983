"""Edge weights, single-source/target widest paths and the exact winner check
against the CPU oracle (bit-exact integers)."""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from tests.test_gpu_parity import GOLD, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def to_np(t):
    return t.cpu().numpy().astype(np.int64)


def profile(m, seed):
    kind = seed % 3
    if kind == 0:
        return workload.mallows(seed, 301, m, 0.93, trunc_mod=4, trunc_lt=1, trunc_k=max(1, m // 5))
    if kind == 1:
        return workload.uniform_ballots(seed, 57, m, min_len=0)
    return workload.pl_zipf(seed, 501, m, 1.0, min(m, 12))


@pytest.mark.parametrize("m", [63, 200, 1100])
@pytest.mark.parametrize("dtype", ["u16", "i32"])
def test_weights_strided_and_single_output(ctx, m, dtype):
    """d as a view with row pitch m + 7; w alone and w^T alone."""
    import torch
    b = profile(m, 11 + m)
    dn = oracle.pairwise(b, m)
    wn = oracle.weights(dn, oracle.WINNING_VOTES)
    npdt = np.uint16 if dtype == "u16" else np.int32
    big = np.zeros((m, m + 7), dtype=npdt)
    big[:, :m] = dn.astype(npdt)
    d = torch.from_numpy(big).cuda()[:, :m]
    assert d.stride(0) == m + 7
    w, wt = ctx.weights(d, "winning_votes")
    assert (to_np(w) == wn).all() and (to_np(wt) == wn.T).all()
    w_only, none_t = ctx.weights(d, "winning_votes", transposed=False)
    assert none_t is None and (to_np(w_only) == wn).all()
    none_w, wt_only = ctx.weights(d, "winning_votes", direct=False)
    assert none_w is None and (to_np(wt_only) == wn.T).all()
    p = ctx.closure(d)
    assert (to_np(p) == oracle.closure(wn)).all()
    beaten, win, _ = oracle.rank(oracle.closure(wn))
    order, beaten_gpu = ctx.ranking(p)
    assert (to_np(beaten_gpu) == beaten).all()


@pytest.mark.parametrize("m", [1, 2, 5, 64, 65, 300, 1000])
@pytest.mark.parametrize("dtype,mode", [("u16", "winning_votes"), ("i32", "margin")])
def test_weights_and_widest(ctx, m, dtype, mode):
    import torch
    b = profile(m, 7 + m)
    dn = oracle.pairwise(b, m)
    wn = oracle.weights(dn, oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES)
    pn = oracle.closure(wn)
    d = torch.from_numpy(dn.astype(np.uint16 if dtype == "u16" else np.int32)).cuda()
    w, wt = ctx.weights(d, mode)
    assert (to_np(w) == wn).all() and (to_np(wt) == wn.T).all()
    rng = np.random.default_rng(m)
    for s in sorted(set([0, m - 1] + list(rng.integers(0, m, size=3)))):
        log(f"[case] widest m={m} {dtype} {mode} s={s}")
        row = to_np(ctx.widest_from(w, int(s)))
        col = to_np(ctx.widest_from(wt, int(s)))
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        assert (row == pn[s]).all(), f"p[{s}][:] differs"
        assert (col == pn[:, s]).all(), f"p[:][{s}] differs"


@pytest.mark.parametrize("m", [3, 40, 129, 500])
def test_verify_every_candidate(ctx, m):
    import torch
    b = profile(m, 100 + m)
    dn = oracle.pairwise(b, m)
    wn = oracle.weights(dn, oracle.WINNING_VOTES)
    pn = oracle.closure(wn)
    beaten, win, _ = oracle.rank(pn)
    d = torch.from_numpy(dn.astype(np.int32)).cuda()
    w, wt = ctx.weights(d)
    cands = range(m) if m <= 40 else sorted(set([0, m - 1] + list(np.nonzero(win)[0]) +
                                                 list(np.random.default_rng(m).integers(0, m, size=6))))
    for c in cands:
        verdict, p_from, p_to, tied = ctx.verify(w, wt, int(c), want_tied=True)
        v = verdict.cpu().numpy()
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        assert (to_np(p_from) == np.where(np.arange(m) == c, 0, pn[c])).all()
        assert (to_np(p_to) == np.where(np.arange(m) == c, 0, pn[:, c])).all()
        assert v[0] == int(win[c]) and v[1] == beaten[c], (c, v)
        ties = [x for x in range(m) if x != c and pn[c, x] == pn[x, c]]
        assert v[3] == len(ties)
        assert sorted(tied.cpu().numpy()[:v[3]].tolist()) == ties
        if v[1]:
            x = v[2]
            assert pn[x, c] > pn[c, x]  # the reported beater beats c
            margins = [pn[y, c] - pn[c, y] for y in range(m) if pn[y, c] > pn[c, y]]
            assert pn[x, c] - pn[c, x] == max(margins)
        else:
            assert v[2] == -1


def test_verify_with_scores_picks_best_scored_beater(ctx):
    import torch
    m = 60
    b = profile(m, 3)
    dn = oracle.pairwise(b, m)
    pn = oracle.closure(oracle.weights(dn, oracle.WINNING_VOTES))
    d = torch.from_numpy(dn.astype(np.int32)).cuda()
    w, wt = ctx.weights(d)
    score = torch.from_numpy(np.random.default_rng(1).standard_normal(m).astype(np.float32)).cuda()
    sc = score.cpu().numpy()
    for c in range(m):
        verdict, _, _, _ = ctx.verify(w, wt, c, score=score)
        v = verdict.cpu().numpy()
        beaters = [y for y in range(m) if pn[y, c] > pn[c, y]]
        if beaters:
            best = max(beaters, key=lambda y: (sc[y], -y))
            assert v[2] == best


def test_verify_mid_workload_winner(ctx):
    """The stored oracle winner of the m=4096 workload passes the exact check,
    and a sampled loser is beaten by exactly as many candidates as stored."""
    import torch
    wl = workload.plain_mid()
    path = os.path.join(GOLD, wl.name + ".json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle results")
    gold = json.load(open(path))
    b = torch.from_numpy(wl.ballots).cuda()
    d = ctx.pairwise(b, wl.m, dtype="u16")
    w, wt = ctx.weights(d)
    for c in (gold["winners"][0], gold["order"][1], gold["order"][-1], 1234):
        log(f"[case] verify m=4096 cand={c}")
        verdict, _, _, _ = ctx.verify(w, wt, int(c))
        v = verdict.cpu().numpy()
        assert v[1] == gold["beaten_by"][c]
        assert v[0] == int(c in gold["winners"])
