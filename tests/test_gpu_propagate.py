"""The paper's winners-only algorithm (label propagation with widths,
Section 4) on the GPU returns exactly the Schulze winner set of the oracle,
for random profiles of many kinds, both weight modes, both counter widths,
both label orders, and the m=4096 workload."""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from tests.test_gpu_parity import GOLD, log

pytestmark = pytest.mark.gpu

MODES = {"winning_votes": oracle.WINNING_VOTES, "margin": oracle.MARGIN}


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def profiles(seed, count):
    rng = np.random.default_rng(seed)
    for k in range(count):
        m = int(rng.integers(1, 40))
        n = int(rng.integers(1, 60))
        kind = k % 4
        if kind == 0:
            b = workload.uniform_ballots(seed, n, m, min_len=0, election=k)
        elif kind == 1:
            b = workload.mallows(seed, n, m, float(rng.uniform(0.5, 1.0)), election=k)
        elif kind == 2:
            b = workload.pl_zipf(seed, n, m, float(rng.uniform(0.5, 1.5)), max(1, m // 3), election=k)
        else:
            b = workload.uniform_ballots(seed, n, m, min_len=m, election=k)
        yield k, b, m


@pytest.mark.parametrize("dtype", ["u16", "i32"])
@pytest.mark.parametrize("mode", ["winning_votes", "margin"])
def test_propagate_random_profiles(ctx, dtype, mode):
    import torch
    rounds = []
    for k, b, m in profiles(4001 + (dtype == "i32"), 120):
        want = oracle.schulze(b, m, MODES[mode])["is_winner"].astype(bool)
        d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype=dtype)
        for borda in (True, False):
            w, nw, st = ctx.winners_propagate(d, mode, borda_order=borda)
            got = w.cpu().numpy().astype(bool)
            assert (got == want).all(), (k, m, b.shape, borda, st)
            assert int(nw.cpu()[0]) == int(want.sum()) == st["n_winners"]
            rounds.append(st["rounds"])
    assert ctx.device_error() == 0
    log(f"[case] propagate {dtype} {mode}: rounds max {max(rounds)} mean {np.mean(rounds):.2f}")


def test_propagate_random_count_matrices(ctx):
    """Tie-heavy count matrices that no profile needs to produce."""
    import torch
    rng = np.random.default_rng(4003)
    for k in range(150):
        m = int(rng.integers(2, 30))
        d = rng.integers(0, 4, size=(m, m)).astype(np.int32)
        np.fill_diagonal(d, 0)
        w = oracle.weights(d.astype(np.int64), oracle.WINNING_VOTES)
        _, want, _ = oracle.rank(oracle.closure(w))
        got, nw, st = ctx.winners_propagate(torch.from_numpy(d).cuda(), "winning_votes", borda_order=k % 2 == 0)
        assert (got.cpu().numpy().astype(bool) == want.astype(bool)).all(), (k, m, st)


def test_propagate_figure1_and_sizes(ctx):
    """Figure 1 (winner a) and larger profiles spanning several sweep blocks."""
    import torch
    fig = json.load(open(os.path.join(GOLD, "figure1.json")))
    names = fig["candidates"]
    dfig = np.zeros((len(names), len(names)), dtype=np.int32)  # d = edge weights: margins and winning votes agree
    for x, y, wxy in fig["edges"]:
        dfig[names.index(x), names.index(y)] = wxy
    for mode in ("winning_votes", "margin"):
        w, nw, st = ctx.winners_propagate(torch.from_numpy(dfig).cuda(), mode)
        assert [names[i] for i in np.nonzero(w.cpu().numpy())[0]] == fig["winners"], st
    cases = []
    for i, (m, n) in enumerate([(100, 401), (257, 300), (600, 200), (1030, 64)]):
        b = workload.mallows(4004, n, m, 0.98, election=i, trunc_mod=3, trunc_lt=1, trunc_k=20)
        cases.append((b, m))
    b = workload.pl_zipf(4004, 3000, 2000, 1.0, 15, election=9)
    cases.append((b, 2000))
    for b, m in cases:
        want = oracle.schulze(b, m)["is_winner"].astype(bool)
        d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype="i32")
        w, nw, st = ctx.winners_propagate(d)
        log(f"[case] propagate m={m} n={b.shape[0]}: {st}")
        assert (w.cpu().numpy().astype(bool) == want).all()


def test_propagate_one_candidate(ctx):
    import torch
    d = torch.zeros((1, 1), dtype=torch.int32, device="cuda")
    w, nw, st = ctx.winners_propagate(d)
    assert int(w.cpu()[0]) == 1 and st["n_winners"] == 1 and st["rounds"] == 1


def test_propagate_mid_workload(ctx):
    import torch
    wl = workload.plain_mid()
    path = os.path.join(GOLD, wl.name + ".json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle results")
    gold = json.load(open(path))
    d = ctx.pairwise(torch.from_numpy(wl.ballots).cuda(), wl.m, dtype="u16")
    for borda in (True, False):
        w, nw, st = ctx.winners_propagate(d, borda_order=borda)
        log(f"[case] propagate mid workload borda={borda}: {st}")
        assert np.nonzero(w.cpu().numpy())[0].tolist() == gold["winners"]
