"""Parity of the HIP path with the CPU oracle, element by element.

Every case runs the whole hot path through the C ABI (pairwise -> closure ->
winners -> ranking) on seeded synthetic profiles and compares d, p,
beaten_by, the winner set and the ranking with the oracle: all integer, so
the bar is bit-exact.  Sizes span several tiles with ragged tails (the count
tile is 128 candidates, the closure tile 64 or 128).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def gpu_path(ctx, ballots, m, dtype="i32", mode="winning_votes", weight=None, schedule="auto"):
    import torch
    ctx.set_closure_schedule(schedule)
    b = torch.from_numpy(np.ascontiguousarray(ballots)).cuda()
    wt = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight, dtype=np.uint32)).cuda()
    d = ctx.pairwise(b, m, voter_weight=wt, dtype=dtype)
    p = ctx.closure(d, mode)
    is_w, nw = ctx.winners(p)
    order, beaten = ctx.ranking(p)
    torch.cuda.synchronize()
    err = ctx.device_error()
    return {
        "err": err,
        "d": d.cpu().numpy().astype(np.int64),
        "p": p.cpu().numpy().astype(np.int64),
        "is_winner": is_w.cpu().numpy().astype(bool),
        "n_winners": int(nw.cpu()[0]),
        "order": order.cpu().numpy(),
        "beaten_by": beaten.cpu().numpy(),
    }


def assert_same(got, want, tag):
    assert got["err"] == 0, f"{tag}: device error {got['err']}"
    for key in ("d", "p", "beaten_by", "is_winner", "order"):
        g, w = got[key], want[key]
        if not np.array_equal(g, w):
            bad = np.argwhere(np.asarray(g) != np.asarray(w))
            raise AssertionError(f"{tag}: {key} differs at {len(bad)} places, first {bad[:5].tolist()}")
    assert got["n_winners"] == int(want["is_winner"].sum()), tag


def check_case(ctx, ballots, m, dtype, mode, weight=None, tag="", schedules=("auto",)):
    want = oracle.schulze(ballots, m, oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES, weight)
    for sched in schedules:
        log(f"[case] {tag} m={m} n={ballots.shape[0]} L={ballots.shape[1]} dtype={dtype} mode={mode} "
            f"closure={sched}")
        got = gpu_path(ctx, ballots, m, dtype, mode, weight, schedule=sched)
        assert_same(got, want, f"{tag}/{sched}")


SIZES = [1, 2, 3, 7, 31, 64, 65, 127, 128, 129, 200, 257, 700, 2100]


BOTH = ("auto", "phased")


@pytest.mark.parametrize("m", SIZES)
def test_full_mallows(ctx, m):
    b = workload.mallows(100 + m, 301, m, 0.9)
    check_case(ctx, b, m, "i32", "winning_votes", tag="full-mallows", schedules=BOTH)
    check_case(ctx, b, m, "u16", "margin", tag="full-mallows", schedules=BOTH)


@pytest.mark.parametrize("m", SIZES)
def test_truncated_mixture(ctx, m):
    k = max(1, m // 3)
    b = workload.mallows(200 + m, 257, m, 0.95, trunc_mod=5, trunc_lt=2, trunc_k=k)
    check_case(ctx, b, m, "u16", "winning_votes", tag="mallows-truncated", schedules=BOTH)
    check_case(ctx, b, m, "i32", "margin", tag="mallows-truncated", schedules=BOTH)


@pytest.mark.parametrize("m", [5, 64, 130, 300])
def test_pl_topk_int32_ballots(ctx, m):
    b = workload.pl_zipf(300 + m, 999, m, 1.1, min(20, m), dtype=np.int32)
    check_case(ctx, b, m, "i32", "winning_votes", tag="pl-zipf")
    check_case(ctx, b, m, "i32", "margin", tag="pl-zipf")


@pytest.mark.parametrize("m,n,k", [(2500, 3000, 5), (1500, 4001, 3)])
def test_short_lists_many_candidates(ctx, m, n, k):
    """Short ballots over many candidates: the pair-scattering route."""
    b = workload.pl_zipf(600 + m, n, m, 1.0, k)
    check_case(ctx, b, m, "i32", "winning_votes", tag="short-lists")


@pytest.mark.parametrize("m", [4, 65, 150])
def test_uniform_ties(ctx, m):
    b = workload.uniform_ballots(400 + m, 123, m, min_len=0)
    check_case(ctx, b, m, "u16", "winning_votes", tag="uniform")
    check_case(ctx, b, m, "i32", "margin", tag="uniform")


@pytest.mark.parametrize("m", [3, 66, 260])
def test_voter_weights(ctx, m):
    rng = np.random.default_rng(m)
    b = workload.mallows(500 + m, 77, m, 0.8, trunc_mod=3, trunc_lt=1, trunc_k=max(1, m // 4))
    w = rng.integers(0, 50, size=77).astype(np.uint32)
    check_case(ctx, b, m, "i32", "winning_votes", weight=w, tag="weighted")
    check_case(ctx, b, m, "u16", "margin", weight=w, tag="weighted")


def test_edge_cases(ctx):
    # no voters: every count is 0, nobody beats anybody
    check_case(ctx, np.zeros((0, 5), dtype=np.uint16), 5, "u16", "winning_votes", tag="no-voters")
    # one voter, full ranking
    check_case(ctx, workload.mallows(1, 1, 130, 0.5), 130, "i32", "winning_votes", tag="one-voter")
    # every ballot empty: all tied
    check_case(ctx, np.full((10, 4), -1, dtype=np.int32), 4, "i32", "margin", tag="empty-ballots")
    # one candidate
    check_case(ctx, np.zeros((3, 1), dtype=np.uint16), 1, "u16", "winning_votes", tag="m=1")
    # ballots listing m-1 candidates are full rankings
    b = workload.mallows(9, 41, 70, 0.9)[:, :69].copy()
    check_case(ctx, b, 70, "i32", "winning_votes", tag="m-1 listed")
    # an even number of voters in perfect opposition: all ties
    perm = workload.permutation(3, 0, 40)
    b = np.stack([perm, perm[::-1]] * 5).astype(np.uint16)
    check_case(ctx, b, 40, "u16", "winning_votes", tag="opposed")
    # an odd number of full rankings (a missing pair partner)
    check_case(ctx, workload.mallows(11, 255, 129, 0.7), 129, "u16", "winning_votes", tag="odd-n")


def test_figure1_via_mcgarvey(ctx):
    from tests import brute
    from tests.test_oracle_pins import figure1
    g, idx, w, table = figure1()
    b = brute.mcgarvey_ballots(4, [(idx[a], idx[c], mu) for a, c, mu in g["edges"]])
    got = gpu_path(ctx, b, 4, "i32", "margin")
    assert (got["p"] == table).all()
    assert list(got["order"]) == [idx["a"], idx["d"], idx["b"], idx["c"]]


def test_plain_small_workload(ctx):
    wl = workload.plain_small()
    check_case(ctx, wl.ballots, wl.m, "i32", "winning_votes", tag=wl.name)


def test_run_twice_identical(ctx):
    b = workload.mallows(77, 3001, 300, 0.97, trunc_mod=10, trunc_lt=3, trunc_k=30)
    a1 = gpu_path(ctx, b, 300, "u16")
    a2 = gpu_path(ctx, b, 300, "u16")
    for key in ("d", "p", "order"):
        assert np.array_equal(a1[key], a2[key])


def test_invalid_ballots_set_device_error(ctx):
    import paper_2505_12976_amd as sz
    long_dup = np.full((1, 66), -1, dtype=np.int32)
    long_dup[0, :5] = [3, 1, 2, 3, 0]
    # uint16 rows of 72 entries take the 16-byte scan and scatter
    u16_range = np.full((3, 72), 0xFFFF, dtype=np.uint16)
    u16_range[:, :70] = np.arange(70, dtype=np.uint16)
    u16_range[1, 40] = 80
    u16_dup = np.full((3, 72), 0xFFFF, dtype=np.uint16)
    u16_dup[:, :71] = np.arange(71, dtype=np.uint16)
    u16_dup[2, 9] = 3
    cases = [(np.array([[0, 1, 1, 2]], dtype=np.int32), 4),      # repeated id
             (np.array([[0, 9, -1, -1]], dtype=np.int32), 4),    # id out of range
             (long_dup, 66),                                      # repeated id, long row
             (u16_range, 72),                                     # id out of range, uint16 long rows
             (u16_dup, 72)]                                       # repeated id, uint16 long rows
    for bad, m in cases:
        log(f"[case] invalid ballot {bad[0, :6].tolist()} m={m}")
        got = gpu_path(ctx, bad, m, "i32")
        assert got["err"] == sz.EBALLOT
        assert ctx.device_error() == 0  # reading the error word resets it


def test_u16_overflow_is_rejected(ctx):
    import torch
    import paper_2505_12976_amd as sz
    b = torch.zeros((70000, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(sz.SchulzeError) as e:
        ctx.pairwise(b, 2, dtype="u16")
    assert e.value.code == sz.ERANGE
    # with voter weights the check happens on the device
    b = torch.tensor([[0, 1]], dtype=torch.int32, device="cuda")
    w = torch.from_numpy(np.array([70000], dtype=np.uint32)).cuda()
    ctx.pairwise(b, 2, voter_weight=w, dtype="u16")
    torch.cuda.synchronize()
    assert ctx.device_error() == sz.ERANGE


@pytest.mark.parametrize("route", ["full", "truncated", "pairs"])
def test_weighted_total_beyond_32_bits_is_rejected(ctx, route):
    """Weighted counts accumulate in 32 bits: a total weight of 2^32 or more
    sets ERANGE (it could wrap a count back into range); a total just below
    2^32 with every count under 2^31 is counted exactly."""
    import torch
    import paper_2505_12976_amd as sz
    m = {"full": 3, "truncated": 40, "pairs": 3000}[route]
    fwd = np.full((1, m), -1, dtype=np.int32)
    bwd = np.full((1, m), -1, dtype=np.int32)
    k = m if route == "full" else 3
    fwd[0, :k] = np.arange(k)
    bwd[0, :k] = np.arange(k)[::-1]
    b = np.concatenate([fwd, bwd])
    # both ballots put the listed candidates above the unlisted ones, so
    # there only totals below 2^31 fit; opposite full rankings split them
    fits = [2 ** 31 - 1, 2 ** 31 - 1] if route == "full" else [2 ** 30, 2 ** 30 - 1]
    for weights, ok in (([2 ** 31, 2 ** 31], False), ([2 ** 32 - 1, 1], False), (fits, True)):
        log(f"[case] weighted total {sum(weights)} route={route} m={m}")
        w = torch.from_numpy(np.array(weights, dtype=np.uint32)).cuda()
        d = ctx.pairwise(torch.from_numpy(b).cuda(), m, voter_weight=w, dtype="i32")
        torch.cuda.synchronize()
        err = ctx.device_error()
        if ok:
            assert err == 0
            want = oracle.pairwise(b, m, weight=np.array(weights, dtype=np.uint32))
            assert (d.cpu().numpy().astype(np.int64) == want).all()
        else:
            assert err == sz.ERANGE


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def _golden(name):
    path = os.path.join(GOLD, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle results for {name}")
    with open(path) as f:
        return json.load(f)


def _check_against_golden(ctx, wl, gold):
    assert hashlib.sha256(np.ascontiguousarray(wl.ballots).tobytes()).hexdigest() == gold["ballots_sha256"], \
        "generator output differs from the one the stored results were made from"
    log(f"[case] {wl.name}: GPU path")
    got = gpu_path(ctx, wl.ballots, wl.m, wl.d_dtype, "winning_votes")
    assert got["err"] == 0
    if _digest(got["d"]) != gold["d_sha256"]:
        rows = np.nonzero(got["d"].sum(axis=1) != np.array(gold["d_row_sums"]))[0]
        raise AssertionError(f"d differs; rows with other sums: {rows[:10].tolist()}")
    if _digest(got["p"]) != gold["p_sha256"]:
        rows = np.nonzero(got["p"].sum(axis=1) != np.array(gold["p_row_sums"]))[0]
        raise AssertionError(f"p differs; rows with other sums: {rows[:10].tolist()}")
    assert got["beaten_by"].tolist() == gold["beaten_by"]
    assert np.nonzero(got["is_winner"])[0].tolist() == gold["winners"]
    assert got["order"].tolist() == gold["order"]
    assert got["n_winners"] == len(gold["winners"])
    return got


def test_plain_mid_workload_full_size(ctx):
    """m=4096, n=60000 Mallows(0.97), 30% top-100: d, p, winners, ranking."""
    wl = workload.plain_mid()
    gold = _golden(wl.name)
    got = _check_against_golden(ctx, wl, gold)
    # independent of the stored digest: sampled rows and columns of d
    rows = np.array([0, 1, 2047, 4095, int(gold["winners"][0])], dtype=np.int32)
    assert (got["d"][rows] == oracle.pairwise_rows(wl.ballots, wl.m, rows)).all()
    assert (got["d"][:, rows].T == oracle.pairwise_cols(wl.ballots, wl.m, rows)).all()


@pytest.mark.slow
def test_plain_large_workload_full_size(ctx):
    """m=16384, n=1e6 top-20 Plackett-Luce Zipf(1.1): d, p, winners, ranking."""
    wl = workload.plain_large()
    gold = _golden(wl.name)
    _check_against_golden(ctx, wl, gold)


def _digest_chunked(a, rows=1024):
    """SHA-256 of a (as int64 little-endian, row-major), hashed in row chunks."""
    h = hashlib.sha256()
    for i in range(0, a.shape[0], rows):
        h.update(np.ascontiguousarray(a[i:i + rows], dtype="<i8").tobytes())
    return h.hexdigest()


@pytest.mark.slow
def test_learned_workload_full_size(ctx):
    """m=32768, n=200000 top-30 Plackett-Luce Zipf(1.0): d against the
    oracle's digest; the winner set of the learned path, of label
    propagation and of the full closure against the oracle's (certified by
    single-source/target widest paths); rows and columns of the GPU closure
    at the winners, the candidates tied with them and a seeded sample against
    the oracle's widest paths; the verify kernel's rows at the winner too."""
    import torch
    from paper_2505_12976_amd.proposer import load_checkpoint
    wl = workload.plain_learned()
    gold = _golden(wl.name)
    m, n = wl.m, wl.n
    assert hashlib.sha256(np.ascontiguousarray(wl.ballots).tobytes()).hexdigest() == gold["ballots_sha256"]
    dev = torch.device("cuda", 0)
    log(f"[case] {wl.name}: count")
    d = ctx.pairwise(torch.from_numpy(wl.ballots).to(dev), m, dtype="i32")
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    d_host = d.cpu().numpy()
    if _digest_chunked(d_host) != gold["d_sha256"]:
        rows = np.nonzero(d_host.sum(axis=1, dtype=np.int64) != np.array(gold["d_row_sums"]))[0]
        raise AssertionError(f"d differs; rows with other sums: {rows[:10].tolist()}")
    del d_host
    want = gold["winners"]
    ckpt = os.path.join(os.path.dirname(GOLD), "..", "paper_2505_12976_amd", "data", "proposer.npz")
    params = torch.from_numpy(load_checkpoint(ckpt)["params"]).to(dev)
    log(f"[case] {wl.name}: learned path")
    w, nw, st = ctx.winners_learned(d, float(n), params)
    assert np.nonzero(w.cpu().numpy())[0].tolist() == want, st
    log(f"[case] {wl.name}: label propagation")
    w, nw, st = ctx.winners_propagate(d)
    assert np.nonzero(w.cpu().numpy())[0].tolist() == want, st
    log(f"[case] {wl.name}: verify at the first winner")
    wgt, wgt_t = ctx.weights(d)
    c0 = int(gold["first_winner"])
    verdict, p_from, p_to, _ = ctx.verify(wgt, wgt_t, c0)
    assert int(verdict[0].item()) == 1
    ref = gold["p_rows_cols"][str(c0)]
    assert _digest_chunked(p_from.cpu().numpy()) == ref["row_sha256"]
    assert _digest_chunked(p_to.cpu().numpy()) == ref["col_sha256"]
    del wgt, wgt_t
    log(f"[case] {wl.name}: full closure")
    p = ctx.closure(d)
    iw, nw = ctx.winners(p)
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    assert np.nonzero(iw.cpu().numpy())[0].tolist() == want
    for c, ref in gold["p_rows_cols"].items():
        c = int(c)
        assert _digest_chunked(p[c].cpu().numpy()) == ref["row_sha256"], f"row {c}"
        assert _digest_chunked(p[:, c].contiguous().cpu().numpy()) == ref["col_sha256"], f"column {c}"
