"""Batched elections in one persistent launch, compared with the oracle run
election by election: d, p, beaten_by, the winner set, the number of
winners and the ranking, all bit-exact.

Batches mix complete rankings (upper-triangle counting with the complement
d[y][x] = n - d[x][y]), ballots listing m-1 candidates, truncated ballots
(every ordered sub-block), empty elections and sizes around the 8-candidate
sub-block, the 32/64/128 closure paddings and the staging widths.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workload
from paper_2505_12976_amd.batch import alloc_outputs, pack
from tests.test_gpu_parity import log

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


def mixed_elections(seed):
    """(ballots uint16, m) pairs of many shapes."""
    out = []
    sizes = [(1, 5), (2, 1), (3, 7), (7, 0), (8, 50), (9, 33), (16, 2), (31, 100), (33, 101), (64, 257),
             (65, 64), (100, 333), (129, 200), (160, 61), (193, 150), (257, 90), (300, 41)]
    for i, (m, n) in enumerate(sizes):
        out.append((workload.mallows(seed, n, m, 0.9, election=i), m))
    # complete rankings written as m-1 entries (the last candidate implied)
    out.append((np.ascontiguousarray(workload.mallows(seed, 77, 40, 0.8, election=40)[:, :39]), 40))
    # truncated elections (L < m - 1): empty ballots, short lists, ties at the bottom
    out.append((workload.uniform_ballots(seed, 120, 90, 30, min_len=0, election=41), 90))
    b = workload.mallows(seed, 200, 70, 0.95, election=42, trunc_mod=2, trunc_lt=1, trunc_k=10)
    out.append((np.ascontiguousarray(b[:, :20]), 70))
    out.append((workload.pl_zipf(seed, 301, 150, 1.0, 12, election=43), 150))
    out.append((workload.uniform_ballots(seed, 9, 5, 2, min_len=0, election=44), 5))
    return out


def election_digests(d, p, beaten_by, is_winner, order):
    """[d, p, ranking outputs] digests of one election, as the stored oracle
    results hold them: the first 32 hex digits of SHA-256 over the int64
    little-endian arrays."""
    def dig(*arrays):
        h = hashlib.sha256()
        for a in arrays:
            h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
        return h.hexdigest()[:32]
    return [dig(d), dig(p), dig(beaten_by, is_winner, order)]


def expected(elections, mode):
    return [oracle.schulze(b, m, MODES[mode]) for b, m in elections]


def run_batch(ctx, elections, mode="winning_votes", dtype=np.uint16, graph=False, max_range_pairs=0,
              plan=None, packed=None, outs=None):
    import torch
    if packed is None:
        bl = []
        for b, _ in elections:
            b = np.asarray(b)
            if dtype == np.int32:
                b = np.where(b == 0xFFFF, -1, b.astype(np.int64)).astype(np.int32)
            bl.append(b)
        packed = pack(bl, [m for _, m in elections], dtype=dtype)
    dev = torch.device("cuda", 0)
    if plan is None:
        plan = ctx.batch_plan(packed.elections, "u16" if dtype == np.uint16 else "i32", mode,
                              max_range_pairs=max_range_pairs)
    ballots = torch.from_numpy(packed.ballots).to(dev)
    if outs is None:
        outs = alloc_outputs(packed, dev)
    ctx.batch_run(plan, ballots, outs["d"], outs["is_winner"], p=outs["p"], n_winners=outs["n_winners"],
                  beaten_by=outs["beaten_by"], order=outs["order"], graph=graph)
    torch.cuda.synchronize()
    return packed, plan, outs


def collect(packed, outs, e):
    return {
        "d": packed.mat(outs["d"], e).cpu().numpy().astype(np.int64),
        "p": packed.mat(outs["p"], e).cpu().numpy().astype(np.int64),
        "is_winner": packed.vec(outs["is_winner"], e).cpu().numpy().astype(bool),
        "beaten_by": packed.vec(outs["beaten_by"], e).cpu().numpy(),
        "order": packed.vec(outs["order"], e).cpu().numpy(),
        "n_winners": int(outs["n_winners"][e].cpu()),
    }


def assert_matches(packed, outs, want, label):
    for e, w in enumerate(want):
        got = collect(packed, outs, e)
        m = packed.elections[e][3]
        tag = f"{label} election {e} m={m} n={packed.elections[e][1]}"
        np.testing.assert_array_equal(got["d"], w["d"], err_msg=tag + " d")
        np.testing.assert_array_equal(got["p"], w["p"], err_msg=tag + " p")
        np.testing.assert_array_equal(got["beaten_by"], w["beaten_by"], err_msg=tag + " beaten_by")
        np.testing.assert_array_equal(got["is_winner"], w["is_winner"], err_msg=tag + " winners")
        np.testing.assert_array_equal(got["order"], w["order"], err_msg=tag + " order")
        assert got["n_winners"] == int(w["is_winner"].sum()), tag


@pytest.mark.parametrize("mode", ["winning_votes", "margin"])
@pytest.mark.parametrize("dtype", [np.uint16, np.int32])
def test_batch_matches_oracle(ctx, mode, dtype):
    els = mixed_elections(3001)
    log(f"[case] batch mixed mode={mode} dtype={np.dtype(dtype).name} E={len(els)}")
    packed, plan, outs = run_batch(ctx, els, mode, dtype)
    assert ctx.device_error() == 0
    assert_matches(packed, outs, expected(els, mode), f"{mode}/{np.dtype(dtype).name}")
    plan.destroy()


@pytest.mark.parametrize("variant", ["registers", "tiled32", "tiled64", "tiled128"])
def test_batch_every_closure_schedule(ctx, variant):
    els = [(b, m) for b, m in mixed_elections(3002)]
    if variant == "registers":
        els = [(b, m) for b, m in els if m <= 192]
    want = expected(els, "winning_votes")
    hi = 192 if variant == "registers" else 1024
    ctx.batch_set_closure(16, 1, hi, variant)
    try:
        log(f"[case] batch closure schedule {variant}")
        assert ctx.batch_get_closure(16, 100) == variant
        packed, plan, outs = run_batch(ctx, els)
        assert ctx.device_error() == 0
        assert_matches(packed, outs, want, variant)
        plan.destroy()
    finally:
        ctx.batch_set_closure(16, 1, hi, "auto")


def test_batch_counts_split_over_voter_ranges(ctx):
    """Several count ranges per election: counts accumulate with atomics."""
    els = [(workload.mallows(3003, n, m, 0.93, election=i), m) for i, (m, n) in
           enumerate([(40, 101), (130, 64), (9, 31), (300, 20)])]
    els.append((workload.uniform_ballots(3003, 77, 50, 20, min_len=0, election=9), 50))
    log("[case] batch multi-range max_range_pairs=7")
    packed, plan, outs = run_batch(ctx, els, max_range_pairs=7)
    assert ctx.device_error() == 0
    assert_matches(packed, outs, expected(els, "winning_votes"), "multi-range")
    plan.destroy()


def test_batch_graph_replays(ctx):
    """The captured graph gives the eager result on every replay, with other
    work and synchronisations between replays, and is re-captured when the
    output pointers change."""
    import torch
    els = mixed_elections(3004)[:12]
    packed, plan, outs = run_batch(ctx, els)
    eager = [collect(packed, outs, e) for e in range(len(els))]
    want = expected(els, "winning_votes")
    assert_matches(packed, outs, want, "eager")
    for rep in range(3):
        for t in outs.values():
            if t is not None:
                t.fill_(7)
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        (x * 3).sum().item()
        log(f"[case] batch graph replay {rep}")
        run_batch(ctx, els, graph=True, plan=plan, packed=packed, outs=outs)
        for e in range(len(els)):
            got = collect(packed, outs, e)
            for k in eager[e]:
                np.testing.assert_array_equal(np.asarray(got[k]), np.asarray(eager[e][k]), err_msg=f"replay {rep} {k}")
    outs2 = alloc_outputs(packed, torch.device("cuda", 0))
    run_batch(ctx, els, graph=True, plan=plan, packed=packed, outs=outs2)
    assert_matches(packed, outs2, want, "recaptured")
    assert ctx.device_error() == 0
    plan.destroy()


def test_batch_closure_only(ctx):
    """Without ballots, d is the input: weights, closure, winners, ranking."""
    import torch
    els = mixed_elections(3005)
    want = expected(els, "margin")
    packed = pack([b for b, _ in els], [m for _, m in els])
    plan = ctx.batch_plan(packed.elections, "u16", "margin", closure_only=True)
    dev = torch.device("cuda", 0)
    outs = alloc_outputs(packed, dev)
    dflat = np.zeros(packed.d_elems, dtype=np.int32)
    for e, w in enumerate(want):
        _, _, _, m, off, _ = packed.elections[e]
        dflat[off:off + m * m] = w["d"].reshape(-1)
    outs["d"].copy_(torch.from_numpy(dflat))
    log("[case] batch closure-only")
    ctx.batch_run(plan, None, outs["d"], outs["is_winner"], p=outs["p"], n_winners=outs["n_winners"],
                  beaten_by=outs["beaten_by"], order=outs["order"])
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    assert_matches(packed, outs, want, "closure-only")
    with pytest.raises(Exception):  # a closure-only plan refuses ballots
        ctx.batch_run(plan, torch.zeros(4, dtype=torch.uint16, device=dev), outs["d"], outs["is_winner"])
    plan.destroy()


def test_batch_int32_closure_for_large_electorates(ctx):
    """More than 65535 voters: the closure runs on int32 values."""
    els = [(workload.mallows(3006, 70001, 20, 0.97, election=0), 20),
           (workload.mallows(3006, 66000, 75, 0.99, election=1), 75),
           (workload.mallows(3006, 300, 33, 0.9, election=2), 33)]
    log("[case] batch int32 values")
    packed, plan, outs = run_batch(ctx, els)
    assert ctx.device_error() == 0
    want = expected(els, "winning_votes")
    assert_matches(packed, outs, want, "int32")
    plan.destroy()
    # top-k levels on int32 values too
    import torch
    plan = ctx.batch_plan(packed.elections, "u16", "winning_votes", topk=20)
    dev = torch.device("cuda", 0)
    level = torch.full((packed.vec_elems,), -7, dtype=torch.int32, device=dev)
    ctx.batch_run(plan, torch.from_numpy(packed.ballots).to(dev), outs["d"], outs["is_winner"], level=level)
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    for e, w in enumerate(want):
        np.testing.assert_array_equal(packed.vec(level, e).cpu().numpy(), oracle.topk_levels(w["w"], 20))
    plan.destroy()


@pytest.mark.parametrize("bad", ["repeat", "range", "after_pad", "short_complete"])
def test_batch_invalid_ballots(ctx, bad):
    b = workload.mallows(3007, 20, 12, 0.9, election=0).copy()
    m = 12
    if bad == "repeat":
        b[5, 3] = b[5, 4]
    elif bad == "range":
        b[7, 0] = 12
    elif bad == "after_pad":
        b = np.ascontiguousarray(b[:, :6])  # truncated election, L = 6 < m - 1
        b[2, 2] = 0xFFFF
    elif bad == "short_complete":
        b[3, 10:] = 0xFFFF  # lists 10 < m - 1 candidates in an election with L = m
    good = (workload.mallows(3007, 30, 9, 0.9, election=1), 9)
    log(f"[case] batch invalid ballot {bad}")
    run_batch(ctx, [good, (b, m)])
    import paper_2505_12976_amd as sz
    assert ctx.device_error() == sz.EBALLOT


def test_batch_rejects_bad_descriptors(ctx):
    import paper_2505_12976_amd as sz
    for el in [(0, 5, 0, 4, 0, 0), (0, 5, 5, 4, 0, 0), (0, -1, 4, 4, 0, 0), (0, 5, 4, 0, 0, 0),
               (0, 5, 4, 1025, 0, 0), (-1, 5, 4, 4, 0, 0)]:
        with pytest.raises(sz.SchulzeError) as ex:
            ctx.batch_plan([el])
        assert ex.value.code == sz.EINVAL
    for args in ((32, 1, 64, "tiled32"),      # 16-bit values only
                 (32, 1, 64, "tiled128"),     # 16-bit values only
                 (16, 200, 256, "registers"),  # beyond the register budget
                 (32, 100, 160, "registers"),
                 (16, 0, 10, "tiled64"), (16, 10, 1025, "tiled64"), (24, 1, 10, "tiled64")):
        with pytest.raises(sz.SchulzeError) as ex:
            ctx.batch_set_closure(*args)
        assert ex.value.code == sz.EINVAL


def test_batch_autotune_then_exact(ctx):
    ms16 = ctx.batch_autotune(16, 320)
    ms32 = ctx.batch_autotune(32, 160)
    log(f"[case] batch autotune 16-bit\n{ms16}\n32-bit\n{ms32}")
    names = ["registers", "tiled32", "tiled64", "tiled128"]
    for bits, ms in ((16, ms16), (32, ms32)):
        for bk in range(ms.shape[0]):
            valid = ms[bk] >= 0
            assert valid.any()
            best = names[int(np.argmin(np.where(valid, ms[bk], np.inf)))]
            assert ctx.batch_get_closure(bits, 32 * (bk + 1)) == best
    els = mixed_elections(3008)
    packed, plan, outs = run_batch(ctx, els)
    assert ctx.device_error() == 0
    assert_matches(packed, outs, expected(els, "winning_votes"), "tuned")
    plan.destroy()
    for bits in (16, 32):
        ctx.batch_set_closure(bits, 1, 1024, "auto")


def test_batch_tuned_schedules_persist(ctx, tmp_path):
    """The tuned schedules are stored per device and library build: the
    second call reads them back, sets them and tunes nothing."""
    from paper_2505_12976_amd.batch import tuned_closures
    path = str(tmp_path / "tuning.json")
    s1, hit1 = tuned_closures(ctx, 16, 96, path=path)
    ctx.batch_set_closure(16, 1, 1024, "auto")
    s2, hit2 = tuned_closures(ctx, 16, 96, path=path)
    log(f"[case] tuned schedules {s1} / {s2}")
    assert not hit1 and hit2 and s1 == s2 and len(s1) == 3
    assert [ctx.batch_get_closure(16, 32 * (b + 1)) for b in range(3)] == s2
    els = [e for e in mixed_elections(3011) if e[1] <= 96]
    packed, plan, outs = run_batch(ctx, els)
    assert ctx.device_error() == 0
    assert_matches(packed, outs, expected(els, "winning_votes"), "persisted schedules")
    plan.destroy()
    ctx.batch_set_closure(16, 1, 1024, "auto")


def test_batch_of_the_batched_workload_shape(ctx):
    """64 elections drawn like the 4096-election workload (m ~ U{8..512},
    n ~ U{50..20000}, phi ~ U[0.5, 1]); the oracle checks every election."""
    flat, desc, (ms, ns, phis) = workload.batch_mallows(1004, 64, n_hi=3000)
    from paper_2505_12976_amd.batch import Packed
    packed = Packed(flat, desc, sum(int(m) * int(m) for m in ms), int(sum(ms)))
    log(f"[case] batch workload shape E=64 sum_n={int(ns.sum())}")
    packed, plan, outs = run_batch(ctx, None, packed=packed, graph=True)
    assert ctx.device_error() == 0
    want = []
    for e in range(64):
        bo, n, L, m, _, _ = desc[e]
        want.append(oracle.schulze(flat[bo:bo + n * m].reshape(n, m), m))
    assert_matches(packed, outs, want, "workload-shape")
    plan.destroy()


@pytest.mark.slow
def test_batch_full_workload_sampled():
    """The 4096-election workload in the configuration the benchmark times
    (autotuned schedules, graph replay): structural properties on every
    election, the oracle on sampled elections including the largest ones."""
    import torch
    import paper_2505_12976_amd as sz
    from paper_2505_12976_amd.batch import Packed
    flat, desc, (ms, ns, phis) = workload.batch_mallows(1004, 4096)
    packed = Packed(flat, desc, int(np.sum(ms * ms)), int(np.sum(ms)))
    log(f"[case] batch full workload: {flat.nbytes / 1e9:.1f} GB of ballots")
    ctx = sz.Context(0)
    try:
        ctx.batch_autotune(16, int(ms.max()))
        plan = ctx.batch_plan(desc, "u16", "winning_votes")
        dev = torch.device("cuda", 0)
        ballots = torch.from_numpy(flat).to(dev)
        outs = alloc_outputs(packed, dev)
        for _ in range(2):  # capture, then replay
            ctx.batch_run(plan, ballots, outs["d"], outs["is_winner"], p=outs["p"], n_winners=outs["n_winners"],
                          beaten_by=outs["beaten_by"], order=outs["order"], graph=True)
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        d_all = outs["d"].cpu().numpy().astype(np.int64)
        p_all = outs["p"].cpu().numpy().astype(np.int64)
        w_all = outs["is_winner"].cpu().numpy().astype(bool)
        bb_all = outs["beaten_by"].cpu().numpy()
        o_all = outs["order"].cpu().numpy()
        nw_all = outs["n_winners"].cpu().numpy()
        for e, (bo, n, L, m, mo, vo) in enumerate(desc):
            d = d_all[mo:mo + m * m].reshape(m, m)
            p = p_all[mo:mo + m * m].reshape(m, m)
            off = ~np.eye(m, dtype=bool)
            assert (np.diag(d) == 0).all() and ((d + d.T)[off] == n).all(), e  # complete rankings
            w = np.where(off & (d > d.T), d, 0)
            assert (p >= w).all() and (np.diag(p) == 0).all(), e
            bb = (p.T > p).sum(axis=1)
            assert (bb_all[vo:vo + m] == bb).all(), e
            assert (w_all[vo:vo + m] == (bb == 0)).all() and nw_all[e] == (bb == 0).sum() >= 1, e
            want_order = np.lexsort((np.arange(m), bb))
            assert (o_all[vo:vo + m] == want_order).all(), e
        # every election against the oracle's stored digests
        gold_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_mallows_E4096.json")
        if os.path.exists(gold_path):
            with open(gold_path) as f:
                gold = json.load(f)
            assert gold["m"] == ms.tolist() and gold["n"] == ns.tolist()
            bad = []
            for e, (bo, n, L, m, mo, vo) in enumerate(desc):
                dg = election_digests(d_all[mo:mo + m * m].reshape(m, m), p_all[mo:mo + m * m].reshape(m, m),
                                      bb_all[vo:vo + m], w_all[vo:vo + m], o_all[vo:vo + m])
                want = gold["elections"][e]
                if dg != want[:3] or int(nw_all[e]) != want[3]:
                    bad.append(e)
            assert not bad, f"{len(bad)} elections differ from the oracle, first {bad[:10]}"
            log("[case] batch full workload: all 4096 elections equal the oracle's digests")
        # the oracle on the largest elections and a seeded sample
        big = list(np.argsort(-(ms * ms * ns))[:3])
        rng = np.random.default_rng(7)
        sample = sorted(set(big) | set(rng.choice(4096, 5, replace=False).tolist()))
        for e in sample:
            bo, n, L, m, mo, vo = desc[e]
            log(f"[case] oracle election {e}: m={m} n={n}")
            want = oracle.schulze(flat[bo:bo + n * m].reshape(n, m), m)
            np.testing.assert_array_equal(d_all[mo:mo + m * m].reshape(m, m), want["d"])
            np.testing.assert_array_equal(p_all[mo:mo + m * m].reshape(m, m), want["p"])
            np.testing.assert_array_equal(o_all[vo:vo + m], want["order"])
        plan.destroy()
    finally:
        ctx.close()


@pytest.mark.parametrize("topk", [1, 3, 1000])
@pytest.mark.parametrize("mode", ["winning_votes", "margin"])
def test_batch_topk_levels(ctx, topk, mode):
    """Top-k levels by iterated winner removal, per election, equal the
    oracle's; the other outputs are unchanged; graph replays agree."""
    import torch
    els = mixed_elections(3011)
    packed = pack([b for b, _ in els], [m for _, m in els])
    plan = ctx.batch_plan(packed.elections, "u16", mode, topk=topk)
    dev = torch.device("cuda", 0)
    ballots = torch.from_numpy(packed.ballots).to(dev)
    outs = alloc_outputs(packed, dev)
    level = torch.full((packed.vec_elems,), -7, dtype=torch.int32, device=dev)
    want = expected(els, mode)
    for graph in (False, True, True):
        log(f"[case] batch topk={topk} mode={mode} graph={graph}")
        level.fill_(-7)
        ctx.batch_run(plan, ballots, outs["d"], outs["is_winner"], p=outs["p"], n_winners=outs["n_winners"],
                      beaten_by=outs["beaten_by"], order=outs["order"], graph=graph, level=level)
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        assert_matches(packed, outs, want, f"topk={topk}")
        for e, w in enumerate(want):
            lv = packed.vec(level, e).cpu().numpy()
            ref = oracle.topk_levels(w["w"], topk)
            np.testing.assert_array_equal(lv, ref, err_msg=f"topk={topk} election {e} m={packed.elections[e][3]}")
    plan.destroy()


def test_batch_level_needs_topk_plan(ctx):
    import torch
    import paper_2505_12976_amd as sz
    els = mixed_elections(3013)[:3]
    packed = pack([b for b, _ in els], [m for _, m in els])
    plan = ctx.batch_plan(packed.elections, "u16")
    dev = torch.device("cuda", 0)
    outs = alloc_outputs(packed, dev)
    level = torch.zeros(packed.vec_elems, dtype=torch.int32, device=dev)
    with pytest.raises(sz.SchulzeError):
        ctx.batch_run(plan, torch.from_numpy(packed.ballots).to(dev), outs["d"], outs["is_winner"], level=level)
    plan.destroy()
