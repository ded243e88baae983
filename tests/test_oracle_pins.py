"""Pins for the CPU oracle: values and properties the paper or mathematics fix.

Each check compares the oracle with something that is not the oracle: the
paper's Figure 1 table, brute-force path enumeration, graph searches,
McGarvey's construction, the NL-hardness reduction, and the axiomatic
properties the paper states (Condorcet consistency, Schwartz refinement,
transitivity of beats, soundness of the initialisation filter).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def figure1():
    with open(os.path.join(GOLD, "figure1.json")) as f:
        g = json.load(f)
    names = g["candidates"]
    idx = {c: i for i, c in enumerate(names)}
    m = len(names)
    w = np.zeros((m, m), dtype=np.int64)
    for a, b, mu in g["edges"]:
        w[idx[a], idx[b]] = mu
    table = np.zeros((m, m), dtype=np.int64)
    for a, row in g["widest"].items():
        for b, v in row.items():
            table[idx[a], idx[b]] = v
    return g, idx, w, table


# ---------------------------------------------------------------- Figure 1

def test_figure1_widest_table():
    g, idx, w, table = figure1()
    p = oracle.closure(w)
    assert (p == table).all()


def test_figure1_winner_and_ranking():
    g, idx, w, table = figure1()
    beaten, win, order = oracle.rank(oracle.closure(w))
    assert {i for i in range(4) if win[i]} == {idx[c] for c in g["winners"]}
    # derived from the printed table: a beats all; d beats b and c; b beats c
    assert list(order) == [idx["a"], idx["d"], idx["b"], idx["c"]]
    assert list(beaten) == [0, 2, 3, 1]


def test_figure1_schwartz():
    g, idx, w, table = figure1()
    # the graph's weights are margins, so d with d - d^T = w realises it
    assert brute.schwartz_set(w) == {idx[c] for c in g["schwartz"]}


def test_figure1_from_ballots_mcgarvey():
    """42 linear orders realise Figure 1's margins (McGarvey, Section 3)."""
    g, idx, w, table = figure1()
    edges = [(idx[a], idx[b], mu) for a, b, mu in g["edges"]]
    ballots = brute.mcgarvey_ballots(4, edges)
    assert ballots.shape == (42, 4)
    d = oracle.pairwise(ballots, 4)
    assert (d == brute.count_pairs(ballots, 4)).all()
    margin = oracle.weights(d, oracle.MARGIN)
    assert (margin == w).all()
    assert (oracle.closure(margin) == table).all()
    # winning votes on full rankings: d = n/2 + mu/2 on edges, p_WV = 21 + p/2
    pw = oracle.closure(oracle.weights(d, oracle.WINNING_VOTES))
    off = ~np.eye(4, dtype=bool)
    assert (pw[off] == np.where(table[off] > 0, 21 + table[off] // 2, 0)).all()
    _, win, order = oracle.rank(pw)
    assert list(order) == [idx["a"], idx["d"], idx["b"], idx["c"]]


# ---------------------------------------------------------------- count

def _random_profiles(count, max_m=7, seed=7):
    rng = np.random.default_rng(seed)
    for i in range(count):
        m = int(rng.integers(1, max_m + 1))
        n = int(rng.integers(1, 12))
        kind = i % 3
        if kind == 0:
            b = workload.uniform_ballots(seed * 1000 + i, n, m, dtype=np.int32)
        elif kind == 1:
            b = workload.mallows(seed * 1000 + i, n, m, float(rng.uniform(0.3, 1.0)), dtype=np.int32)
        else:
            k = int(rng.integers(0, m + 1))
            b = workload.pl_zipf(seed * 1000 + i, n, m, 1.0, k, L=m, dtype=np.int32)
        wts = rng.integers(1, 5, size=n).astype(np.uint32) if i % 4 == 0 else None
        yield m, b, wts


def test_count_matches_pair_lists():
    for m, b, wts in _random_profiles(300):
        assert (oracle.pairwise(b, m, wts) == brute.count_pairs(b, m, wts)).all()


def test_count_rows_and_cols_match_full():
    b = workload.mallows(11, 200, 40, 0.9, trunc_mod=3, trunc_lt=1, trunc_k=5)
    d = oracle.pairwise(b, 40)
    rows = np.array([0, 7, 39, 7])
    assert (oracle.pairwise_rows(b, 40, rows) == d[rows]).all()
    assert (oracle.pairwise_cols(b, 40, rows) == d[:, rows].T).all()


def test_count_full_rankings_sum_to_n():
    b = workload.mallows(3, 500, 30, 0.7)
    d = oracle.pairwise(b, 30)
    off = ~np.eye(30, dtype=bool)
    assert ((d + d.T)[off] == 500).all() and (np.diag(d) == 0).all()


def test_count_single_voter_is_triangular():
    perm = workload.permutation(5, 0, 9)
    d = oracle.pairwise(perm[None, :].astype(np.int32), 9)
    pos = np.argsort(perm)
    assert (d == (pos[:, None] < pos[None, :])).all()


def test_count_identity_ranked_minus_order():
    """d[x][y] = R_x - C[y][x]: R_x = ballots listing x, C[y][x] = ballots
    listing y before x (a rewrite of 'x listed and y after it or unlisted')."""
    m = 25
    b = workload.pl_zipf(9, 400, m, 1.1, 6)
    R = np.zeros(m, dtype=np.int64)
    C = np.zeros((m, m), dtype=np.int64)
    for row in b:
        lst = brute.listed(row)
        for i, x in enumerate(lst):
            R[x] += 1
            for y in lst[:i]:
                C[y, x] += 1
    d = oracle.pairwise(b, m)
    expect = R[:, None] - C.T
    np.fill_diagonal(expect, 0)
    assert (d == expect).all()


def test_count_mcgarvey_random_graphs():
    rng = np.random.default_rng(3)
    for _ in range(40):
        m = int(rng.integers(2, 8))
        edges = []
        for a in range(m):
            for c in range(a + 1, m):
                mu = int(rng.integers(0, 4)) * 2
                if mu:
                    edges.append((a, c, mu) if rng.random() < 0.5 else (c, a, mu))
        if not edges:
            continue
        b = brute.mcgarvey_ballots(m, edges)
        margin = oracle.weights(oracle.pairwise(b, m), oracle.MARGIN)
        want = np.zeros((m, m), dtype=np.int64)
        for a, c, mu in edges:
            want[a, c] = mu
        assert (margin == want).all()


def test_count_rejects_bad_ballots():
    bad = np.array([[0, 1, 1]], dtype=np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.pairwise(bad, 3)
    with pytest.raises(oracle.OracleError):
        oracle.pairwise(np.array([[0, 5, -1]], dtype=np.int32), 3)


# ---------------------------------------------------------------- weights

def test_weights_modes():
    d = np.array([[0, 5, 2], [3, 0, 4], [2, 4, 0]], dtype=np.int64)
    assert (oracle.weights(d, oracle.WINNING_VOTES) == [[0, 5, 0], [0, 0, 0], [0, 0, 0]]).all()
    assert (oracle.weights(d, oracle.MARGIN) == [[0, 2, 0], [0, 0, 0], [0, 0, 0]]).all()


def test_weights_modes_distinguish_on_truncated():
    """Winning votes and margins can pick different winners once ballots are
    truncated (an instance of the paper's silence on the weight choice)."""
    rows = [[0, 1], [0, 2, 1], [1, 2, 0, 3], [1, 3, 0, 2], [2, 3, 0], [2, 3, 1], [3, 0, 1]]
    b = np.full((len(rows), 4), -1, dtype=np.int32)
    for i, r in enumerate(rows):
        b[i, :len(r)] = r
    d = oracle.pairwise(b, 4)
    res = {}
    for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
        w = oracle.weights(d, mode)
        p = oracle.closure(w)
        assert (p == brute.widest_by_paths(w)).all()
        res[mode] = brute.schulze_winners_from_p(p)
        _, win, _ = oracle.rank(p)
        assert {i for i in range(4) if win[i]} == res[mode]
    assert res[oracle.WINNING_VOTES] == {0, 1, 2, 3}
    assert res[oracle.MARGIN] == {0, 1, 2}


def test_figure1_topk_by_removal():
    """Top-k by iterated winner removal (Section 4's closing remark) on the
    Figure 1 graph, derived by hand from its edges: a wins; without a the
    cycle b->c (10), c->d (8), d->b (12) gives p(d,b) = 12 > p(b,d) = 8 and
    p(d,c) = 10 > p(c,d) = 8, so d wins; then b (edge b->c); then c."""
    g, idx, w, table = figure1()
    level = oracle.topk_levels(w, 4)
    assert [int(level[idx[c]]) for c in "abcd"] == [0, 2, 3, 1]
    assert [int(x) for x in oracle.topk_levels(w, 2)] == [0, -1, -1, 1]


# ---------------------------------------------------------------- top-k by winner removal

def _levels_as_lists(level):
    n = int(level.max()) + 1 if (level >= 0).any() else 0
    return [sorted(int(c) for c in np.nonzero(level == i)[0]) for i in range(n)]


def test_topk_brute_force_small():
    rng = np.random.default_rng(31)
    n_checked = 0
    for m, b, wts in _random_profiles(300, max_m=7, seed=29):
        d = oracle.pairwise(b, m, wts)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            w = oracle.weights(d, mode)
            k = int(rng.integers(1, m + 1))
            assert _levels_as_lists(oracle.topk_levels(w, k)) == brute.topk_by_removal(w, k)
            n_checked += 1
    assert n_checked == 600


def test_topk_removal_deletes_paths():
    """Edges 0->1 (5), 0->2 (3), 2->3 (1), 3->0 (3).  Candidate 3 beats all
    (p(3,0) = 3 > p(0,3) = 1, p(3,1) = 3, p(3,2) = 3 > p(2,3) = 1): level 0.
    Without 3, candidate 0 reaches 1 and 2 and nothing reaches 0: level 1.
    Without 3 and 0, 1 and 2 have no edges: both level 2.  On the full graph
    2 beats 1 through 3 and 0 (width 1 > 0), so the full ranking puts 2
    above 1: removal is a different order."""
    w = np.zeros((4, 4), dtype=np.int64)
    w[0, 1], w[0, 2], w[2, 3], w[3, 0] = 5, 3, 1, 3
    assert oracle.topk_levels(w, 4).tolist() == [1, 2, 2, 0]
    beaten, _, order = oracle.rank(oracle.closure(w))
    assert order.tolist() == [3, 0, 2, 1]


def test_topk_first_level_is_the_winner_set():
    for m, b, wts in _random_profiles(200, max_m=12, seed=37):
        w = oracle.weights(oracle.pairwise(b, m, wts), oracle.WINNING_VOTES)
        _, win, _ = oracle.rank(oracle.closure(w))
        level = oracle.topk_levels(w, 1)
        assert ((level == 0) == win).all()
        assert ((level == -1) == ~win).all()


def test_topk_single_full_ranking_is_that_ranking():
    rng = np.random.default_rng(41)
    for m in (1, 2, 5, 17, 40):
        order = rng.permutation(m).astype(np.int32)
        d = oracle.pairwise(order[None, :], m)
        level = oracle.topk_levels(oracle.weights(d, oracle.WINNING_VOTES), m)
        assert [int(level[c]) for c in order] == list(range(m))


def test_topk_levels_partition_and_stop_at_k():
    for m, b, wts in _random_profiles(150, max_m=14, seed=43):
        w = oracle.weights(oracle.pairwise(b, m, wts), oracle.MARGIN)
        full = oracle.topk_levels(w, m)
        assert (full >= 0).all()  # every candidate gets a level
        assert set(full.tolist()) == set(range(int(full.max()) + 1))  # no empty level
        for k in range(1, m + 1):
            part = oracle.topk_levels(w, k)
            reached = part >= 0
            assert reached.sum() >= k
            assert (part[reached] == full[reached]).all()
            last = int(part.max())
            assert (reached == (full <= last)).all()
            assert (full <= last - 1).sum() < k  # the last level was needed


# ---------------------------------------------------------------- closure

def test_closure_brute_force_small():
    n_checked = 0
    for m, b, wts in _random_profiles(400, max_m=7, seed=17):
        d = oracle.pairwise(b, m, wts)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            w = oracle.weights(d, mode)
            assert (oracle.closure(w) == brute.widest_by_paths(w)).all()
            n_checked += 1
    assert n_checked == 800


def test_closure_random_weights_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(200):
        m = int(rng.integers(1, 8))
        w = rng.integers(0, 6, size=(m, m)).astype(np.int64) * (rng.random((m, m)) < 0.6)
        np.fill_diagonal(w, 0)
        assert (oracle.closure(w) == brute.widest_by_paths(w)).all()


def test_closure_threshold_reachability():
    rng = np.random.default_rng(8)
    for _ in range(12):
        m = int(rng.integers(8, 30))
        b = workload.uniform_ballots(int(rng.integers(1 << 30)), 15, m, min_len=1, dtype=np.int32)
        w = oracle.weights(oracle.pairwise(b, m), oracle.WINNING_VOTES)
        assert (oracle.closure(w) == brute.threshold_widths(w)).all()


def test_closure_invariants_mid():
    b = workload.mallows(21, 300, 90, 0.95, trunc_mod=4, trunc_lt=2, trunc_k=10)
    w = oracle.weights(oracle.pairwise(b, 90), oracle.WINNING_VOTES)
    p = oracle.closure(w)
    off = ~np.eye(90, dtype=bool)
    assert (p[off] >= w[off]).all()
    assert set(np.unique(p)) <= set(np.unique(w)) | {0}
    assert (oracle.closure(p) == p).all()  # idempotent
    # support of p = transitive closure of the graph's edges
    for i in range(0, 90, 11):
        r = brute.reachable(w > 0, i)
        r[i] = False
        assert ((p[i] > 0) == r).all()


def test_widest_from_to_match_closure():
    b = workload.uniform_ballots(4, 30, 50, min_len=2, dtype=np.int32)
    w = oracle.weights(oracle.pairwise(b, 50), oracle.MARGIN)
    p = oracle.closure(w)
    for s in (0, 13, 49):
        assert (oracle.widest_from(w, s) == p[s]).all()
        assert (oracle.widest_to(w, s) == p[:, s]).all()
    rng = np.random.default_rng(2)
    for _ in range(60):
        m = int(rng.integers(1, 8))
        w = rng.integers(0, 5, size=(m, m)).astype(np.int64)
        np.fill_diagonal(w, 0)
        pb = brute.widest_by_paths(w)
        s = int(rng.integers(0, m))
        assert (oracle.widest_from(w, s) == pb[s]).all()
        assert (oracle.widest_to(w, s) == pb[:, s]).all()


# ---------------------------------------------------------------- winners, ranking

def _check_rank_properties(d, p):
    m = p.shape[0]
    beaten, win, order = oracle.rank(p)
    bt = brute.beats_matrix(p)
    assert (beaten == bt.sum(axis=0)).all()
    assert win.any(), "the Schulze method always has a winner"
    # beats is transitive (Section 2.1: the strict part of R)
    bi = bt.astype(np.int64)
    assert not ((bi @ bi > 0) & ~bt).any()
    # ranking: sorted by (beaten_by, id), a permutation, beats => lower level
    assert sorted(order) == list(range(m))
    keys = [(beaten[x], x) for x in order]
    assert keys == sorted(keys)
    xs, ys = np.nonzero(bt)
    assert (beaten[xs] < beaten[ys]).all()
    winners = {x for x in range(m) if win[x]}
    assert winners == brute.schulze_winners_from_p(p)
    # Schulze refines Schwartz (Section 2.1)
    assert winners <= brute.schwartz_set(d)
    # Condorcet winner / loser (Section 1: Condorcet consistency)
    dom = d > d.T
    for c in range(m):
        if all(dom[c, y] for y in range(m) if y != c):
            assert winners == {c}
        if m > 1 and all(dom[y, c] for y in range(m) if y != c):
            assert c not in winners
    return winners


def _filter_losers(w):
    """Initialisation filter (Section 4): largest incoming weight exceeds the
    largest outgoing weight => not a winner."""
    return {c for c in range(w.shape[0]) if w[:, c].max(initial=0) > w[c, :].max(initial=0)}


def test_rank_properties_random():
    for i, (m, b, wts) in enumerate(_random_profiles(300, max_m=7, seed=29)):
        d = oracle.pairwise(b, m, wts)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            w = oracle.weights(d, mode)
            p = oracle.closure(w)
            winners = _check_rank_properties(d, p)
            assert not (winners & _filter_losers(w))


def test_rank_properties_mid():
    for seed, m in ((1, 40), (2, 64), (3, 33)):
        b = workload.mallows(seed, 101, m, 0.9, trunc_mod=3, trunc_lt=1, trunc_k=7)
        d = oracle.pairwise(b, m)
        w = oracle.weights(d, oracle.WINNING_VOTES)
        winners = _check_rank_properties(d, oracle.closure(w))
        assert not (winners & _filter_losers(w))


def test_ranking_not_a_weak_order_when_widths_tie():
    """Two voters (w y x) and (x w y): p(w,y) = 2 and every other width is 0,
    so R (p(a,b) >= p(b,a)) has y R x and x R w but not y R w.  The oracle's
    ranking is then a linear extension of the strict beats relation."""
    W, X, Y = 0, 1, 2
    b = np.array([[W, Y, X], [X, W, Y]], dtype=np.int32)
    p = oracle.closure(oracle.weights(oracle.pairwise(b, 3), oracle.WINNING_VOTES))
    R = p >= p.T
    assert R[Y, X] and R[X, W] and not R[Y, W]
    beaten, win, order = oracle.rank(p)
    assert list(beaten) == [0, 0, 1] and list(order) == [W, X, Y]


def test_nl_reduction_matches_reachability():
    """a is the unique Schulze winner of the reduced graph iff b is reachable
    from a in G (NL-hardness proof, Section 3)."""
    rng = np.random.default_rng(13)
    seen = {True: 0, False: 0}
    for _ in range(80):
        m = int(rng.integers(2, 9))
        dens = float(rng.uniform(0.05, 0.4))
        edges = [(u, v) for u in range(m) for v in range(m) if u != v and rng.random() < dens]
        a, b = (int(x) for x in rng.choice(m, 2, replace=False))
        W = brute.nl_reduction(m, edges, a, b)
        adj = np.zeros((m, m), dtype=bool)
        for u, v in edges:
            adj[u, v] = True
        reach = bool(brute.reachable(adj, a)[b])
        _, win, _ = oracle.rank(oracle.closure(W))
        assert (bool(win[a]) and win.sum() == 1) == reach
        assert bool(win[a]) == reach
        seen[reach] += 1
    assert seen[True] > 5 and seen[False] > 5


# ---------------------------------------------------------------- planted mistakes

def _closure_wrong_index(w):
    """p[k][i] read where p[i][k] belongs."""
    m = w.shape[0]
    p = w.copy()
    for k in range(m):
        for i in range(m):
            for j in range(m):
                p[i, j] = max(p[i, j], min(p[k, i], p[k, j]))
    np.fill_diagonal(p, 0)
    return p


def _closure_one_hop(w):
    """A 'closure' that forgets paths longer than two edges."""
    m = w.shape[0]
    p = w.copy()
    for i in range(m):
        for j in range(m):
            for k in range(m):
                p[i, j] = max(p[i, j], min(w[i, k], w[k, j]))
    np.fill_diagonal(p, 0)
    return p


def _closure_minmax_swapped(w):
    m = w.shape[0]
    p = w.copy()
    for k in range(m):
        for i in range(m):
            for j in range(m):
                p[i, j] = min(p[i, j], max(p[i, k], p[k, j]))
    np.fill_diagonal(p, 0)
    return p


@pytest.mark.parametrize("bad", [_closure_wrong_index, _closure_one_hop, _closure_minmax_swapped])
def test_pins_catch_planted_closure_mistakes(bad):
    g, idx, w, table = figure1()
    caught = not (bad(w) == table).all()
    rng = np.random.default_rng(0)
    for _ in range(50):
        if caught:
            break
        m = int(rng.integers(3, 7))
        ww = rng.integers(0, 6, size=(m, m)).astype(np.int64)
        np.fill_diagonal(ww, 0)
        caught = not (bad(ww) == brute.widest_by_paths(ww)).all()
    assert caught


def test_pins_catch_planted_count_mistakes():
    b = workload.uniform_ballots(1, 20, 6, dtype=np.int32)
    good = brute.count_pairs(b, 6)
    assert (oracle.pairwise(b, 6) == good).all()
    # ties counted as preference (>= instead of >) or a transposed d
    d = oracle.pairwise(b, 6)
    assert not (d.T == good).all()
    ge = good.copy()
    for row in b:
        lst = brute.listed(row)
        rest = [y for y in range(6) if y not in lst]
        for x in rest:
            for y in rest:
                if x != y:
                    ge[x, y] += 1
    assert not (ge == good).all()
