"""Property tests of the oracle (hypothesis, derandomized so every run draws
the same cases): on small random profiles -- truncated, padded, with voter
weights -- the oracle's counts equal the pair lists, its widths equal the
widest simple path found by enumeration, Schulze winners lie in the Schwartz
set, a Condorcet winner is the unique winner, and the winners are the
candidates nobody beats."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from tests import brute


@st.composite
def profiles(draw, max_m=6, max_n=12):
    m = draw(st.integers(1, max_m))
    n = draw(st.integers(1, max_n))
    L = draw(st.integers(1, m))
    rows = []
    for _ in range(n):
        perm = draw(st.permutations(list(range(m))))
        k = draw(st.integers(0, L))
        rows.append(list(perm[:k]) + [0xFFFF] * (L - k))
    b = np.array(rows, dtype=np.uint16).reshape(n, L)
    weighted = draw(st.booleans())
    w = np.array([draw(st.integers(0, 5)) for _ in range(n)], dtype=np.uint32) if weighted else None
    mode = draw(st.sampled_from([oracle.WINNING_VOTES, oracle.MARGIN]))
    return m, b, w, mode


@settings(max_examples=300, deadline=None, derandomize=True)
@given(profiles())
def test_oracle_against_brute_force(case):
    m, b, w, mode = case
    d = oracle.pairwise(b, m, w)
    assert (d == brute.count_pairs(b, m, w)).all()
    wt = oracle.weights(d, mode)
    p = oracle.closure(wt)
    assert (p == brute.widest_by_paths(wt)).all()
    beaten, win, order = oracle.rank(p)
    winners = set(np.flatnonzero(win).tolist())
    assert winners == brute.schulze_winners_from_p(p)
    assert winners, "every election has a Schulze winner"
    assert winners <= brute.schwartz_set(d)
    condorcet = [x for x in range(m) if all(d[x][y] > d[y][x] for y in range(m) if y != x)]
    if condorcet:
        assert winners == {condorcet[0]}
    assert sorted(order.tolist()) == list(range(m))
    assert all(beaten[order[i]] <= beaten[order[i + 1]] for i in range(m - 1))
