"""Independent brute-force references used to pin the oracle.

Pure Python, written from the definitions in a different form than the
oracle (pair lists instead of rank comparisons, path enumeration instead of
Floyd-Warshall, graph search instead of matrices), so that a mistake in one
is not repeated in the other.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def listed(ballot) -> list[int]:
    """The listed prefix of a ballot row (stops at the first padding entry)."""
    out = []
    for c in ballot:
        c = int(c)
        if c < 0 or c == 0xFFFF:
            break
        out.append(c)
    return out


def count_pairs(ballots, m: int, weight=None) -> np.ndarray:
    """d[x][y] from pair lists: for every ballot, each listed x gets the
    ballot's weight against every candidate listed after it and against
    every unlisted candidate (Section 2.1: weak orders, unlisted tied last)."""
    d = np.zeros((m, m), dtype=np.int64)
    for v, row in enumerate(ballots):
        om = 1 if weight is None else int(weight[v])
        lst = listed(row)
        seen = set(lst)
        rest = [y for y in range(m) if y not in seen]
        for i, x in enumerate(lst):
            for y in lst[i + 1:]:
                d[x, y] += om
            for y in rest:
                d[x, y] += om
    return d


def widest_by_paths(w: np.ndarray) -> np.ndarray:
    """p[a][b] = max over simple a->b paths of the smallest edge weight on the
    path (edges are entries > 0); 0 when b is unreachable; diagonal 0.
    Exponential: only for m <= 7."""
    m = w.shape[0]
    p = np.zeros((m, m), dtype=np.int64)

    def dfs(a, u, width, on_path):
        for v in range(m):
            e = int(w[u, v])
            if e <= 0 or v in on_path:
                continue
            nw = e if width is None else min(width, e)
            if v != a and nw > p[a, v]:
                p[a, v] = nw
            on_path.add(v)
            dfs(a, v, nw, on_path)
            on_path.remove(v)

    for a in range(m):
        dfs(a, a, None, {a})
    return p


def reachable(adj: np.ndarray, s: int) -> np.ndarray:
    """BFS over a boolean adjacency matrix; the source counts as reached."""
    m = adj.shape[0]
    seen = np.zeros(m, dtype=bool)
    seen[s] = True
    q = deque([s])
    while q:
        u = q.popleft()
        for v in np.nonzero(adj[u])[0]:
            if not seen[v]:
                seen[v] = True
                q.append(v)
    return seen


def threshold_widths(w: np.ndarray) -> np.ndarray:
    """p[i][j] = largest t such that j is reachable from i using only edges of
    weight >= t (0 if none): the widest-path width as a threshold search."""
    m = w.shape[0]
    p = np.zeros((m, m), dtype=np.int64)
    for t in sorted(set(int(x) for x in w.ravel() if x > 0)):
        adj = w >= t
        for i in range(m):
            r = reachable(adj, i)
            r[i] = False
            # the reached set of i itself is not reached by i unless via a cycle
            p[i, r] = t
    np.fill_diagonal(p, 0)
    return p


def beats_matrix(p: np.ndarray) -> np.ndarray:
    return p > p.T


def schulze_winners_from_p(p: np.ndarray) -> set[int]:
    b = beats_matrix(p)
    return {x for x in range(p.shape[0]) if not b[:, x].any()}


def tarjan_scc(adj: np.ndarray) -> list[list[int]]:
    """Strongly connected components (Tarjan, iterative)."""
    m = adj.shape[0]
    index = [None] * m
    low = [0] * m
    on = [False] * m
    stack, comps, counter = [], [], [0]
    nbrs = [list(np.nonzero(adj[u])[0]) for u in range(m)]
    for root in range(m):
        if index[root] is not None:
            continue
        work = [(root, 0)]
        while work:
            u, i = work.pop()
            if i == 0:
                index[u] = low[u] = counter[0]
                counter[0] += 1
                stack.append(u)
                on[u] = True
            recurse = False
            while i < len(nbrs[u]):
                v = nbrs[u][i]
                i += 1
                if index[v] is None:
                    work.append((u, i))
                    work.append((v, 0))
                    recurse = True
                    break
                if on[v]:
                    low[u] = min(low[u], index[v])
            if recurse:
                continue
            if low[u] == index[u]:
                comp = []
                while True:
                    x = stack.pop()
                    on[x] = False
                    comp.append(x)
                    if x == u:
                        break
                comps.append(sorted(comp))
            if work:
                parent = work[-1][0]
                low[parent] = min(low[parent], low[u])
    return comps


def schwartz_set(d: np.ndarray) -> set[int]:
    """Union of the SCCs of the dominance graph (x -> y iff d[x][y] > d[y][x])
    that no outside vertex dominates (Section 2.1)."""
    dom = d > d.T
    out = set()
    for comp in tarjan_scc(dom):
        cs = set(comp)
        others = [x for x in range(d.shape[0]) if x not in cs]
        if not any(dom[o, c] for o in others for c in comp):
            out |= cs
    return out


def mcgarvey_ballots(m: int, edges) -> np.ndarray:
    """McGarvey's construction (cited in Section 3): for an edge (a, b) of even
    weight mu, mu/2 pairs of linear orders [a, b, rest ascending] and
    [rest descending, a, b]; each pair adds margin +2 to (a, b) and 0 to every
    other pair.  Returns int32 ballots (sum of mu rows, m columns)."""
    rows = []
    for a, b, mu in edges:
        assert mu > 0 and mu % 2 == 0
        rest = [c for c in range(m) if c not in (a, b)]
        for _ in range(mu // 2):
            rows.append([a, b] + rest)
            rows.append(rest[::-1] + [a, b])
    return np.array(rows, dtype=np.int32).reshape(-1, m)


def nl_reduction(m: int, edges, a: int, b: int):
    """The NL-hardness reduction of Section 3 from Reachability (G, a, b):
    drop edges into a and out of b; replace one edge of every symmetric pair
    by a midpoint vertex; add r_u with edges (b, r_u), (r_u, u) for every
    u != b; weight 2 on (r_a, a) and 4 elsewhere.  Returns the weight matrix
    of the new graph (vertices 0..m-1 keep their ids)."""
    E = {(u, v) for (u, v) in edges if u != v and v != a and u != b}
    out = []
    nid = m
    done = set()
    for (u, v) in sorted(E):
        if (u, v) in done:
            continue
        if (v, u) in E:
            wmid = nid
            nid += 1
            out += [(u, wmid), (wmid, v), (v, u)]
            done |= {(u, v), (v, u)}
        else:
            out.append((u, v))
            done.add((u, v))
    r_of = {}
    for u in range(m):
        if u == b:
            continue
        r_of[u] = nid
        out += [(b, nid), (nid, u)]
        nid += 1
    W = np.zeros((nid, nid), dtype=np.int64)
    for (u, v) in out:
        W[u, v] = 4
    W[r_of[a], a] = 2
    return W


def topk_by_removal(w: np.ndarray, k: int) -> list[list[int]]:
    """Levels of top-k by iterated winner removal, as lists of candidate ids:
    the Schulze winners of the candidates left (widths by path enumeration
    on the subgraph they induce), removed, again, until at least k are
    ranked or none is left.  Exponential: only for m <= 7."""
    left = list(range(w.shape[0]))
    levels: list[list[int]] = []
    ranked = 0
    while left and ranked < k:
        sub = np.array([[int(w[a, b]) for b in left] for a in left], dtype=np.int64).reshape(len(left), len(left))
        win = sorted(left[i] for i in schulze_winners_from_p(widest_by_paths(sub)))
        levels.append(win)
        ranked += len(win)
        left = [c for c in left if c not in win]
    return levels


def features(ballots, m: int, n_voters: float, mode: int) -> np.ndarray:
    """The 16 per-candidate feature columns, one candidate at a time from
    pair-list counts (Python integers, exact), scaled in float64 at the end.

    Columns (x = the candidate, y over the other m-1 candidates; "edge
    weight" is the tournament graph's, winning votes for mode 0, positive
    margin for mode 1, Section 2.1):
      0 wins (d[x][y] > d[y][x]) / (m-1)    1 ties (d[x][y] = d[y][x]) / (m-1)
      2 sum d[x][y] / (m-1) / n             3 largest out-weight / n
      4 largest in-weight / n               5 1 if in-weight max > out-weight max
      6 sum out-weights / (m-1) / n         7 sum in-weights / (m-1) / n
      8 smallest d[x][y]-d[y][x] / n        9 largest d[x][y]-d[y][x] / n
      10 ln(m) / 10                         11 wins / most wins of any candidate
      12 sum d[x][y] / the largest such sum 13 largest out-weight / its largest value
      14 (largest out - largest in) / n     15 1
    Ratios over a zero maximum are 0; with m = 1 every sum and extreme is 0."""
    d = count_pairs(ballots, m)

    def edge(a, b):
        da, db = int(d[a, b]), int(d[b, a])
        if da <= db:
            return 0
        return da if mode == 0 else da - db

    rows = []
    for x in range(m):
        wins = ties = borda = 0
        out_w, in_w = [], []
        margins = []
        for y in range(m):
            if y == x:
                continue
            a, b = int(d[x, y]), int(d[y, x])
            wins += a > b
            ties += a == b
            borda += a
            out_w.append(edge(x, y))
            in_w.append(edge(y, x))
            margins.append(a - b)
        rows.append({"wins": wins, "ties": ties, "borda": borda,
                     "out_max": max(out_w, default=0), "in_max": max(in_w, default=0),
                     "out_sum": sum(out_w), "in_sum": sum(in_w),
                     "mg_min": min(margins, default=0), "mg_max": max(margins, default=0)})
    den = (m - 1) if m > 1 else None
    n = float(n_voters) if n_voters > 0 else 1.0
    top_wins = max(r["wins"] for r in rows)
    top_borda = max(r["borda"] for r in rows)
    top_out = max(r["out_max"] for r in rows)
    F = np.zeros((m, 16), dtype=np.float64)
    for x, r in enumerate(rows):
        per = (lambda v: v / den) if den else (lambda v: 0.0)
        F[x] = [per(r["wins"]), per(r["ties"]), per(r["borda"]) / n,
                r["out_max"] / n, r["in_max"] / n, 1.0 if r["in_max"] > r["out_max"] else 0.0,
                per(r["out_sum"]) / n, per(r["in_sum"]) / n,
                r["mg_min"] / n, r["mg_max"] / n,
                np.log(m) / 10.0,
                r["wins"] / top_wins if top_wins else 0.0,
                r["borda"] / top_borda if top_borda else 0.0,
                r["out_max"] / top_out if top_out else 0.0,
                (r["out_max"] - r["in_max"]) / n, 1.0]
    return F
