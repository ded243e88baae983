"""CPU oracle for the Schulze method's hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the GPU library (``paper_2505_12976_amd``).

The arithmetic lives in ``oracle.c`` (plain C, 64-bit integers, OpenMP over
independent output rows); this module builds it with gcc, loads it with
ctypes and converts numpy arrays.  Each function restates a definition from
the paper's voting preliminaries (Section 2.1):

* :func:`pairwise`  -- d[x][y], total weight of voters preferring x to y.
* :func:`weights`   -- weighted tournament graph: winning votes (mode 0) or
  majority margin (mode 1, the paper's mu).
* :func:`closure`   -- p(a,b), width of a widest path (Floyd-Warshall over
  (max, min), the original sequential algorithm named in Section 5.2).
* :func:`rank`      -- beats relation, winners, ranking by (beaten_by, id).
* :func:`widest_from` / :func:`widest_to` -- single-source/target widest
  paths by dense Dijkstra (the path problems of the NL-membership proof,
  Section 3).
* :func:`topk_levels` -- top-k by repeatedly taking the Schulze winners of
  the candidates not yet ranked and removing them (the closing remark of
  Section 4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

WINNING_VOTES = 0
MARGIN = 1


class OracleError(RuntimeError):
    pass


def build() -> str:
    """Compile oracle.c into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                           _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_pairwise.argtypes = [vp, ctypes.c_int, i64, i32, i32, vp, vp]
    lib.oracle_pairwise_rows.argtypes = [vp, ctypes.c_int, i64, i32, i32, vp, vp, i64, vp]
    lib.oracle_pairwise_cols.argtypes = [vp, ctypes.c_int, i64, i32, i32, vp, vp, i64, vp]
    lib.oracle_weights.argtypes = [vp, i32, ctypes.c_int, vp]
    lib.oracle_closure.argtypes = [vp, i32, vp]
    lib.oracle_rank.argtypes = [vp, i32, vp, vp, vp]
    lib.oracle_widest_from.argtypes = [vp, i32, i32, vp]
    lib.oracle_widest_to.argtypes = [vp, i32, i32, vp]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    for name in ("oracle_pairwise", "oracle_pairwise_rows", "oracle_pairwise_cols", "oracle_weights",
                 "oracle_closure", "oracle_rank", "oracle_widest_from", "oracle_widest_to", "oracle_set_threads"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise OracleError(f"{what} failed with code {rc}")
    return rc


def _ballots(ballots: np.ndarray):
    b = np.ascontiguousarray(ballots)
    if b.ndim != 2:
        raise ValueError("ballots must be an (n, L) array")
    if b.dtype == np.uint16:
        return b, 0
    if b.dtype == np.int32:
        return b, 1
    raise ValueError("ballots must be uint16 or int32")


def _weights_arg(weight, n):
    if weight is None:
        return None, None
    w = np.ascontiguousarray(weight, dtype=np.uint32)
    if w.shape != (n,):
        raise ValueError("voter weights must have shape (n,)")
    return w, w.ctypes.data


def pairwise(ballots: np.ndarray, m: int, weight=None) -> np.ndarray:
    """d[x][y] = total weight of voters ranking x strictly above y (int64, m x m)."""
    b, d32 = _ballots(ballots)
    n, L = b.shape
    w, wp = _weights_arg(weight, n)
    d = np.empty((m, m), dtype=np.int64)
    _check(_load().oracle_pairwise(b.ctypes.data, d32, n, L, m, wp, d.ctypes.data), "oracle_pairwise")
    return d


def pairwise_rows(ballots: np.ndarray, m: int, rows, weight=None) -> np.ndarray:
    """Rows of d for the listed candidates: out[r] = d[rows[r], :]."""
    b, d32 = _ballots(ballots)
    n, L = b.shape
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    w, wp = _weights_arg(weight, n)
    out = np.empty((len(rows), m), dtype=np.int64)
    _check(_load().oracle_pairwise_rows(b.ctypes.data, d32, n, L, m, wp, rows.ctypes.data, len(rows),
                                        out.ctypes.data), "oracle_pairwise_rows")
    return out


def pairwise_cols(ballots: np.ndarray, m: int, cols, weight=None) -> np.ndarray:
    """Columns of d for the listed candidates: out[c] = d[:, cols[c]]."""
    b, d32 = _ballots(ballots)
    n, L = b.shape
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    w, wp = _weights_arg(weight, n)
    out = np.empty((len(cols), m), dtype=np.int64)
    _check(_load().oracle_pairwise_cols(b.ctypes.data, d32, n, L, m, wp, cols.ctypes.data, len(cols),
                                        out.ctypes.data), "oracle_pairwise_cols")
    return out


def weights(d: np.ndarray, mode: int = WINNING_VOTES) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.int64)
    m = d.shape[0]
    w = np.empty_like(d)
    _check(_load().oracle_weights(d.ctypes.data, m, mode, w.ctypes.data), "oracle_weights")
    return w


def closure(w: np.ndarray) -> np.ndarray:
    """Widest-path widths p (int64, zero diagonal) of the weight matrix w."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    m = w.shape[0]
    p = np.empty_like(w)
    _check(_load().oracle_closure(w.ctypes.data, m, p.ctypes.data), "oracle_closure")
    return p


def rank(p: np.ndarray):
    """(beaten_by int32[m], is_winner bool[m], order int32[m])."""
    p = np.ascontiguousarray(p, dtype=np.int64)
    m = p.shape[0]
    beaten = np.empty(m, dtype=np.int32)
    win = np.empty(m, dtype=np.uint8)
    order = np.empty(m, dtype=np.int32)
    _check(_load().oracle_rank(p.ctypes.data, m, beaten.ctypes.data, win.ctypes.data,
                               order.ctypes.data), "oracle_rank")
    return beaten, win.astype(bool), order


def widest_from(w: np.ndarray, s: int) -> np.ndarray:
    """out[v] = p(s, v); out[s] = 0."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    out = np.empty(w.shape[0], dtype=np.int64)
    _check(_load().oracle_widest_from(w.ctypes.data, w.shape[0], s, out.ctypes.data), "oracle_widest_from")
    return out


def widest_to(w: np.ndarray, t: int) -> np.ndarray:
    """out[v] = p(v, t); out[t] = 0."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    out = np.empty(w.shape[0], dtype=np.int64)
    _check(_load().oracle_widest_to(w.ctypes.data, w.shape[0], t, out.ctypes.data), "oracle_widest_to")
    return out


def topk_levels(w: np.ndarray, k: int) -> np.ndarray:
    """level[c] = the round in which c is a Schulze winner of the candidates
    left after removing the winners of all earlier rounds, for the rounds
    needed to rank at least k candidates (all rounds when k >= m); -1 for
    candidates not reached.  Removing a candidate deletes its edges, so each
    round's widths come from the closure of the subgraph induced by the
    candidates still in (Section 4, last remark of the algorithm's
    description; the winners of a round are those no remaining candidate
    beats, Section 2.1)."""
    w = np.asarray(w, dtype=np.int64)
    m = w.shape[0]
    level = np.full(m, -1, dtype=np.int32)
    alive = np.ones(m, dtype=bool)
    ranked, rnd = 0, 0
    while ranked < k and alive.any():
        idx = np.nonzero(alive)[0]
        p = closure(w[np.ix_(idx, idx)])
        beaten = (p.T > p).any(axis=1)  # some remaining y with p(y, x) > p(x, y)
        win = idx[~beaten]
        level[win] = rnd
        alive[win] = False
        ranked += len(win)
        rnd += 1
    return level


def set_threads(threads: int) -> int:
    """Threads of the oracle's parallel loops (timing only); returns the previous count."""
    return int(_load().oracle_set_threads(int(threads)))


def schulze(ballots: np.ndarray, m: int, mode: int = WINNING_VOTES, weight=None) -> dict:
    """The whole path on the CPU: d, w, p, beaten_by, winners, order."""
    d = pairwise(ballots, m, weight)
    w = weights(d, mode)
    p = closure(w)
    beaten, win, order = rank(p)
    return {"d": d, "w": w, "p": p, "beaten_by": beaten, "is_winner": win, "order": order}


def features(d: np.ndarray, n_voters: float, mode: int = WINNING_VOTES) -> np.ndarray:
    """m x 16 per-candidate features of the weighted tournament graph (float64
    arithmetic, float32 result); column meanings as in the GPU library."""
    d = np.asarray(d, dtype=np.int64)
    m = d.shape[0]
    dt = d.T
    off = ~np.eye(m, dtype=bool)
    w_out = np.where(off & (d > dt), d if mode == WINNING_VOTES else d - dt, 0)
    w_in = w_out.T
    marg = np.where(off, d - dt, 0)
    cope = ((d > dt) & off).sum(axis=1)
    ties = ((d == dt) & off).sum(axis=1)
    borda = np.where(off, d, 0).sum(axis=1)
    mx_out, mx_in = w_out.max(axis=1), w_in.max(axis=1)
    big = np.iinfo(np.int64).max
    mn = np.where(off, marg, big).min(axis=1) if m > 1 else np.zeros(m, dtype=np.int64)
    mxm = np.where(off, marg, -big).max(axis=1) if m > 1 else np.zeros(m, dtype=np.int64)
    inv_m1 = 1.0 / (m - 1) if m > 1 else 0.0
    inv_n = 1.0 / n_voters if n_voters > 0 else 1.0
    F = np.zeros((m, 16), dtype=np.float64)
    F[:, 0] = cope * inv_m1
    F[:, 1] = ties * inv_m1
    F[:, 2] = borda * inv_m1 * inv_n
    F[:, 3] = mx_out * inv_n
    F[:, 4] = mx_in * inv_n
    F[:, 5] = (mx_in > mx_out).astype(np.float64)
    F[:, 6] = w_out.sum(axis=1) * inv_m1 * inv_n
    F[:, 7] = w_in.sum(axis=1) * inv_m1 * inv_n
    F[:, 8] = mn * inv_n
    F[:, 9] = mxm * inv_n
    F[:, 10] = np.log(m) * 0.1
    F[:, 11] = cope / cope.max() if cope.max() > 0 else 0.0
    F[:, 12] = borda / borda.max() if borda.max() > 0 else 0.0
    F[:, 13] = mx_out / mx_out.max() if mx_out.max() > 0 else 0.0
    F[:, 14] = (mx_out - mx_in) * inv_n
    F[:, 15] = 1.0
    return F.astype(np.float32)
