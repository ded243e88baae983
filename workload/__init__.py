"""Seeded synthetic preference profiles for the Schulze method.

The ballots stand in for the paper's Spotify chart profiles (Section 5.1,
Table 1), which are not available: full or truncated rankings drawn from a
Mallows model, and top-k rankings drawn from Plackett-Luce with Zipf weights.
The generator is plain C (``gen.c``); this module builds it, loads it with
ctypes and names the workloads.  It holds no part of the method's
arithmetic, so the CPU oracle and the GPU library can both take its output
as input bytes.

Ballot layout: ``(n, L)`` array of candidate ids, best first, padded with
0xFFFF (uint16) or -1 (int32); unlisted candidates are unranked and tied
below every ranked one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None

GEN_FLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas"]


def build() -> str:
    """Compile gen.c into libgen.so next to it (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *GEN_FLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gen_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, i32p]
    lib.gen_mallows.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_double, i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_int, ctypes.c_void_p]
    lib.gen_pl_zipf.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_double, i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                ctypes.c_void_p]
    lib.gen_uniform_int.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.gen_uniform_real.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.gen_uniform_ballots.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p]
    lib.gen_mallows_topk.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_double, i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                     ctypes.c_void_p]
    for f in (lib.gen_permutation, lib.gen_mallows, lib.gen_pl_zipf, lib.gen_uniform_int,
              lib.gen_uniform_real, lib.gen_uniform_ballots, lib.gen_mallows_topk):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def permutation(seed: int, stream: int, m: int) -> np.ndarray:
    out = np.empty(m, dtype=np.int32)
    _check(_load().gen_permutation(seed, stream, m, _i32p(out)), "gen_permutation")
    return out


def _ballot_dtype(m: int, dtype):
    if dtype is None:
        dtype = np.uint16 if m <= 65535 else np.int32
    dtype = np.dtype(dtype)
    if dtype not in (np.dtype(np.uint16), np.dtype(np.int32)):
        raise ValueError("ballot dtype must be uint16 or int32")
    return dtype


def mallows(seed: int, n: int, m: int, phi: float, *, election: int = 0, L: int | None = None,
            trunc_mod: int = 0, trunc_lt: int = 0, trunc_k: int = 0, ref_order=None,
            dtype=None) -> np.ndarray:
    """Mallows(phi) rankings around a seeded reference order.

    Voter v is cut to its top ``trunc_k`` when ``v % trunc_mod < trunc_lt``.
    """
    dtype = _ballot_dtype(m, dtype)
    L = m if L is None else L
    if ref_order is None:
        ref_order = permutation(seed, election, m)
    ref_order = np.ascontiguousarray(ref_order, dtype=np.int32)
    out = np.empty((n, L), dtype=dtype)
    rc = _load().gen_mallows(seed, election, n, m, phi, _i32p(ref_order), L, trunc_mod, trunc_lt,
                             trunc_k, int(dtype == np.int32), out.ctypes.data)
    _check(rc, "gen_mallows")
    return out


def pl_zipf(seed: int, n: int, m: int, s: float, k: int, *, election: int = 0, L: int | None = None,
            pop_order=None, dtype=None) -> np.ndarray:
    """Top-k Plackett-Luce rankings with Zipf(s) weights over a seeded popularity order."""
    dtype = _ballot_dtype(m, dtype)
    L = k if L is None else L
    if pop_order is None:
        pop_order = permutation(seed, election, m)
    pop_order = np.ascontiguousarray(pop_order, dtype=np.int32)
    out = np.empty((n, max(L, 1)), dtype=dtype)
    rc = _load().gen_pl_zipf(seed, election, n, m, s, _i32p(pop_order), k, max(L, 1),
                             int(dtype == np.int32), out.ctypes.data)
    _check(rc, "gen_pl_zipf")
    return out


def mallows_topk(seed: int, n: int, m: int, phi: float, k: int, *, election: int = 0, L: int | None = None,
                 ref_order=None, dtype=None) -> np.ndarray:
    """Top-k of Mallows(phi) rankings (inversion-vector sampling, O(k^2) per voter)."""
    dtype = _ballot_dtype(m, dtype)
    L = k if L is None else L
    if ref_order is None:
        ref_order = permutation(seed, election, m)
    ref_order = np.ascontiguousarray(ref_order, dtype=np.int32)
    out = np.empty((n, max(L, 1)), dtype=dtype)
    rc = _load().gen_mallows_topk(seed, election, n, m, phi, _i32p(ref_order), k, max(L, 1),
                                  int(dtype == np.int32), out.ctypes.data)
    _check(rc, "gen_mallows_topk")
    return out


def uniform_ballots(seed: int, n: int, m: int, L: int | None = None, *, min_len: int = 0,
                    election: int = 0, dtype=None) -> np.ndarray:
    """Random-length lists of distinct random ids (heavy ties, edge cases)."""
    dtype = _ballot_dtype(m, dtype)
    L = m if L is None else L
    out = np.empty((n, L), dtype=dtype)
    rc = _load().gen_uniform_ballots(seed, election, n, m, L, min_len, int(dtype == np.int32),
                                     out.ctypes.data)
    _check(rc, "gen_uniform_ballots")
    return out


def uniform_int(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    rc = _load().gen_uniform_int(seed, stream, count, lo, hi,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    _check(rc, "gen_uniform_int")
    return out


def uniform_real(seed: int, stream: int, count: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    rc = _load().gen_uniform_real(seed, stream, count, lo, hi,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(rc, "gen_uniform_real")
    return out


# ---------------------------------------------------------------------------
# Named workloads.  Each stands in for a preference data set of the paper's
# shape (dense tournament graphs built from truncated rankings, Section 5.1).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    m: int
    n: int
    ballots: np.ndarray
    d_dtype: str                     # "u16" or "i32": counter width of d and p
    recipe: str
    extra: dict = field(default_factory=dict)


def plain_small(seed: int = 1001) -> Workload:
    """m=64, n=1000 full Mallows(0.8) rankings; int32 counts."""
    b = mallows(seed, 1000, 64, 0.8)
    return Workload("mallows_m64_n1000", 64, 1000, b, "i32",
                    "Mallows phi=0.8, full rankings, m=64, n=1000, seed %d" % seed)


def plain_mid(seed: int = 1002, n: int = 60000, m: int = 4096) -> Workload:
    """m=4096, n=60000 Mallows(0.97); voters with v % 10 < 3 cut to top-100; uint16 counts."""
    b = mallows(seed, n, m, 0.97, trunc_mod=10, trunc_lt=3, trunc_k=100)
    return Workload("mallows_m%d_n%d_top100x30pct" % (m, n), m, n, b, "u16",
                    "Mallows phi=0.97, m=%d, n=%d, v%%10<3 truncated to top-100, seed %d" % (m, n, seed))


def plain_large(seed: int = 1003, n: int = 1_000_000, m: int = 16384) -> Workload:
    """m=16384, n=1e6 top-20 Plackett-Luce with Zipf(1.1) weights; int32 counts."""
    b = pl_zipf(seed, n, m, 1.1, 20)
    return Workload("plzipf_m%d_n%d_top20" % (m, n), m, n, b, "i32",
                    "Plackett-Luce Zipf s=1.1, top-20, m=%d, n=%d, seed %d" % (m, n, seed))


def plain_paper(seed: int = 1006, n: int = 15553, m: int = 14187) -> Workload:
    """The paper's largest chart shape (m=14187 candidates, n=15553 voters,
    top-150 lists; Table 1), drawn here as Plackett-Luce with Zipf(1.0)
    weights; uint16 counts.  For context next to the paper's single-core
    timings; no chart data is used."""
    b = pl_zipf(seed, n, m, 1.0, 150)
    return Workload("plzipf_m%d_n%d_top150" % (m, n), m, n, b, "u16",
                    "Plackett-Luce Zipf s=1.0, top-150, m=%d, n=%d, seed %d" % (m, n, seed))


def plain_learned(seed: int = 1005, n: int = 200_000, m: int = 32768) -> Workload:
    """m=32768, n=200000 top-30 Plackett-Luce with Zipf(1.0) weights; int32 counts."""
    b = pl_zipf(seed, n, m, 1.0, 30)
    return Workload("plzipf_m%d_n%d_top30" % (m, n), m, n, b, "i32",
                    "Plackett-Luce Zipf s=1.0, top-30, m=%d, n=%d, seed %d" % (m, n, seed))


def batch_params(seed: int = 1004, count: int = 4096, m_lo: int = 8, m_hi: int = 512, n_lo: int = 50,
                 n_hi: int = 20000, phi_lo: float = 0.5, phi_hi: float = 1.0):
    """Per-election sizes of a batch of independent elections:
    m ~ U{m_lo..m_hi}, n ~ U{n_lo..n_hi}, phi ~ U[phi_lo, phi_hi]."""
    ms = uniform_int(seed, 11, count, m_lo, m_hi)
    ns = uniform_int(seed, 12, count, n_lo, n_hi)
    phis = uniform_real(seed, 13, count, phi_lo, phi_hi)
    return ms.astype(np.int64), ns.astype(np.int64), phis


def batch_election(seed: int, e: int, m: int, n: int, phi: float) -> np.ndarray:
    """Ballots of election e of a batch: n full Mallows(phi) rankings (uint16)
    around the election's own seeded reference order."""
    return mallows(seed, int(n), int(m), float(phi), election=int(e), dtype=np.uint16)


def batch_mallows(seed: int = 1004, count: int = 4096, progress=None, **size_kw):
    """A batch of `count` elections of full Mallows rankings with the sizes of
    batch_params, ballots written back to back into one flat uint16 array.
    Returns (flat ballots, descriptors, (ms, ns, phis)); a descriptor is
    (ballot_off, n, L, m, mat_off, vec_off) with L = m and the m x m and
    m-entry output blocks laid out back to back.  progress: None or a
    callable given the number of elections generated, every 512."""
    ms, ns, phis = batch_params(seed, count, **size_kw)
    total = int(np.sum(ms * ns))
    flat = np.empty(max(total, 1), dtype=np.uint16)
    desc = []
    bo = mo = vo = 0
    lib = _load()
    for e in range(count):
        m, n = int(ms[e]), int(ns[e])
        ref = permutation(seed, e, m)
        rc = lib.gen_mallows(seed, e, n, m, float(phis[e]), _i32p(ref), m, 0, 0, 0, 0,
                             flat.ctypes.data + 2 * bo)
        _check(rc, "gen_mallows")
        desc.append((bo, n, m, m, mo, vo))
        if progress is not None and (e + 1) % 512 == 0:
            progress(e + 1)
        bo += n * m
        mo += m * m
        vo += m
    return flat, desc, (ms, ns, phis)


def training_mixture(seed: int, count: int, m_lo: int = 256, m_hi: int = 2048, full_m_hi: int = 1024):
    """Elections for training the proposer: m ~ U{m_lo..m_hi}, n = round(rho m)
    with rho ~ U[3, 12].  Election e is, by e mod 10:
      0-4  Plackett-Luce top-k with Zipf(s) weights, s ~ U[0.8, 1.2], k ~ U{10..50};
      5-8  Mallows top-k, phi ~ U[0.9, 1.0], k ~ U{10..50};
      9    full Mallows rankings, phi ~ U[0.9, 1.0], with m capped at full_m_hi
           (near phi = 1 these often have no Condorcet winner).
    Yields dicts with the ballots (uint16) and the drawn parameters."""
    ms = uniform_int(seed, 1, count, m_lo, m_hi)
    rhos = uniform_real(seed, 2, count, 3.0, 12.0)
    ks = uniform_int(seed, 3, count, 10, 50)
    ss = uniform_real(seed, 4, count, 0.8, 1.2)
    phis = uniform_real(seed, 5, count, 0.9, 1.0)
    for e in range(count):
        m, k = int(ms[e]), int(ks[e])
        kind_id = e % 10
        if kind_id == 9:
            m = min(m, full_m_hi)
        n = int(round(rhos[e] * m))
        if kind_id <= 4:
            b = pl_zipf(seed, n, m, float(ss[e]), k, election=e)
            kind = "plzipf s=%.3f k=%d" % (ss[e], k)
        elif kind_id <= 8:
            b = mallows_topk(seed, n, m, float(phis[e]), k, election=e)
            kind = "mallows-topk phi=%.3f k=%d" % (phis[e], k)
        else:
            b = mallows(seed, n, m, float(phis[e]), election=e)
            kind = "mallows phi=%.3f" % phis[e]
        yield {"election": e, "m": m, "n": n, "kind": kind, "ballots": b}


def near_impartial_mixture(seed: int, count: int, m_lo: int = 256, m_hi: int = 512):
    """Elections of full Mallows rankings with phi ~ U[0.995, 1.0] (close to
    impartial culture, where a Condorcet winner is rare): m ~ U{m_lo..m_hi},
    n = round(rho m) with rho ~ U[3, 12].  Yields dicts like training_mixture."""
    ms = uniform_int(seed, 1, count, m_lo, m_hi)
    rhos = uniform_real(seed, 2, count, 3.0, 12.0)
    phis = uniform_real(seed, 5, count, 0.995, 1.0)
    for e in range(count):
        m = int(ms[e])
        n = int(round(rhos[e] * m))
        b = mallows(seed, n, m, float(phis[e]), election=e)
        yield {"election": e, "m": m, "n": n, "kind": "mallows phi=%.4f" % phis[e], "ballots": b}
