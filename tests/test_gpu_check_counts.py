"""The exact winner check straight from the pairwise counts
(schulze_verify_counts: weights formed inside the sweeps, row-and-column
gathers for small frontiers, a dense pass over the tile pairs of d for large
ones) against the oracle's widest paths, bit-exact, for every candidate of
small profiles, both count widths and both weight rules, strided counts, tie-
heavy profiles and count matrices built so that widest paths are long (many
sweeps with small frontiers)."""
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


def chain_counts(m, seed):
    """Counts whose widest paths run along a hidden Hamiltonian chain: the
    chain's pairs have wide margins, every other pair a narrow one, so the
    widest path between far-apart chain vertices has many edges."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m)
    d = rng.integers(40, 60, size=(m, m))
    d = np.triu(d, 1)
    d = d + (100 - d.T) * np.tri(m, m, -1, dtype=np.int64)  # d[i][j] + d[j][i] = 100 off the diagonal
    np.fill_diagonal(d, 0)
    for k in range(m - 1):
        a, b = perm[k], perm[k + 1]
        d[a, b], d[b, a] = 100 - k % 7, k % 7
    return np.ascontiguousarray(d)


def check(ctx, dn, mode, dtype, cands, pitch=0, tag=""):
    import torch
    m = dn.shape[0]
    wn = oracle.weights(dn, oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES)
    pn = oracle.closure(wn)
    beaten, win, _ = oracle.rank(pn)
    npdt = np.uint16 if dtype == "u16" else np.int32
    big = np.zeros((m, m + pitch), dtype=npdt)
    big[:, :m] = dn.astype(npdt)
    d = torch.from_numpy(big).cuda()[:, :m]
    for c in cands:
        log(f"[case] check-counts {tag} m={m} {dtype} {mode} pitch+{pitch} cand={c}")
        verdict, p_from, p_to, tied = ctx.verify_counts(d, int(c), mode, want_tied=True)
        v = verdict.cpu().numpy()
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        assert (to_np(p_from) == np.where(np.arange(m) == c, 0, pn[c])).all(), (tag, c, "p(c, .)")
        assert (to_np(p_to) == np.where(np.arange(m) == c, 0, pn[:, c])).all(), (tag, c, "p(., c)")
        assert v[0] == int(win[c]) and v[1] == beaten[c], (tag, c, v)
        ties = [x for x in range(m) if x != c and pn[c, x] == pn[x, c]]
        assert v[3] == len(ties)
        assert sorted(tied.cpu().numpy()[:v[3]].tolist()) == ties
        if v[1]:
            x = v[2]
            margins = [pn[y, c] - pn[c, y] for y in range(m) if pn[y, c] > pn[c, y]]
            assert pn[x, c] - pn[c, x] == max(margins)
        else:
            assert v[2] == -1


def sample(m, seed, k=6):
    if m <= 65:
        return range(m)
    return sorted(set([0, m - 1] + list(np.random.default_rng(seed).integers(0, m, size=k))))


@pytest.mark.parametrize("m", [1, 2, 3, 17, 40, 63, 64, 65, 129, 500, 1000])
@pytest.mark.parametrize("dtype,mode", [("u16", "winning_votes"), ("i32", "winning_votes"), ("u16", "margin"),
                                        ("i32", "margin")])
def test_check_counts_profiles(ctx, m, dtype, mode):
    dn = oracle.pairwise(profile(m, 200 + m), m)
    wn = oracle.weights(dn, oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES)
    win = oracle.rank(oracle.closure(wn))[1]
    cands = sorted(set(sample(m, m)) | set(np.nonzero(win)[0].tolist()))
    check(ctx, dn, mode, dtype, cands, tag="profile")


@pytest.mark.parametrize("m,pitch", [(100, 7), (257, 3), (640, 1)])
def test_check_counts_strided(ctx, m, pitch):
    """Row pitch not a multiple of the vector length: element-wise tiles."""
    dn = oracle.pairwise(profile(m, 300 + m), m)
    check(ctx, dn, "winning_votes", "i32", sample(m, 3 * m), pitch=pitch, tag="strided")
    check(ctx, dn, "margin", "u16", sample(m, 5 * m), pitch=pitch, tag="strided")


@pytest.mark.parametrize("m", [30, 200, 700])
def test_check_counts_long_paths(ctx, m):
    """Widest paths of up to m - 1 edges: sweeps with frontiers of a few
    vertices, one after another (gathers), after dense passes."""
    dn = chain_counts(m, m)
    check(ctx, dn, "winning_votes", "i32", sample(m, m, k=4), tag="chain")
    check(ctx, dn, "margin", "u16", sample(m, 2 * m, k=4), tag="chain")


def test_check_counts_ties(ctx):
    """Few voters, many equal counts: tied candidates listed exactly."""
    for seed, m in ((1, 50), (2, 90)):
        b = workload.uniform_ballots(seed, 6, m, min_len=0)
        dn = oracle.pairwise(b, m)
        check(ctx, dn, "winning_votes", "i32", range(0, m, 3), tag="ties")


def test_check_counts_mid_workload(ctx):
    """m=4096: the stored oracle winner passes and sampled losers are beaten
    by exactly as many candidates as stored; the same rows as schulze_verify
    on the weights."""
    import torch
    wl = workload.plain_mid()
    path = os.path.join(GOLD, wl.name + ".json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle results")
    gold = json.load(open(path))
    d = ctx.pairwise(torch.from_numpy(wl.ballots).cuda(), wl.m, dtype="u16")
    w, wt = ctx.weights(d)
    for c in (gold["winners"][0], gold["order"][1], gold["order"][-1], 1234):
        log(f"[case] check-counts m=4096 cand={c}")
        verdict, p_from, p_to, _ = ctx.verify_counts(d, int(c))
        v = verdict.cpu().numpy()
        assert v[1] == gold["beaten_by"][c]
        assert v[0] == int(c in gold["winners"])
        v2, f2, t2, _ = ctx.verify(w, wt, int(c))
        assert torch.equal(p_from, f2) and torch.equal(p_to, t2) and torch.equal(verdict, v2)


def test_check_counts_rejects_bad_arguments(ctx):
    import torch
    import paper_2505_12976_amd as sz
    d = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    lib, h = ctx._lib, ctx._h
    out = torch.zeros(8, dtype=torch.int32, device="cuda")
    p = out.data_ptr()
    assert lib.schulze_verify_counts(h, None, d.data_ptr(), 4, 4, sz.I32, 0, 4, None, p, p, p, None) == sz.EINVAL
    assert lib.schulze_verify_counts(h, None, d.data_ptr(), 4, 4, sz.I32, 5, 0, None, p, p, p, None) == sz.EINVAL
    assert lib.schulze_verify_counts(h, None, d.data_ptr(), 3, 4, sz.I32, 0, 0, None, p, p, p, None) == sz.EINVAL
    assert lib.schulze_verify_counts(h, None, d.data_ptr(), 4, 4, sz.I32, 0, 0, None, None, p, p, None) == sz.EINVAL


def test_check_counts_stopped_sweeps(ctx):
    """A run capped below the sweeps it needs, and a grid barrier allowed a
    single poll, stop every workgroup and set the device error word; with
    the defaults restored the same call gives the oracle's rows."""
    import torch
    import paper_2505_12976_amd as sz
    m = 300
    dn = chain_counts(m, 77)
    pn = oracle.closure(oracle.weights(dn, oracle.WINNING_VOTES))
    d = torch.from_numpy(dn.astype(np.int32)).cuda()
    try:
        for spin, cap in ((0, 3), (1, 0)):
            log(f"[case] check-counts m={m} limits spin={spin} sweeps={cap}")
            ctx.set_sweep_limits(spin, cap)
            ctx.verify_counts(d, 5)
            torch.cuda.synchronize()
            assert ctx.device_error() == sz.EDEVICE
    finally:
        ctx.set_sweep_limits(0, 0)
    log(f"[case] check-counts m={m} default limits")
    _, p_from, p_to, _ = ctx.verify_counts(d, 5)
    assert ctx.device_error() == 0
    assert (to_np(p_from) == np.where(np.arange(m) == 5, 0, pn[5])).all()
    assert (to_np(p_to) == np.where(np.arange(m) == 5, 0, pn[:, 5])).all()
