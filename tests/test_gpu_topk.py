"""Top-k by iterated winner removal (the closing remark of Section 4) on the
GPU: each level is the Schulze winner set of the candidates left, found by
the label-propagation algorithm with the removed candidates' edges deleted.
Levels must equal the oracle's exactly, for random profiles of many kinds,
both weight modes, both counter widths, both label orders, every k, tie-heavy
count matrices, the pinned small graphs, and larger sizes."""
import numpy as np
import pytest

import oracle
from tests.test_gpu_parity import log
from tests.test_gpu_propagate import MODES, profiles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def check(ctx, d_np, dtype, mode, k, borda, tag):
    import torch
    want = oracle.topk_levels(oracle.weights(d_np.astype(np.int64), MODES[mode]), k)
    tdt = torch.uint16 if dtype == "u16" else torch.int32
    d = torch.from_numpy(d_np.astype(np.uint16 if dtype == "u16" else np.int32)).cuda()
    assert d.dtype == tdt
    level, st = ctx.topk_propagate(d, k, mode, borda_order=borda)
    got = level.cpu().numpy()
    assert (got == want).all(), (tag, k, borda, st, got.tolist(), want.tolist())
    assert st["levels"] == int(want.max()) + 1
    assert st["ranked"] == int((want >= 0).sum())
    return st


@pytest.mark.parametrize("dtype", ["u16", "i32"])
@pytest.mark.parametrize("mode", ["winning_votes", "margin"])
def test_topk_random_profiles(ctx, dtype, mode):
    import torch
    rng = np.random.default_rng(5001 + (dtype == "i32"))
    levels = []
    for i, b, m in profiles(5003 + (mode == "margin"), 80):
        d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype="i32").cpu().numpy()
        k = int(rng.integers(1, m + 1))
        for borda in (True, False):
            st = check(ctx, d, dtype, mode, k, borda, f"profile {i} m={m}")
            levels.append(st["levels"])
        check(ctx, d, dtype, mode, m, True, f"profile {i} m={m} all")
    assert ctx.device_error() == 0
    log(f"[case] topk {dtype} {mode}: levels max {max(levels)} mean {np.mean(levels):.2f}")


def test_topk_random_count_matrices(ctx):
    """Tie-heavy count matrices: many tied candidates per level."""
    rng = np.random.default_rng(5007)
    for i in range(100):
        m = int(rng.integers(2, 30))
        d = rng.integers(0, 4, size=(m, m)).astype(np.int64)
        np.fill_diagonal(d, 0)
        check(ctx, d, "i32", "winning_votes", int(rng.integers(1, m + 1)), i % 2 == 0, f"matrix {i}")
    assert ctx.device_error() == 0


def test_topk_pinned_graphs(ctx):
    """The graph where removal deletes a deciding path (levels 1, 2, 2, 0)
    and the Figure 1 graph (levels a 0, b 2, c 3, d 1), given as margins."""
    w = np.zeros((4, 4), dtype=np.int64)
    w[0, 1], w[0, 2], w[2, 3], w[3, 0] = 5, 3, 1, 3
    for k in (1, 2, 3, 4):
        check(ctx, w, "i32", "margin", k, True, "removal")
        check(ctx, w, "u16", "margin", k, False, "removal")
    a, b, c, dd = range(4)
    f = np.zeros((4, 4), dtype=np.int64)
    for x, y, mu in ((a, b, 4), (a, c, 6), (b, c, 10), (c, dd, 8), (dd, a, 2), (dd, b, 12)):
        f[x, y] = mu
    import torch
    level, st = ctx.topk_propagate(torch.from_numpy(f.astype(np.int32)).cuda(), 4, "margin")
    assert level.cpu().numpy().tolist() == [0, 2, 3, 1]


def test_topk_one_candidate_and_full_ranking(ctx):
    import torch
    check(ctx, np.zeros((1, 1), dtype=np.int64), "i32", "winning_votes", 1, True, "m=1")
    rng = np.random.default_rng(5011)
    for m in (2, 33, 300):
        order = rng.permutation(m).astype(np.int32)
        d = ctx.pairwise(torch.from_numpy(order[None, :]).cuda(), m, dtype="i32").cpu().numpy()
        st = check(ctx, d, "i32", "winning_votes", m, True, f"single ranking m={m}")
        assert st["levels"] == m


@pytest.mark.parametrize("m,n", [(257, 300), (700, 120), (1200, 2000)])
def test_topk_sizes(ctx, m, n):
    """Several sweep blocks and ragged tails; k = 10, and every level at the
    smallest size (the oracle recloses the remaining subgraph per level)."""
    import torch
    import workload
    b = workload.pl_zipf(5013 + m, n, m, 1.0, 12, L=12)
    d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype="i32").cpu().numpy()
    for k in ((10, m) if m < 300 else (10,)):
        st = check(ctx, d, "i32", "winning_votes", k, True, f"m={m} n={n}")
        log(f"[case] topk m={m} n={n} k={k}: {st}")


def test_topk_rejects_bad_k(ctx):
    import torch
    import paper_2505_12976_amd as sz
    d = torch.zeros((4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(sz.SchulzeError):
        ctx.topk_propagate(d, 0)
