"""Value-ranked int32 closures against the oracle.

An int32 closure of m >= 1024 candidates runs on the ranks of the weight
values in packed uint16 when there are at most 65535 distinct nonzero values,
all below 2^24, and on int32 otherwise.  The widest-path recurrence of
Section 2.1 only compares values, so both give the oracle's widths exactly.
Each case checks the output against the oracle and, through
schulze_closure_value_bits, which of the two paths the device chose.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

RANKED = 16    # value width of the recurrence: ranks in packed uint16
FALLBACK = 32  # int32 values
# block sums, scan (deciding), word ranks, ranks from d, store (gated on the
# decision); the marking of the values runs with the weights
RANK_LAUNCHES = 5


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
    c.set_value_ranking(True)
    c.close()


def oriented(rng, m, values):
    """Count matrix with d[x][y] = values[k] for one orientation of each pair and 0 the other way."""
    iu, ju = np.triu_indices(m, 1)
    flip = rng.random(iu.size) < 0.5
    a, b = np.where(flip, ju, iu), np.where(flip, iu, ju)
    d = np.zeros((m, m), dtype=np.int64)
    d[a, b] = values
    return d


def run(ctx, d, mode, ranking):
    import torch
    ctx.set_value_ranking(ranking)
    ctx.set_timing(True)
    ctx.reset_timing()
    dt = torch.from_numpy(np.ascontiguousarray(d, dtype=np.int32)).cuda()
    p = ctx.closure(dt, mode)
    torch.cuda.synchronize()
    launches, _ = ctx.kernel_time("value_rank")
    ctx.set_timing(False)
    assert ctx.device_error() == 0
    return p.cpu().numpy().astype(np.int64), launches, ctx.closure_value_bits()


def check(ctx, d, mode, expect_bits, tag):
    want = oracle.closure(oracle.weights(d, oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES))
    log(f"[case] {tag} m={d.shape[0]} mode={mode} distinct={len(np.unique(d))}")
    got, launches, bits = run(ctx, d, mode, True)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{tag}: ranked closure differs at {len(bad)} places, first {bad[:5].tolist()}"
    # the ranking kernels run (and decide) from m = 1024 on; below that the int32 closure runs directly
    want_launches = RANK_LAUNCHES if d.shape[0] >= 1024 else 0
    assert launches == want_launches, f"{tag}: {launches} ranking launches, expected {want_launches}"
    assert bits == expect_bits, f"{tag}: the recurrence ran on {bits}-bit values, expected {expect_bits}"
    off, launches_off, bits_off = run(ctx, d, mode, False)
    assert launches_off == 0 and bits_off == 32
    assert np.array_equal(off, want), f"{tag}: int32 closure differs"


@pytest.mark.parametrize("m", [1024, 1100, 2048, 2100])
def test_few_values_take_ranks(ctx, m):
    rng = np.random.default_rng(70 + m)
    d = rng.integers(0, 4000, size=(m, m), dtype=np.int64)
    np.fill_diagonal(d, 0)
    check(ctx, d, "winning_votes", RANKED, "few-values")


@pytest.mark.parametrize("m", [1100, 1027])
def test_counts_with_rare_values_take_ranks(ctx, m):
    """Counts of truncated ballots: thousands of distinct weight values, many
    of them once only, in a matrix whose last block of 64 is partial (m = 1100:
    16-byte reads of d; m = 1027: one element at a time) -- every value,
    including those only in the partial blocks, must be ranked."""
    import workload
    b = workload.pl_zipf(74 + m, 3000, m, 1.0, 24)
    d = oracle.pairwise(b, m)
    check(ctx, d, "winning_votes", RANKED, "rare-values")


def test_margins_take_ranks(ctx):
    rng = np.random.default_rng(71)
    m = 1500
    d = rng.integers(0, 100000, size=(m, m), dtype=np.int64)
    d = np.minimum(d, d.T + rng.integers(0, 300, size=(m, m)))  # small margins, few distinct
    np.fill_diagonal(d, 0)
    check(ctx, d, "margin", RANKED, "margins")


def test_largest_rankable_value(ctx):
    rng = np.random.default_rng(72)
    m = 1024
    vals = rng.choice(np.array([1, 2, 1000, (1 << 24) - 2, (1 << 24) - 1], dtype=np.int64), size=m * (m - 1) // 2)
    check(ctx, oriented(rng, m, vals), "winning_votes", RANKED, "max-value")


def test_value_too_wide_falls_back(ctx):
    rng = np.random.default_rng(73)
    m = 1024
    vals = rng.integers(1, 50, size=m * (m - 1) // 2)
    vals[rng.integers(0, vals.size)] = 1 << 24
    check(ctx, oriented(rng, m, vals), "winning_votes", FALLBACK, "value-2^24")
    vals[rng.integers(0, vals.size)] = (1 << 31) - 1
    check(ctx, oriented(rng, m, vals), "winning_votes", FALLBACK, "value-int32-max")


@pytest.mark.parametrize("distinct,bits", [(65535, RANKED), (65536, FALLBACK)])
def test_distinct_value_limit(ctx, distinct, bits):
    rng = np.random.default_rng(74 + distinct)
    m = 1024
    pool = rng.choice(np.arange(1, 1 << 24, dtype=np.int64), size=distinct, replace=False)
    vals = np.concatenate([pool, rng.choice(pool, size=m * (m - 1) // 2 - distinct)])
    rng.shuffle(vals)
    check(ctx, oriented(rng, m, vals), "winning_votes", bits, f"distinct-{distinct}")


def test_many_values_fall_back(ctx):
    rng = np.random.default_rng(75)
    m = 1100
    d = rng.integers(0, 1 << 23, size=(m, m), dtype=np.int64)
    np.fill_diagonal(d, 0)
    check(ctx, d, "winning_votes", FALLBACK, "many-values")


def test_all_zero_and_one_value(ctx):
    m = 1024
    d = np.zeros((m, m), dtype=np.int64)
    check(ctx, d, "winning_votes", RANKED, "all-zero")
    rng = np.random.default_rng(76)
    check(ctx, oriented(rng, m, np.full(m * (m - 1) // 2, 12345)), "winning_votes", RANKED, "one-value")


def test_below_threshold_runs_int32(ctx):
    rng = np.random.default_rng(77)
    m = 1023
    d = rng.integers(0, 4000, size=(m, m), dtype=np.int64)
    np.fill_diagonal(d, 0)
    check(ctx, d, "winning_votes", FALLBACK, "m-1023")


@pytest.mark.parametrize("tile", [64, 128])
def test_closure_tile_sizes(ctx, tile):
    """Every tile size gives the oracle's widths, for both value widths, ranked or not."""
    import torch
    rng = np.random.default_rng(78 + tile)
    try:
        ctx.set_closure_tile(tile)
        for m in (130, 1100):
            d = rng.integers(0, 3000, size=(m, m), dtype=np.int64)
            np.fill_diagonal(d, 0)
            want = oracle.closure(oracle.weights(d, oracle.WINNING_VOTES))
            log(f"[case] tile={tile} m={m}")
            for dt in (np.uint16, np.int32):
                for ranking in (True, False):
                    ctx.set_value_ranking(ranking)
                    dd = torch.from_numpy(d.astype(dt)).cuda()
                    p = ctx.closure(dd, "winning_votes")
                    torch.cuda.synchronize()
                    assert ctx.device_error() == 0
                    got = p.cpu().numpy().astype(np.int64)
                    assert np.array_equal(got, want), f"tile={tile} m={m} dtype={dt} ranking={ranking}"
    finally:
        ctx.set_closure_tile(0)
        ctx.set_value_ranking(True)


@pytest.mark.parametrize("m", [3000, 6200])
def test_closure_grid_not_a_multiple_of_tiles(ctx, m):
    """Sizes whose count of block rows does not divide the persistent grid
    (uint16: 47 rows of 64-wide tiles over 1280 workgroups, 49 rows of
    128-wide tiles over 768; int32: 24 rows over 256), so that the owner
    map deals the tiles unevenly over block columns."""
    import torch
    rng = np.random.default_rng(m)
    d = rng.integers(0, 3000, size=(m, m), dtype=np.int64)
    np.fill_diagonal(d, 0)
    want = oracle.closure(oracle.weights(d, oracle.WINNING_VOTES))
    cases = [(np.uint16, True)] + ([(np.int32, True), (np.int32, False)] if m == 3000 else [])
    try:
        for dt, ranking in cases:
            log(f"[case] grid m={m} dtype={np.dtype(dt).name} ranking={ranking}")
            ctx.set_value_ranking(ranking)
            p = ctx.closure(torch.from_numpy(d.astype(dt)).cuda(), "winning_votes")
            torch.cuda.synchronize()
            assert ctx.device_error() == 0
            got = p.cpu().numpy().astype(np.int64)
            bad = np.argwhere(got != want)
            assert bad.size == 0, f"m={m} dtype={dt} ranking={ranking}: {len(bad)} differences, first {bad[:5].tolist()}"
    finally:
        ctx.set_value_ranking(True)
