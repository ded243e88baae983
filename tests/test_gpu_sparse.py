"""Truncated ballots over many candidates (the sparse form of the counts,
d[x][y] = R_x - C[y][x]): the bucketed count (listed entries sorted by
candidate, rows of C accumulated in LDS) and the atomic pair scattering give
the oracle's d exactly; rows whose occurrences span several accumulation
chunks, both LDS row sizes (m up to 16384 and up to 32768), voter weights
(including zero) and repeated ids are covered."""
import numpy as np
import pytest

import oracle
import workload
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.set_sparse_count("bucketed")
    c.close()


def gpu_counts(ctx, b, m, mode, weight=None):
    import torch
    ctx.set_sparse_count(mode)
    wt = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight, dtype=np.uint32)).cuda()
    d = ctx.pairwise(torch.from_numpy(np.ascontiguousarray(b)).cuda(), m, voter_weight=wt, dtype="i32")
    torch.cuda.synchronize()
    err = ctx.device_error()
    return d, err


@pytest.mark.parametrize("m,n,k,s", [(600, 5000, 12, 1.5), (2500, 3000, 5, 1.0), (1500, 4001, 3, 1.1),
                                     (4000, 20000, 8, 1.3)])
def test_sparse_counts_match_oracle(ctx, m, n, k, s):
    b = workload.pl_zipf(700 + m, n, m, s, k)
    want = oracle.pairwise(b, m)
    for mode in ("bucketed", "atomic"):
        log(f"[case] sparse m={m} n={n} k={k} s={s} {mode}")
        d, err = gpu_counts(ctx, b, m, mode)
        assert err == 0
        got = d.cpu().numpy().astype(np.int64)
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"{mode}: d differs at {len(bad)} places, first {bad[:5].tolist()}"


def test_sparse_hot_rows_span_chunks(ctx):
    """Zipf(2.0): the favourite is listed by almost every ballot, so its
    row collects far more than one chunk of occurrences."""
    m, n, k = 500, 30000, 10
    b = workload.pl_zipf(711, n, m, 2.0, k)
    listed = np.array([(row[1:] != 0xFFFF).sum() for row in b[:2000]])
    assert listed.mean() > 5
    want = oracle.pairwise(b, m)
    d, err = gpu_counts(ctx, b, m, "bucketed")
    assert err == 0 and (d.cpu().numpy().astype(np.int64) == want).all()


def test_sparse_voter_weights(ctx):
    rng = np.random.default_rng(713)
    m, n = 900, 2500
    b = workload.pl_zipf(713, n, m, 1.0, 6)
    w = rng.integers(0, 7, size=n).astype(np.uint32)  # zeros included
    want = oracle.pairwise(b, m, w)
    for mode in ("bucketed", "atomic"):
        d, err = gpu_counts(ctx, b, m, mode, weight=w)
        assert err == 0
        assert (d.cpu().numpy().astype(np.int64) == want).all(), mode


@pytest.mark.parametrize("m", [16384, 16385, 20000])
def test_sparse_large_m_sampled(ctx, m):
    """Both LDS row sizes; sampled rows and columns against the oracle and the
    whole matrix against the atomic route."""
    import torch
    b = workload.pl_zipf(717 + m, 4000, m, 1.0, 12)
    d1, err1 = gpu_counts(ctx, b, m, "bucketed")
    d2, err2 = gpu_counts(ctx, b, m, "atomic")
    assert err1 == 0 and err2 == 0
    assert torch.equal(d1, d2)
    rows = np.array([0, 1, m // 2, m - 1], dtype=np.int32)
    got = d1.cpu().numpy()
    assert (got[rows] == oracle.pairwise_rows(b, m, rows)).all()
    assert (got[:, rows].T == oracle.pairwise_cols(b, m, rows)).all()


def test_sparse_repeated_id_is_reported(ctx):
    import paper_2505_12976_amd as sz
    b = workload.pl_zipf(719, 3000, 2000, 1.0, 6).copy()
    b[17, 3] = b[17, 1]
    for mode in ("bucketed", "atomic"):
        d, err = gpu_counts(ctx, b, 2000, mode)
        assert err == sz.EBALLOT, mode


@pytest.mark.parametrize("case", ["odd-L", "int32-ids", "words", "pieces-L-10", "L-48", "L-80", "full-mixed",
                                  "weights-full-mixed"])
def test_sparse_row_layouts(ctx, case):
    """Ballot layouts of the bucketed count: rows read as 16-byte pieces
    (uint16 ids, even L up to 64, n L a multiple of 8; the last ballot ends
    the buffer), as 32-bit words (even L, n L not a multiple of 8), one id at
    a time (odd L, int32 ids), rows longer than a wavefront, and full
    rankings counted densely next to the bucketed truncated ballots (counts
    added to the dense part)."""
    rng = np.random.default_rng(731)
    weight = None
    if case == "words":
        m, b = 3000, workload.pl_zipf(737, 6001, 3000, 1.0, 12)
        assert (b.size % 8) != 0 and b.shape[1] % 2 == 0
    elif case == "pieces-L-10":
        m, b = 3000, workload.pl_zipf(738, 6004, 3000, 1.1, 10)
        assert b.size % 8 == 0
        b[-1, :] = np.arange(10, dtype=b.dtype)  # the last ballot lists ten ids
    elif case == "odd-L":
        m, b = 3000, workload.pl_zipf(731, 6000, 3000, 1.0, 7)
    elif case == "int32-ids":
        m, b = 3000, workload.pl_zipf(732, 6000, 3000, 1.0, 8, dtype=np.int32)
    elif case == "L-48":
        m, b = 4000, workload.pl_zipf(733, 3000, 4000, 1.0, 40, L=48)
    elif case == "L-80":
        m, b = 5000, workload.pl_zipf(734, 3000, 5000, 1.2, 70, L=80)
    else:
        m = 3000
        trunc = workload.pl_zipf(735, 5000, m, 1.0, 6, L=m)
        full = workload.mallows(736, 21, m, 0.9)
        b = np.concatenate([trunc, full])
        b = b[rng.permutation(len(b))]
        if case == "weights-full-mixed":
            weight = rng.integers(0, 5, size=len(b)).astype(np.uint32)
    want = oracle.pairwise(b, m, weight)
    log(f"[case] sparse layout {case}: m={m} n={len(b)} L={b.shape[1]}")
    d, err = gpu_counts(ctx, b, m, "bucketed", weight=weight)
    assert err == 0
    got = d.cpu().numpy().astype(np.int64)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{case}: d differs at {len(bad)} places, first {bad[:5].tolist()}"
