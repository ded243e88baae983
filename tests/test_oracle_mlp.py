"""Pins for the CPU reference of the learned proposer and of the features."""
import numpy as np
import pytest

import oracle
from oracle import mlp
import workload
from tests import brute


def small_problem(seed=0, M=40, E=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, mlp.NF))
    cuts = np.sort(rng.choice(np.arange(1, M), E - 1, replace=False))
    off = np.concatenate([[0], cuts, [M]]).astype(np.int64)
    win = np.zeros(M, dtype=np.uint8)
    for e in range(E):
        a, b = off[e], off[e + 1]
        win[rng.integers(a, b)] = 1
        if b - a > 2 and e == 0:
            win[a] = 1  # a tied winner pair
    return X, off, win


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert (mlp.bf16(x) == want).all()


def test_backward_matches_finite_differences():
    X, off, win = small_problem()
    p = mlp.init_params(3).astype(np.float64)
    f = mlp.forward(p, X, rounding=False, dtype=np.float64)
    _, ds = mlp.seg_loss(f["s"], off, win, dtype=np.float64)
    g = mlp.backward(p, X, ds, rounding=False, dtype=np.float64)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 300, replace=False),
                          [mlp.OFF_B1, mlp.OFF_B2, mlp.OFF_W3, mlp.OFF_B3]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_value(pp, X, off, win) - mlp.loss_value(pm, X, off, win)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 + 1e-5 * abs(fd), (k, fd, g[k])


def test_seg_loss_direct_formula():
    from scipy.special import logsumexp
    rng = np.random.default_rng(2)
    s = rng.standard_normal(30)
    off = np.array([0, 10, 11, 30])
    win = np.zeros(30, dtype=np.uint8)
    win[[3, 10, 12, 29]] = 1
    loss, ds = mlp.seg_loss(s, off, win, dtype=np.float64)
    want = np.mean([logsumexp(s[a:b]) - logsumexp(s[a:b][win[a:b] == 1])
                    for a, b in zip(off[:-1], off[1:])])
    assert abs(loss - want) < 1e-12
    h = 1e-6
    for k in range(30):
        sp, sm = s.copy(), s.copy()
        sp[k] += h
        sm[k] -= h
        fd = (mlp.seg_loss(sp, off, win, np.float64)[0] - mlp.seg_loss(sm, off, win, np.float64)[0]) / (2 * h)
        assert abs(fd - ds[k]) < 1e-7


def test_rounded_forward_close_to_exact():
    X, off, win = small_problem(5, M=200)
    p = mlp.init_params(7)
    a = mlp.forward(p, X, rounding=True)["s"]
    b = mlp.forward(p, X, rounding=False, dtype=np.float64)["s"]
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-2


FEATURE_CASES = [(1, 7, 25, 1), (2, 12, 25, 1), (3, 1, 25, 1), (4, 30, 25, 1), (5, 2, 4, 0), (6, 9, 10, 0),
                 (7, 16, 6, 3), (8, 5, 40, 5)]


def _feature_profile(seed, m, n, min_len):
    return workload.uniform_ballots(seed, n, m, min_len=min(min_len, m), dtype=np.int32)


def test_features_brute_force():
    """Every one of the 16 columns against pair-list brute force, both weight
    modes, on profiles with ties, truncation, m = 1 and m = 2."""
    seen_ties = seen_neg = seen_filter = False
    for seed, m, n, min_len in FEATURE_CASES:
        b = _feature_profile(seed, m, n, min_len)
        d = oracle.pairwise(b, m)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            F = oracle.features(d, float(n), mode)
            want = brute.features(b, m, float(n), mode)
            assert F.dtype == np.float32 and F.shape == (m, 16)
            np.testing.assert_allclose(F, want.astype(np.float32), rtol=2e-7, atol=1e-9,
                                       err_msg=f"seed={seed} m={m} mode={mode}")
            seen_ties |= bool((want[:, 1] > 0).any())
            seen_neg |= bool((want[:, 8] < 0).any())
            seen_filter |= bool((want[:, 5] == 1).any())
            # the filter flag never marks a winner (Section 4)
            w = oracle.weights(d, mode)
            _, win, _ = oracle.rank(oracle.closure(w))
            assert not (win & (F[:, 5] == 1)).any()
    assert seen_ties and seen_neg and seen_filter


def _features_margin_over_w(d, n, mode):
    """Planted: smallest/largest margin taken over the edge weights."""
    F = oracle.features(d, n, mode).astype(np.float64)
    w = oracle.weights(d, mode)
    m = d.shape[0]
    off = ~np.eye(m, dtype=bool)
    F[:, 8] = np.where(off, w, np.iinfo(np.int64).max).min(axis=1) / n
    F[:, 9] = np.where(off, w, -1).max(axis=1) / n
    return F


def _features_in_out_swapped(d, n, mode):
    """Planted: largest in- and out-weight exchanged (columns 3 and 4)."""
    F = oracle.features(d, n, mode).astype(np.float64)
    F[:, [3, 4]] = F[:, [4, 3]]
    return F


def _features_diagonal_counted(d, n, mode):
    """Planted: ties counted with the diagonal (x against itself)."""
    F = oracle.features(d, n, mode).astype(np.float64)
    m = d.shape[0]
    F[:, 1] = (((d == d.T)).sum(axis=1)) / max(m - 1, 1)
    return F


def _features_mean_over_m(d, n, mode):
    """Planted: mean in-weight divided by m instead of m - 1."""
    F = oracle.features(d, n, mode).astype(np.float64)
    w = oracle.weights(d, mode)
    F[:, 7] = w.sum(axis=0) / d.shape[0] / n
    return F


def _features_margin_transposed(d, n, mode):
    """Planted: margins read as d[y][x] - d[x][y]."""
    F = oracle.features(d, n, mode).astype(np.float64)
    m = d.shape[0]
    off = ~np.eye(m, dtype=bool)
    mg = d.T - d
    F[:, 8] = np.where(off, mg, np.iinfo(np.int64).max).min(axis=1) / n
    F[:, 9] = np.where(off, mg, np.iinfo(np.int64).min).max(axis=1) / n
    return F


def _features_ratio_of_sum(d, n, mode):
    """Planted: normalised out-weight over the column's sum instead of its maximum."""
    F = oracle.features(d, n, mode).astype(np.float64)
    F[:, 13] = F[:, 3] / F[:, 3].sum() if F[:, 3].sum() > 0 else 0.0
    return F


@pytest.mark.parametrize("bad", [_features_margin_over_w, _features_in_out_swapped, _features_diagonal_counted,
                                 _features_mean_over_m, _features_margin_transposed, _features_ratio_of_sum])
def test_feature_pins_catch_planted_mistakes(bad):
    caught = False
    for seed, m, n, min_len in FEATURE_CASES:
        if m < 3:
            continue
        b = _feature_profile(seed, m, n, min_len)
        d = oracle.pairwise(b, m)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            want = brute.features(b, m, float(n), mode)
            got = bad(d, float(n), mode)
            caught |= not np.allclose(got, want, rtol=2e-7, atol=1e-9)
    assert caught
