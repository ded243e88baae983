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


def test_features_brute_force():
    for seed, m in ((1, 7), (2, 12), (3, 1), (4, 30)):
        b = workload.uniform_ballots(seed, 25, m, min_len=1, dtype=np.int32)
        d = oracle.pairwise(b, m)
        for mode in (oracle.WINNING_VOTES, oracle.MARGIN):
            F = oracle.features(d, 25.0, mode)
            w = oracle.weights(d, mode)
            for x in range(m):
                others = [y for y in range(m) if y != x]
                assert F[x, 0] == np.float32(sum(d[x, y] > d[y, x] for y in others) / max(m - 1, 1))
                assert F[x, 5] == float(max([w[y, x] for y in others], default=0) >
                                        max([w[x, y] for y in others], default=0))
                assert np.isclose(F[x, 2], sum(d[x, y] for y in others) / max(m - 1, 1) / 25.0)
                assert np.isclose(F[x, 6], sum(w[x, y] for y in others) / max(m - 1, 1) / 25.0)
            # the filter flag never marks a winner (Section 4)
            _, win, _ = oracle.rank(oracle.closure(w))
            assert not (win & (F[:, 5] == 1)).any()
