"""Features, the proposer network's forward/backward kernels, the segmented
loss and Adam, against the CPU reference (oracle/mlp.py, same BF16 rounding
points; FP32 accumulation order differs, so the bar is a relative L2 error
per tensor)."""
import numpy as np
import pytest

import oracle
from oracle import mlp
import workload
from tests.test_gpu_parity import log

pytestmark = pytest.mark.gpu

TENSORS = {
    "W1": (mlp.OFF_W1, mlp.OFF_B1), "b1": (mlp.OFF_B1, mlp.OFF_W2), "W2": (mlp.OFF_W2, mlp.OFF_B2),
    "b2": (mlp.OFF_B2, mlp.OFF_W3), "W3": (mlp.OFF_W3, mlp.OFF_B3), "b3": (mlp.OFF_B3, mlp.NPARAM),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_12976_amd as sz
    assert torch.cuda.is_available()
    c = sz.Context(0)
    yield c
    c.close()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def cuda(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).cuda()


@pytest.mark.parametrize("m,dtype,mode", [(1, "i32", "winning_votes"), (5, "u16", "margin"), (64, "i32", "margin"),
                                          (300, "u16", "winning_votes"), (1000, "i32", "winning_votes"),
                                          (5000, "i32", "margin"), (9000, "u16", "winning_votes")])
def test_features(ctx, m, dtype, mode):
    import torch
    b = workload.pl_zipf(m, 400, m, 1.0, min(m, 15))
    dn = oracle.pairwise(b, m)
    md = oracle.MARGIN if mode == "margin" else oracle.WINNING_VOTES
    want = oracle.features(dn, 400.0, md)
    d = cuda(dn, np.uint16 if dtype == "u16" else np.int32)
    got = ctx.features(d, 400.0, mode).cpu().numpy()
    torch.cuda.synchronize()
    assert np.allclose(got, want, rtol=1e-5, atol=1e-6), np.abs(got - want).max(axis=0)
    assert (got[:, 5] == want[:, 5]).all()


def problem(M, E, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, mlp.NF)).astype(np.float32)
    X[:, 15] = 1.0
    cuts = np.sort(rng.choice(np.arange(1, M), E - 1, replace=False)) if E > 1 else np.array([], dtype=np.int64)
    off = np.concatenate([[0], cuts, [M]]).astype(np.int64)
    win = np.zeros(M, dtype=np.uint8)
    for e in range(E):
        win[rng.integers(off[e], off[e + 1])] = 1
    return X, off, win


@pytest.mark.parametrize("M,E", [(1, 1), (63, 2), (64, 3), (1000, 17), (20000, 40)])
def test_forward_loss_backward(ctx, M, E):
    import torch
    X, off, win = problem(M, E, M)
    p = mlp.init_params(M)
    log(f"[case] mlp M={M} E={E}")
    pt, Xt = cuda(p), cuda(X)
    s = ctx.mlp_forward(pt, Xt)
    ds, loss = ctx.mlp_loss(s, cuda(off), cuda(win))
    g = ctx.mlp_backward(pt, Xt, ds)
    torch.cuda.synchronize()
    s_g, ds_g, loss_g, g_g = s.cpu().numpy(), ds.cpu().numpy(), loss.cpu().numpy(), g.cpu().numpy()

    f = mlp.forward(p, X)
    assert rel_l2(s_g, f["s"]) < 1e-2
    # loss and its gradient from the GPU scores (isolates the loss kernel)
    lw, dsw = mlp.seg_loss(s_g, off, win)
    assert abs(loss_g.mean() - lw) <= 1e-5 * max(1.0, abs(lw))
    assert np.allclose(ds_g, dsw, rtol=1e-4, atol=1e-7)
    # gradients from the GPU's dscore (isolates the backward kernel)
    gw = mlp.backward(p, X, ds_g)
    full = np.linalg.norm(gw)
    if full == 0:  # e.g. one candidate that wins: no gradient at all
        assert not np.abs(g_g).any()
        return
    for name, (a, b) in TENSORS.items():
        # a tensor whose gradient cancels (b3: softmax gradients sum to zero per
        # election) is measured against the whole gradient's scale
        denom = max(np.linalg.norm(gw[a:b]), 1e-3 * full)
        err = np.linalg.norm(g_g[a:b].astype(np.float64) - gw[a:b]) / denom
        assert err < 1e-2, (name, err)


def test_backward_is_deterministic(ctx):
    import torch
    X, off, win = problem(5000, 9, 11)
    pt, Xt = cuda(mlp.init_params(1)), cuda(X)
    s = ctx.mlp_forward(pt, Xt)
    ds, _ = ctx.mlp_loss(s, cuda(off), cuda(win))
    g1 = ctx.mlp_backward(pt, Xt, ds).cpu().numpy()
    g2 = ctx.mlp_backward(pt, Xt, ds).cpu().numpy()
    torch.cuda.synchronize()
    assert (g1.view(np.uint32) == g2.view(np.uint32)).all()


def test_adam_step(ctx):
    import torch
    rng = np.random.default_rng(0)
    p = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    g = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    m1 = rng.standard_normal(mlp.NPARAM).astype(np.float32) * 0.1
    m2 = np.abs(rng.standard_normal(mlp.NPARAM)).astype(np.float32) * 0.1
    pt, m1t, m2t = cuda(p), cuda(m1), cuda(m2)
    ctx.mlp_adam(pt, cuda(g), m1t, m2t, lr=1e-3, step=3)
    torch.cuda.synchronize()
    b1, b2, eps, t = 0.9, 0.999, 1e-8, 3
    a = b1 * m1.astype(np.float64) + (1 - b1) * g
    v = b2 * m2.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    want = p - 1e-3 * (a / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    assert np.allclose(pt.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
    assert np.allclose(m1t.cpu().numpy(), a, rtol=1e-5, atol=1e-7)
