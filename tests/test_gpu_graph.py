"""Calls captured in a HIP graph and replayed: the int32 closure (both the
value-ranked and the plain int32 variant, decided on the device) and the
proposer's train step.  Every replay is checked against the oracle or the
eager result, with eager work and synchronisations between replays."""
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
    c.close()


def _counts(kind, m):
    """int32 counts whose weights the closure ranks ("ranked": a few
    thousand distinct values) or cannot rank ("wide": values of 2^25 and
    more, so the int32 recurrence runs)."""
    if kind == "ranked":
        b = workload.pl_zipf(71, 3000, m, 1.0, 24)
        return oracle.pairwise(b, m).astype(np.int32)
    rng = np.random.default_rng(72)
    d = rng.integers(1 << 25, 1 << 26, size=(m, m), dtype=np.int64)
    np.fill_diagonal(d, 0)
    return d.astype(np.int32)


@pytest.mark.parametrize("kind,m", [("ranked", 1100), ("wide", 1100), ("ranked", 2200)])
def test_closure_captured_in_graph(ctx, kind, m):
    import torch
    d_np = _counts(kind, m)
    want = oracle.closure(oracle.weights(d_np.astype(np.int64), oracle.WINNING_VOTES))
    dev = torch.device("cuda", 0)
    d = torch.from_numpy(d_np).to(dev)
    p = torch.empty_like(d)
    log(f"[case] graph closure {kind} m={m}: eager call")
    ctx.closure(d, out=p)  # sizes the workspace
    torch.cuda.synchronize()
    assert ctx.device_error() == 0
    assert (p.cpu().numpy().astype(np.int64) == want).all()
    assert ctx.closure_value_bits() == (16 if kind == "ranked" else 32)
    g = torch.cuda.CUDAGraph()
    log(f"[case] graph closure {kind} m={m}: capture")
    with torch.cuda.graph(g):
        ctx.closure(d, out=p)
    for rep in range(3):
        p.fill_(-1)
        other = torch.empty_like(d)
        ctx.closure(d, out=other)  # eager work on the same workspace between replays
        torch.cuda.synchronize()
        log(f"[case] graph closure {kind} m={m}: replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert ctx.device_error() == 0
        got = p.cpu().numpy().astype(np.int64)
        assert (got == want).all(), f"replay {rep}: {(got != want).sum()} entries differ"
        assert (other.cpu().numpy().astype(np.int64) == want).all()
    del g


def test_train_step_captured_in_graph(ctx):
    import torch
    from paper_2505_12976_amd.proposer import init_params
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(81)
    sizes = [37, 300, 5, 128, 900]
    M = sum(sizes)
    feat = torch.from_numpy(rng.standard_normal((M, 16)).astype(np.float32)).to(dev)
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)).to(dev)
    win_np = np.zeros(M, dtype=np.uint8)
    o = 0
    for s in sizes:
        win_np[o + rng.integers(0, s)] = 1
        o += s
    win = torch.from_numpy(win_np).to(dev)
    p0 = torch.from_numpy(init_params(11)).to(dev)

    def state():
        return {"params": p0.clone(), "m1": torch.zeros_like(p0), "m2": torch.zeros_like(p0),
                "grad": torch.zeros_like(p0), "step": torch.zeros(1, dtype=torch.int32, device=dev),
                "loss": torch.zeros(len(sizes), dtype=torch.float32, device=dev)}

    def step(st):
        ctx.mlp_train_step(st["params"], st["m1"], st["m2"], st["grad"], st["step"], feat, off, win, lr=3e-3,
                           loss=st["loss"])

    # eager reference: the separate calls, one Adam step at a time
    ref = state()
    for t in range(1, 5):
        score = ctx.mlp_forward(ref["params"], feat)
        ds, loss = ctx.mlp_loss(score, off, win)
        ctx.mlp_backward(ref["params"], feat, ds, out=ref["grad"])
        ctx.mlp_adam(ref["params"], ref["grad"], ref["m1"], ref["m2"], 3e-3, t)
        ref.setdefault("losses", []).append(loss.clone())
    eager = state()
    for _ in range(4):
        step(eager)
    torch.cuda.synchronize()
    for k in ("params", "m1", "m2", "grad"):
        assert torch.equal(eager[k], ref[k]), k
    assert int(eager["step"].item()) == 4
    # one step captured, replayed four times
    gst = state()
    step(gst)  # eager first step sizes the workspace
    torch.cuda.synchronize()
    assert torch.equal(gst["loss"], ref["losses"][0])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(gst)
    for t in range(2, 5):
        junk = ctx.mlp_forward(p0, feat)  # eager work between replays
        torch.cuda.synchronize()
        log(f"[case] graph train step replay {t}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(gst["loss"], ref["losses"][t - 1]), t
        assert int(gst["step"].item()) == t
        del junk
    for k in ("params", "m1", "m2", "grad"):
        assert torch.equal(gst[k], ref[k]), k
    del g
