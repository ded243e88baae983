"""Failure paths of the frontier sweeps, forced from the host with
schulze_set_sweep_limits so that every kernel still ends normally: a run
capped below the sweeps it needs, and a grid barrier allowed a single poll,
stop every workgroup of the launch and report SCHULZE_EDEVICE; the learned
and label-propagation winners then return SCHULZE_EDEVICE instead of a
winner set.  With the defaults restored the same calls give the oracle's
results."""
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
    c.set_sweep_limits(0, 0)
    c.close()


def chain(m, seed):
    """Weights whose widest paths from 0 run along the chain 0 -> 1 -> ... ->
    m-1 (one more vertex per sweep), over small random weights elsewhere."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 50, size=(m, m), dtype=np.int64)
    np.fill_diagonal(w, 0)
    w[np.arange(m - 1), np.arange(1, m)] = 1000
    return w


def test_sweep_cap_stops_the_widest_path_run(ctx):
    import torch
    import paper_2505_12976_amd as sz
    m = 300
    wn = chain(m, 901)
    w = torch.from_numpy(wn.astype(np.int32)).cuda()
    want = oracle.widest_from(wn, 0)
    log(f"[case] widest m={m} capped at 3 sweeps")
    ctx.set_sweep_limits(0, 3)
    ctx.widest_from(w, 0)
    torch.cuda.synchronize()
    assert ctx.device_error() == sz.EDEVICE
    ctx.set_sweep_limits(0, 0)
    log(f"[case] widest m={m} default limits")
    got = ctx.widest_from(w, 0).cpu().numpy().astype(np.int64)
    assert ctx.device_error() == 0
    assert (got == want).all()


def test_barrier_poll_limit_stops_the_run(ctx):
    import torch
    import paper_2505_12976_amd as sz
    m = 4096
    rng = np.random.default_rng(902)
    wn = rng.integers(0, 1 << 20, size=(m, m), dtype=np.int64)
    np.fill_diagonal(wn, 0)
    w = torch.from_numpy(wn.astype(np.int32)).cuda()
    log(f"[case] widest m={m} with one barrier poll allowed")
    ctx.set_sweep_limits(1, 0)
    ctx.widest_from(w, 5)
    torch.cuda.synchronize()
    assert ctx.device_error() == sz.EDEVICE
    ctx.set_sweep_limits(0, 0)
    log(f"[case] widest m={m} default limits")
    got = ctx.widest_from(w, 5).cpu().numpy().astype(np.int64)
    assert ctx.device_error() == 0
    assert (got == oracle.widest_from(wn, 5)).all()


@pytest.mark.parametrize("path", ["learned", "propagate"])
def test_winner_calls_report_a_stopped_sweep(ctx, path):
    import torch
    import paper_2505_12976_amd as sz
    m, n = 600, 5000
    b = workload.pl_zipf(903, n, m, 1.0, 12)
    dn = oracle.pairwise(b, m)
    d = torch.from_numpy(dn.astype(np.int32)).cuda()

    def call():
        if path == "learned":
            ctx.set_proposer("borda")
            return ctx.winners_learned(d, float(n), None)
        return ctx.winners_propagate(d)

    log(f"[case] {path} winners m={m} with sweeps capped at 1")
    ctx.set_sweep_limits(0, 1)
    with pytest.raises(sz.SchulzeError) as e:
        call()
    assert e.value.code == sz.EDEVICE
    assert ctx.device_error() == sz.EDEVICE
    ctx.set_sweep_limits(0, 0)
    log(f"[case] {path} winners m={m} default limits")
    w, nw, _ = call()
    assert ctx.device_error() == 0
    got = np.flatnonzero(w.cpu().numpy())
    _, win, _ = oracle.rank(oracle.closure(oracle.weights(dn)))
    assert (got == np.flatnonzero(win)).all() and int(nw.cpu()[0]) == len(got)
    if path == "learned":
        ctx.set_proposer("network")
