"""schulze_verify_noalloc (sweep state in the library's static device
scratch, no allocation) against schulze_verify (context workspace): the same
verdict, widths and tied set, on two calls in a row, the second smaller."""
import numpy as np
import pytest

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


def _weights(ctx, seed, m, dtype):
    import torch
    b = workload.mallows(seed, 900, m, 0.93, trunc_mod=4, trunc_lt=1, trunc_k=30)
    d = ctx.pairwise(torch.from_numpy(b).cuda(), m, dtype=dtype)
    return ctx.weights(d)


@pytest.mark.parametrize("dtype", ["i32", "u16"])
def test_verify_noalloc_matches_verify(ctx, dtype):
    import torch
    for m, seed in ((1500, 91), (333, 92)):  # the second call is smaller
        w, wt = _weights(ctx, seed, m, dtype)
        score = torch.from_numpy(np.random.default_rng(seed).standard_normal(m).astype(np.float32)).cuda()
        for cand in (0, m // 2, m - 1):
            log(f"[case] verify_noalloc dtype={dtype} m={m} cand={cand}")
            ref = ctx.verify(w, wt, cand, score=score, want_tied=True)
            got = ctx.verify(w, wt, cand, score=score, want_tied=True, noalloc=True)
            torch.cuda.synchronize()
            assert ctx.device_error() == 0
            vr, vg = ref[0].cpu().numpy(), got[0].cpu().numpy()
            assert (vr == vg).all(), (vr, vg)
            assert torch.equal(ref[1], got[1]) and torch.equal(ref[2], got[2])
            nt = int(vr[3])
            assert sorted(ref[3][:nt].cpu().tolist()) == sorted(got[3][:nt].cpu().tolist())
