"""Proposer checkpoints: a save/load round trip keeps every array, the step
and the metadata; a damaged file (one parameter changed, the step changed)
or an unknown version is refused; the shipped checkpoint loads."""
import os

import numpy as np
import pytest

from paper_2505_12976_amd import proposer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _arrays(seed):
    rng = np.random.default_rng(seed)
    n = proposer.N_PARAMS
    return (rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32),
            rng.random(n).astype(np.float32))


def test_round_trip(tmp_path):
    p, m, v = _arrays(1)
    path = str(tmp_path / "c.npz")
    proposer.save_checkpoint(path, p, m, v, 17, {"seed": 5, "note": "x"})
    c = proposer.load_checkpoint(path)
    assert np.array_equal(c["params"], p) and np.array_equal(c["adam_m"], m) and np.array_equal(c["adam_v"], v)
    assert c["step"] == 17 and c["meta"] == {"seed": "5", "note": "x"}


def _rewrite(src, dst, **changes):
    with np.load(src, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d.update(changes)
    np.savez(dst, **d)


@pytest.mark.parametrize("what", ["param", "step", "meta", "version"])
def test_damaged_checkpoint_is_refused(tmp_path, what):
    p, m, v = _arrays(2)
    good = str(tmp_path / "good.npz")
    bad = str(tmp_path / "bad.npz")
    proposer.save_checkpoint(good, p, m, v, 3, {"k": "v"})
    if what == "param":
        q = p.copy()
        q[1234] = np.nextafter(q[1234], np.float32(np.inf))  # one ulp
        _rewrite(good, bad, params=q)
    elif what == "step":
        _rewrite(good, bad, step=np.int64(4))
    elif what == "meta":
        _rewrite(good, bad, meta_values=np.array(["w"], dtype=str))
    else:
        _rewrite(good, bad, version=np.int64(1))
    with pytest.raises(ValueError):
        proposer.load_checkpoint(bad)


def test_shipped_checkpoint_loads():
    c = proposer.load_checkpoint(os.path.join(ROOT, "paper_2505_12976_amd", "data", "proposer.npz"))
    assert c["params"].shape == (proposer.N_PARAMS,) and np.isfinite(c["params"]).all()
