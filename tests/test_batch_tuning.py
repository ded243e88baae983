"""Persisted batch closure schedules (host logic, with a stand-in context):
a miss tunes and writes the table, a hit sets the stored schedules without
tuning, another device, library build or value width is a miss, a longer
m_max or retune tunes again, and an unreadable file is rewritten."""
import json

import numpy as np

from paper_2505_12976_amd.batch import tuned_closures

NAMES = ["registers", "tiled32", "tiled64", "tiled128"]


class FakeCtx:
    def __init__(self):
        self.tuned = 0
        self.set_calls = []

    def batch_autotune(self, bits, m_max):
        self.tuned += 1
        nb = (m_max + 31) // 32
        return np.arange(nb * 4, dtype=np.float32).reshape(nb, 4)

    def batch_get_closure(self, bits, m):
        return NAMES[(m // 32 + bits) % 4]

    def batch_set_closure(self, bits, lo, hi, v):
        self.set_calls.append((bits, lo, hi, v))


def test_miss_then_hit(tmp_path):
    path = str(tmp_path / "t.json")
    c = FakeCtx()
    s1, hit1 = tuned_closures(c, 16, 200, path=path, device_key="gfx950|X|256", library="abc")
    assert not hit1 and c.tuned == 1 and len(s1) == 7
    c2 = FakeCtx()
    s2, hit2 = tuned_closures(c2, 16, 200, path=path, device_key="gfx950|X|256", library="abc")
    assert hit2 and c2.tuned == 0 and s2 == s1
    assert c2.set_calls == [(16, 32 * b + 1, 32 * (b + 1), s1[b]) for b in range(7)]
    # a smaller m_max is served from the same entry
    s3, hit3 = tuned_closures(FakeCtx(), 16, 64, path=path, device_key="gfx950|X|256", library="abc")
    assert hit3 and s3 == s1[:2]
    table = json.load(open(path))
    assert list(table) == ["gfx950|X|256|abc|16"] and table["gfx950|X|256|abc|16"]["m_max"] == 200


def test_other_keys_and_retune(tmp_path):
    path = str(tmp_path / "t.json")
    tuned_closures(FakeCtx(), 16, 100, path=path, device_key="d1", library="l1")
    for kw in ({"device_key": "d2", "library": "l1"}, {"device_key": "d1", "library": "l2"}):
        c = FakeCtx()
        _, hit = tuned_closures(c, 16, 100, path=path, **kw)
        assert not hit and c.tuned == 1
    c = FakeCtx()
    _, hit = tuned_closures(c, 32, 100, path=path, device_key="d1", library="l1")
    assert not hit and c.tuned == 1
    c = FakeCtx()
    _, hit = tuned_closures(c, 16, 300, path=path, device_key="d1", library="l1")  # beyond the stored buckets
    assert not hit and c.tuned == 1
    c = FakeCtx()
    _, hit = tuned_closures(c, 16, 100, path=path, device_key="d1", library="l1", retune=True)
    assert not hit and c.tuned == 1
    assert len(json.load(open(path))) == 4  # the last two rewrote d1|l1|16


def test_unreadable_file_is_rewritten(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    c = FakeCtx()
    _, hit = tuned_closures(c, 16, 40, path=str(path), device_key="d", library="l")
    assert not hit and c.tuned == 1 and "d|l|16" in json.load(open(path))
