"""Host side of batches (CPU only): packing of elections into one flat
ballot array with descriptors, and the batched workload's generator."""
import numpy as np

import workload
from paper_2505_12976_amd.batch import pack


def test_pack_lays_out_elections_back_to_back():
    a = workload.mallows(11, 5, 4, 0.9, election=0)
    b = workload.uniform_ballots(11, 3, 7, 2, election=1)
    c = np.zeros((0, 3), dtype=np.uint16)
    pk = pack([a, b, c], [4, 7, 3])
    assert pk.elections == [(0, 5, 4, 4, 0, 0), (20, 3, 2, 7, 16, 4), (26, 0, 3, 3, 65, 11)]
    assert pk.d_elems == 16 + 49 + 9 and pk.vec_elems == 14
    np.testing.assert_array_equal(pk.ballots[:20].reshape(5, 4), a)
    np.testing.assert_array_equal(pk.ballots[20:26].reshape(3, 2), b)
    flat = np.arange(pk.d_elems)
    np.testing.assert_array_equal(pk.mat(flat, 1), np.arange(16, 65).reshape(7, 7))
    np.testing.assert_array_equal(pk.vec(np.arange(14), 2), [11, 12, 13])


def test_pack_int32_keeps_negative_padding():
    b = np.array([[2, 0, -1], [1, -1, -1]], dtype=np.int32)
    pk = pack([b], [3], dtype=np.int32)
    assert pk.ballots.dtype == np.int32
    np.testing.assert_array_equal(pk.ballots, b.reshape(-1))


def test_batched_workload_sizes_and_rankings():
    ms, ns, phis = workload.batch_params(1004, 4096)
    assert ms.min() >= 8 and ms.max() <= 512 and ns.min() >= 50 and ns.max() <= 20000
    assert 0.5 <= phis.min() and phis.max() <= 1.0
    # the generator is deterministic per election and writes permutations
    flat, desc, (ms8, ns8, _) = workload.batch_mallows(1004, 6, n_hi=400)
    for e, (bo, n, L, m, mo, vo) in enumerate(desc):
        rows = flat[bo:bo + n * m].reshape(n, m)
        assert (np.sort(rows, axis=1) == np.arange(m)).all()
        np.testing.assert_array_equal(rows, workload.batch_election(1004, e, m, n, workload.batch_params(
            1004, 6, n_hi=400)[2][e]))
    assert [d[4] for d in desc] == list(np.concatenate([[0], np.cumsum(ms8 * ms8)[:-1]]))
