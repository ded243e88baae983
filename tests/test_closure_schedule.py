"""The persistent closure's work schedule, simulated on the CPU.

`k_fw_persist` (csrc/closure.hip) runs the blocked (max, min) recurrence of
Section 2.1 as one cooperative launch: every tile has a fixed owner
workgroup, published diagonal and panel tiles raise flags, and workgroups
wait on flags.  This test replays, in Python, the per-workgroup order of
that kernel (owner map, lookahead of the next diagonal, early and critical
panels, the two-rounds-ahead diagonal, the non-blocking flag checks) under
random interleavings, and checks that (a) no interleaving deadlocks and
(b) every interleaving yields the oracle's closure.  It models the
schedule, not the GPU code: the GPU parity tests check the kernel itself.
"""
import numpy as np
import pytest

import oracle


def owner(I, J, nb, G):
    return (I * nb + (I + J) % nb) % G


def owned_tiles(w, nb, G):
    """Tiles of workgroup w in the kernel's order: numbers k = w, w + G, ...
    below nb^2, each standing for block row I = k // nb and column
    J = (k mod nb - I) mod nb; returned as tile ids I nb + J."""
    out = []
    for k in range(w, nb * nb, G):
        I = k // nb
        out.append(I * nb + (k % nb - I) % nb)
    return out


def test_owned_tiles_invert_the_owner_map():
    for nb in (1, 2, 5, 8, 13, 32):
        for G in (1, 3, nb, nb + 1, 2 * nb, 3 * nb + 2, 64):
            seen = []
            for w in range(G):
                ts = owned_tiles(w, nb, G)
                assert all(owner(t // nb, t % nb, nb, G) == w for t in ts)
                seen += ts
            assert sorted(seen) == list(range(nb * nb))


def wg_program(w, nb, G, flags, gate):
    """The order in which workgroup w takes its items: ('diag'|'panel'|'rest'|'probe', round, I, J, flags waited on).
    gate: early steps while nb^2 <= gate * G (20 for uint16, 8 for int32)."""
    owned = owned_tiles(w, nb, G)
    early = nb * nb <= gate * G
    has_panels = lambda r: any(((t // nb) == r) != ((t % nb) == r) for t in owned)

    def panels(r):
        for t in owned:
            I, J = divmod(t, nb)
            if (I == r) != (J == r):
                yield ('panel', r, I, J, [(r, 0)])

    panels_done, diag_done = -1, -1
    for r in range(-1, nb):
        if r >= 0 and panels_done != r:
            if has_panels(r):
                yield from panels(r)
            panels_done = r
        next_panels = False
        if r + 1 < nb:
            if owner(r + 1, r + 1, nb, G) == w and diag_done < r + 1:
                if r >= 0:
                    yield ('rest', r, r + 1, r + 1, [(r, 1 + r + 1), (r, 1 + nb + r + 1)])
                yield ('diag', r + 1, r + 1, r + 1, [])
                diag_done = r + 1
            if r < 0:
                continue
            for t in owned:
                I, J = divmod(t, nb)
                if I == r or J == r or (I != r + 1 and J != r + 1) or (I == r + 1 and J == r + 1):
                    continue
                yield ('rest', r, I, J, [(r, 1 + J), (r, 1 + nb + I)])
            next_panels = early and has_panels(r + 1)
            critical = r + 2 < nb and (owner(r + 1, r + 2, nb, G) == w or owner(r + 2, r + 1, nb, G) == w)
            if next_panels and not critical:
                yield ('probe', r + 1, 0, 0, [])
            if next_panels and (critical or (r + 1, 0) in flags):
                yield from panels(r + 1)  # each waits for round r+1's diagonal
                panels_done, next_panels = r + 1, False
        ahead = -1
        if early and nb <= G and r + 2 < nb and owner(r + 2, r + 2, nb, G) == w:
            yield ('rest', r, r + 2, r + 2, [(r, 1 + r + 2), (r, 1 + nb + r + 2)])
            yield ('rest', r + 1, r + 2, r + 2, [(r + 1, 1 + r + 2), (r + 1, 1 + nb + r + 2)])
            yield ('diag', r + 2, r + 2, r + 2, [])
            diag_done, ahead = r + 2, (r + 2) * nb + (r + 2)
        for t in owned:
            I, J = divmod(t, nb)
            if I == r or J == r or I == r + 1 or J == r + 1 or t == ahead:
                continue
            if next_panels:
                yield ('probe', r + 1, 0, 0, [])
                if (r + 1, 0) in flags:
                    yield from panels(r + 1)
                    panels_done, next_panels = r + 1, False
            yield ('rest', r, I, J, [(r, 1 + J), (r, 1 + nb + I)])


def maxmin(A, Bm):
    return np.max(np.minimum(A[:, :, None], Bm[None, :, :]), axis=1)


def simulate(w0, B, G, rng, gate):
    m = w0.shape[0]
    nb = m // B
    P = w0.copy()
    ring, flags = {}, set()
    progs = [wg_program(w, nb, G, flags, gate) for w in range(G)]
    pending = [next(p, None) for p in progs]
    tile = lambda a, b: P[a * B:(a + 1) * B, b * B:(b + 1) * B]
    while any(x is not None for x in pending):
        ready = [w for w in range(G) if pending[w] is not None and all(f in flags for f in pending[w][4])]
        if not ready:
            raise RuntimeError("deadlock")
        w = ready[rng.integers(len(ready))]
        kind, r, I, J, _ = pending[w]
        if kind == 'diag':
            D = tile(r, r).copy()
            for k in range(B):
                D = np.maximum(D, np.minimum(D[:, k:k + 1], D[k:k + 1, :]))
            tile(r, r)[:] = D
            ring[(r, 0)] = D.copy()
            flags.add((r, 0))
        elif kind == 'panel':
            D, C = ring[(r, 0)], tile(I, J).copy()
            if I == r:
                new, slot = np.maximum(C, maxmin(D, C)), 1 + J
            else:
                new, slot = np.maximum(C, maxmin(C, D)), 1 + nb + I
            tile(I, J)[:] = new
            ring[(r, slot)] = new.copy()
            flags.add((r, slot))
        elif kind == 'rest':
            tile(I, J)[:] = np.maximum(tile(I, J), maxmin(ring[(r, 1 + nb + I)], ring[(r, 1 + J)]))
        pending[w] = next(progs[w], None)
    np.fill_diagonal(P, 0)
    return P


# (m, B, G): early steps on and off, G a multiple of nb, G >= nb but not a
# multiple (G = nb + 1 gives tile (r+2, r+2) and panel (r+1, r+2) one owner),
# G < nb, one to several tiles per workgroup
@pytest.mark.parametrize("m,B,G", [(16, 4, 3), (24, 4, 7), (32, 8, 5), (32, 4, 64), (40, 4, 16), (64, 8, 8),
                                   (48, 4, 12), (64, 4, 40), (36, 4, 9), (44, 4, 11), (36, 4, 10), (44, 4, 12),
                                   (44, 4, 13), (40, 4, 23), (44, 4, 7)])
@pytest.mark.parametrize("gate", [8, 20])
def test_schedule_never_deadlocks_and_closes_exactly(m, B, G, gate):
    rng = np.random.default_rng(m * 1000 + G)
    w = rng.integers(0, 9, size=(m, m)).astype(np.int64) * (rng.random((m, m)) < 0.5)
    np.fill_diagonal(w, 0)
    want = oracle.closure(w)
    for _ in range(4):
        assert (simulate(w, B, G, rng, gate) == want).all()


@pytest.mark.parametrize("nb,G", [(111, 768), (64, 1280), (96, 768), (100, 768), (9, 10), (13, 5), (520, 768)])
def test_owner_map_balance(nb, G):
    """Every workgroup owns floor or ceil of nb^2 / G tiles; block rows spread
    over distinct workgroups when nb <= G, block columns too when nb divides G."""
    I, J = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    o = owner(I, J, nb, G)
    cnt = np.bincount(o.ravel(), minlength=G)
    assert cnt.max() - cnt.min() <= 1 and cnt.sum() == nb * nb
    if nb <= G:
        assert all(len(set(o[i, :])) == nb for i in range(nb))
        if G % nb == 0:
            assert all(len(set(o[:, j])) == nb for j in range(nb))
