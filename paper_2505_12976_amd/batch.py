"""Packing of many elections into one batch for ``Context.batch_run``.

Marshalling only: the ballots of every election are laid out back to back
in one flat array, and each election gets a descriptor (ballot offset, n, L,
m, offset of its m x m blocks in d and p, offset of its m-entry blocks in
the per-candidate outputs).  All arithmetic runs in the library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Packed:
    ballots: np.ndarray   # flat uint16 or int32 ids
    elections: list       # (ballot_off, n, L, m, mat_off, vec_off) per election
    d_elems: int          # elements of d and p
    vec_elems: int        # elements of is_winner, beaten_by, order

    def mat(self, t, e):
        """View of election e's m x m block of a flat d or p tensor."""
        _, _, _, m, off, _ = self.elections[e]
        return t[off:off + m * m].reshape(m, m)

    def vec(self, t, e):
        """View of election e's m-entry block of a flat per-candidate tensor."""
        _, _, _, m, _, off = self.elections[e]
        return t[off:off + m]


def pack(ballot_list, m_list, dtype=np.uint16) -> Packed:
    """ballot_list[e]: (n_e, L_e) array of ids (padding 0xFFFF or negative)."""
    dtype = np.dtype(dtype)
    sizes = [int(b.size) for b in ballot_list]
    flat = np.empty(max(sum(sizes), 1), dtype=dtype)
    elections = []
    bo = mo = vo = 0
    for b, m in zip(ballot_list, m_list):
        b = np.asarray(b)
        n, L = (b.shape if b.ndim == 2 else (0, 1))
        if b.size:
            flat[bo:bo + b.size] = b.reshape(-1).astype(dtype, copy=False)
        elections.append((bo, int(n), int(L), int(m), mo, vo))
        bo += int(b.size)
        mo += int(m) * int(m)
        vo += int(m)
    return Packed(flat, elections, mo, vo)


def alloc_outputs(packed: Packed, device, with_p=True):
    """Device tensors for a batch run: d, p (or None), is_winner, n_winners,
    beaten_by, order."""
    import torch
    E = len(packed.elections)
    d = torch.empty(max(packed.d_elems, 1), dtype=torch.int32, device=device)
    p = torch.empty_like(d) if with_p else None
    w = torch.empty(max(packed.vec_elems, 1), dtype=torch.uint8, device=device)
    nw = torch.empty(max(E, 1), dtype=torch.int32, device=device)
    bb = torch.empty(max(packed.vec_elems, 1), dtype=torch.int32, device=device)
    order = torch.empty_like(bb)
    return {"d": d, "p": p, "is_winner": w, "n_winners": nw, "beaten_by": bb, "order": order}
