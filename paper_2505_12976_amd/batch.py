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


# ------------------------------------------------------------------ persisted schedules
def _library_digest() -> str:
    import hashlib
    from . import LIB_PATH
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        for block in iter(lambda: f.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()[:16]


def _device_key(ctx) -> str:
    import torch
    p = torch.cuda.get_device_properties(ctx._torch_device)
    return f"{getattr(p, 'gcnArchName', '?')}|{p.name}|{p.multi_processor_count}"


def default_tuning_path() -> str:
    import os
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "schulze_mi355x", "batch_closure.json")


def tuned_closures(ctx, value_bits: int, m_max: int, path: str | None = None, device_key: str | None = None,
                   library: str | None = None, retune: bool = False):
    """Closure schedules of the batch kernel per bucket of 32 candidates up
    to m_max, for values of value_bits bits.  The table is kept in a JSON
    file (default: default_tuning_path()) keyed by the device (architecture,
    name, compute units), the library build (a digest of libschulze.so) and
    the value width: a hit sets the stored schedules, a miss (or retune, or
    a stored table that stops below m_max) runs Context.batch_autotune and
    stores its choice.  Returns (schedules per bucket, True if they came
    from the file)."""
    import json
    import os
    path = path or default_tuning_path()
    key = "|".join([device_key or _device_key(ctx), library or _library_digest(), str(int(value_bits))])
    nb = (int(m_max) + 31) // 32
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}  # unreadable: tune again and rewrite it
    entry = table.get(key)
    if not retune and isinstance(entry, dict) and len(entry.get("schedules", [])) >= nb:
        sched = list(entry["schedules"][:nb])
        for b, v in enumerate(sched):
            ctx.batch_set_closure(value_bits, 32 * b + 1, 32 * (b + 1), v)
        return sched, True
    ms = ctx.batch_autotune(value_bits, int(m_max))
    sched = [ctx.batch_get_closure(value_bits, 32 * (b + 1)) for b in range(nb)]
    table[key] = {"schedules": sched, "m_max": int(m_max), "ms": [[float(x) for x in row] for row in ms]}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return sched, False
