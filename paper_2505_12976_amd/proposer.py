"""Training and use of the learned winner proposer on the GPU.

Every arithmetic step runs in the library's kernels (features, BF16 MFMA
forward/backward, segmented loss, Adam); this module only keeps the data on
the device and drives the loop.  Labels are Schulze winner sets computed by
the library's own exact path (counts -> closure -> winners).

Checkpoints are ``.npz`` files (no pickled objects) holding the FP32
parameters, the Adam moments and the step counter.
"""
from __future__ import annotations

import numpy as np

NF, NH = 16, 128
N_PARAMS = NF * NH + NH + NH * NH + NH + NH + 1
CHECKPOINT_VERSION = 2  # 2: a CRC-32 of every stored array and the step


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initial parameters (float32), layout W1|b1|W2|b2|W3|b3."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    o = 0
    p[o:o + NF * NH] = rng.standard_normal(NF * NH) * np.sqrt(2.0 / NF)
    o += NF * NH + NH
    p[o:o + NH * NH] = rng.standard_normal(NH * NH) * np.sqrt(2.0 / NH)
    o += NH * NH + NH
    p[o:o + NH] = rng.standard_normal(NH) * np.sqrt(1.0 / NH)
    return p


def _checkpoint_crc(version: int, params, adam_m, adam_v, step: int, keys, values) -> int:
    """CRC-32 over the stored arrays (little-endian bytes), the step and the
    metadata strings, in a fixed order."""
    import zlib
    crc = zlib.crc32(np.int64(version).tobytes())
    for a in (params, adam_m, adam_v):
        crc = zlib.crc32(np.ascontiguousarray(a, dtype="<f4").tobytes(), crc)
    crc = zlib.crc32(np.int64(step).tobytes(), crc)
    for k, v in zip(keys, values):
        crc = zlib.crc32(str(k).encode() + b"\0" + str(v).encode() + b"\0", crc)
    return crc


def save_checkpoint(path: str, params: np.ndarray, adam_m: np.ndarray, adam_v: np.ndarray, step: int,
                    meta: dict | None = None) -> None:
    meta = meta or {}
    keys = [str(k) for k in meta.keys()]
    values = [str(v) for v in meta.values()]
    p32, m32, v32 = (np.asarray(a, dtype=np.float32) for a in (params, adam_m, adam_v))
    crc = _checkpoint_crc(CHECKPOINT_VERSION, p32, m32, v32, step, keys, values)
    np.savez(path, version=np.int64(CHECKPOINT_VERSION), params=p32, adam_m=m32, adam_v=v32, step=np.int64(step),
             meta_keys=np.array(keys, dtype=str), meta_values=np.array(values, dtype=str), crc32=np.int64(crc))


def load_checkpoint(path: str) -> dict:
    """Read a checkpoint written by save_checkpoint; ValueError if its version
    is unknown, its CRC does not match its contents or its size is wrong."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["version"]) != CHECKPOINT_VERSION:
            raise ValueError(f"unsupported checkpoint version {int(z['version'])}")
        out = {k: z[k] for k in ("params", "adam_m", "adam_v")}
        out["step"] = int(z["step"])
        keys, values = z["meta_keys"].tolist(), z["meta_values"].tolist()
        stored = int(z["crc32"])
    out["meta"] = dict(zip(keys, values))
    if _checkpoint_crc(CHECKPOINT_VERSION, out["params"], out["adam_m"], out["adam_v"], out["step"], keys,
                       values) != stored:
        raise ValueError("checkpoint CRC mismatch: the file is damaged")
    if out["params"].shape != (N_PARAMS,):
        raise ValueError("checkpoint has the wrong number of parameters")
    return out


class Trainer:
    """Accumulates (features, winner mask) per election on the GPU and fits
    the network with minibatches of whole elections."""

    def __init__(self, ctx, params: np.ndarray | None = None, seed: int = 0):
        import torch
        self.ctx = ctx
        dev = ctx._torch_device
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.from_numpy(p.copy()).to(dev)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)  # Adam steps, advanced on the device
        self.step = 0
        self._feats, self._wins, self._sizes = [], [], []
        self.feat = self.win = self.offsets = None

    def add(self, feat, winner_mask) -> None:
        """feat: (m, 16) float32 CUDA tensor; winner_mask: (m,) uint8 CUDA tensor."""
        self._feats.append(feat)
        self._wins.append(winner_mask)
        self._sizes.append(feat.shape[0])

    def finalize(self) -> None:
        import torch
        self.feat = torch.cat(self._feats).contiguous()
        self.win = torch.cat(self._wins).contiguous()
        off = np.concatenate([[0], np.cumsum(self._sizes)]).astype(np.int64)
        self.offsets_host = off
        self.offsets = torch.from_numpy(off).to(self.feat.device)
        self._feats, self._wins = [], []

    @property
    def n_elections(self) -> int:
        return len(self._sizes)

    def fit(self, epochs: int = 4, batch: int = 256, lr: float = 1e-3, log=None) -> list:
        """Adam over minibatches of `batch` consecutive elections (the
        elections are drawn independently, so consecutive blocks are i.i.d.);
        each epoch starts at a different block.  Returns mean losses per epoch."""
        import torch
        if self.feat is None:
            self.finalize()
        E = self.n_elections
        off = self.offsets_host
        starts = list(range(0, E, batch))
        history = []
        for ep in range(epochs):
            shift = ep % max(1, len(starts))
            order = starts[shift:] + starts[:shift]
            total = torch.zeros((), dtype=torch.float64, device=self.params.device)
            count = 0
            for e0 in order:
                e1 = min(E, e0 + batch)
                r0, r1 = int(off[e0]), int(off[e1])
                feat = self.feat[r0:r1]
                win = self.win[r0:r1]
                seg = (self.offsets[e0:e1 + 1] - r0).contiguous()
                loss = self.ctx.mlp_train_step(self.params, self.m1, self.m2, self.grad, self.step_dev, feat, seg,
                                               win, lr=lr)
                self.step += 1
                total += loss.sum(dtype=torch.float64)
                count += e1 - e0
            history.append(float(total.item()) / max(count, 1))
            if log:
                log(f"epoch {ep}: mean loss {history[-1]:.4f}")
        torch.cuda.synchronize()
        return history

    def save(self, path: str, meta: dict | None = None) -> None:
        save_checkpoint(path, self.params.cpu().numpy(), self.m1.cpu().numpy(), self.m2.cpu().numpy(), self.step,
                        meta)


def filtered_argmax(score: np.ndarray, feat: np.ndarray) -> int:
    """Best-scored candidate that the initialisation filter keeps (ties ->
    lowest id); all candidates if the filter removes every one."""
    keep = feat[:, 5] == 0
    if not keep.any():
        keep[:] = True
    s = np.where(keep, score, -np.inf)
    return int(np.argmax(s))
