"""CPU reference of the learned winner proposer (TEST INFRASTRUCTURE ONLY).

A 16 -> 128 -> 128 -> 1 ReLU network over per-candidate features, the
segmented softmax loss over elections, and its gradients, written out with
numpy.  It shares no code with the GPU library.  The parameter layout is
the library's:

    W1[16][128] | b1[128] | W2[128][128] | b2[128] | W3[128] | b3[1]

``rounding=True`` (float32 arithmetic) rounds to bfloat16 (nearest even) at
the points the GPU kernels do: inputs, W1, W2, W3, h1, h2, dz2, dz1.
``rounding=False`` with float64 is the exact-arithmetic model whose
gradients are checked against central finite differences.

The network itself is not from the paper; its inputs mirror quantities the
paper uses: Borda scores (the vertex-id order of Section 4) and the
initialisation filter (largest incoming vs outgoing edge weight, Section 4).
"""
from __future__ import annotations

import numpy as np

NF, NH = 16, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + NF * NH
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def unpack(params: np.ndarray):
    p = np.asarray(params)
    return (p[OFF_W1:OFF_B1].reshape(NF, NH), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(NH, NH),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation (float32)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, dtype=np.float32)
    p[OFF_W1:OFF_B1] = rng.standard_normal(NF * NH) * np.sqrt(2.0 / NF)
    p[OFF_W2:OFF_B2] = rng.standard_normal(NH * NH) * np.sqrt(2.0 / NH)
    p[OFF_W3:OFF_B3] = rng.standard_normal(NH) * np.sqrt(1.0 / NH)
    return p


def forward(params, X, rounding: bool = True, dtype=np.float32) -> dict:
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(params, dtype=dtype))
    X = np.asarray(X, dtype=dtype)
    r = bf16 if rounding else (lambda a: a)
    x = r(X)
    z1 = x @ r(W1) + b1
    h1 = r(np.maximum(z1, 0))
    z2 = h1 @ r(W2) + b2
    h2 = r(np.maximum(z2, 0))
    s = h2 @ r(W3) + b3
    return {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "s": s}


def seg_loss(s, offsets, winner, dtype=np.float32):
    """Mean over elections of log sum_all exp(s) - log sum_winners exp(s), and
    its gradient with respect to s."""
    s = np.asarray(s, dtype=dtype)
    ds = np.zeros_like(s)
    E = len(offsets) - 1
    total = 0.0
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        seg = s[a:b]
        wm = np.asarray(winner[a:b], dtype=bool)
        if not wm.any():
            continue
        mx = seg.max()
        ex = np.exp(seg - mx)
        sa, sw = ex.sum(), ex[wm].sum()
        total += np.log(sa) - np.log(sw)
        g = ex / sa
        g[wm] -= ex[wm] / sw
        ds[a:b] = g / E
    return total / E, ds


def backward(params, X, ds, rounding: bool = True, dtype=np.float32) -> np.ndarray:
    """Gradient of sum(ds * s) with respect to the parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(params, dtype=dtype))
    r = bf16 if rounding else (lambda a: a)
    f = forward(params, X, rounding, dtype)
    ds = np.asarray(ds, dtype=dtype)
    g = np.zeros(NPARAM, dtype=dtype)
    g[OFF_W3:OFF_B3] = f["h2"].T @ ds
    g[OFF_B3] = ds.sum()
    dz2 = r(np.where(f["z2"] > 0, np.outer(ds, r(W3)), 0).astype(dtype))
    g[OFF_W2:OFF_B2] = (f["h1"].T @ dz2).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dh1 = dz2 @ r(W2).T
    dz1 = r(np.where(f["h1"] > 0, dh1, 0).astype(dtype))
    g[OFF_W1:OFF_B1] = (f["x"].T @ dz1).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    return g


def loss_value(params, X, offsets, winner, rounding=False, dtype=np.float64):
    return seg_loss(forward(params, X, rounding, dtype)["s"], offsets, winner, dtype)[0]
