"""CPU oracle of the learned candidate scorer -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy: the 288 -> 256 -> 256 -> 1 network (GELU in its tanh form,
sigmoid output, MSE loss), its gradient by the chain rule, one Adam step, the
per-polygon shape features and the per-pair input rows.  The scorer is not
in the paper (it is an added systems form); what pins these functions:

- ``backward``: central finite differences of ``loss`` (tests);
- ``forward_mixed`` / ``backward_mixed`` (the network as trained: hidden
  activations BF16 between the layers, the backward products' operands BF16):
  with the rounding switched off they equal ``forward`` / ``backward``
  exactly, and with it on they stay within BF16's rounding of them (tests);
- ``gelu``: the erf form of GELU, which the tanh form approximates to ~1e-3;
- ``adam_step``: the closed form of the first step, lr * g / (|g| + eps);
- ``poly_features`` / ``pair_features``: shoelace areas, perimeters and
  centroids of rectangles and triangles in closed form (tests), and Jhat
  equal to the fraction of equal signature entries by construction.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 288, 256
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HID * N_IN
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
N_PARAMS = OFF_B3 + 1
GELU_C = math.sqrt(2.0 / math.pi)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest BF16 (ties to even), as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    u = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(N_HID, N_IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(N_HID, N_HID),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(GELU_C * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3 * 0.044715 * z * z)


def forward(X, params):
    W1, b1, W2, b2, w3, b3 = unpack(params)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    z3 = h2 @ w3 + b3
    y = 1.0 / (1.0 + np.exp(-z3))
    return {"z1": z1, "h1": h1, "z2": z2, "h2": h2, "y": y}


def loss(X, params, label):
    y = forward(X, params)["y"]
    return float(np.mean((y - label) ** 2))


def backward(X, params, label):
    """Gradient of mean (y - label)^2 with respect to the parameter block."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    a = forward(X, params)
    B = X.shape[0]
    y = a["y"]
    dz3 = 2.0 * (y - label) / B * y * (1.0 - y)
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = a["h2"].T @ dz3
    g[OFF_B3] = dz3.sum()
    dz2 = np.outer(dz3, w3) * gelu_grad(a["z2"])
    g[OFF_W2:OFF_B2] = (dz2.T @ a["h1"]).reshape(-1)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(a["z1"])
    g[OFF_W1:OFF_B1] = (dz1.T @ X).reshape(-1)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    return g


def _bf16(x, on=True):
    """FP64 values rounded as an FP32 computation hands them to BF16 storage
    (to FP32, then to the nearest BF16, ties to even), back in FP64."""
    if not on:
        return x
    return bf16_round(np.asarray(x, dtype=np.float32)).astype(np.float64)


def forward_mixed(X, params, bf16=True):
    """The network as its matrix-core kernels define it: BF16 weights and
    inputs (the caller passes BF16-valued ones), the hidden activations
    GELU(z1) and GELU(z2) stored as BF16 between the layers, everything else
    exact (FP64 here)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    z1 = X @ W1.T + b1
    h1 = _bf16(gelu(z1), bf16)
    z2 = h1 @ W2.T + b2
    h2 = _bf16(gelu(z2), bf16)
    z3 = h2 @ w3 + b3
    y = 1.0 / (1.0 + np.exp(-z3))
    return {"z1": z1, "h1": h1, "z2": z2, "h2": h2, "y": y}


def backward_mixed(X, params, label, bf16=True, terms=False):
    """Gradient of the batch MSE through ``forward_mixed`` by the chain rule,
    each stored activation used where the forward pass used it (a rounding
    passes the gradient through unchanged), and the operands of the two
    backward matrix products dz2 and dz1 rounded to BF16 as the matrix cores
    take them; the bias gradients add the unrounded dz.  With ``terms`` also
    returns, per gradient entry, the sum of the absolute values of the terms
    added into it (a scale for rounding bounds)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    a = forward_mixed(X, params, bf16)
    B = X.shape[0]
    y = a["y"]
    dz3 = 2.0 * (y - label) / B * y * (1.0 - y)
    g = np.zeros(N_PARAMS)
    S = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = a["h2"].T @ dz3
    S[OFF_W3:OFF_B3] = np.abs(a["h2"]).T @ np.abs(dz3)
    g[OFF_B3] = dz3.sum()
    S[OFF_B3] = np.abs(dz3).sum()
    dz2 = np.outer(dz3, w3) * gelu_grad(a["z2"])
    dz2b = _bf16(dz2, bf16)
    g[OFF_W2:OFF_B2] = (dz2b.T @ a["h1"]).reshape(-1)
    S[OFF_W2:OFF_B2] = (np.abs(dz2b).T @ np.abs(a["h1"])).reshape(-1)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    S[OFF_B2:OFF_W3] = np.abs(dz2).sum(axis=0)
    dz1 = (dz2b @ W2) * gelu_grad(a["z1"])
    dz1b = _bf16(dz1, bf16)
    g[OFF_W1:OFF_B1] = (dz1b.T @ X).reshape(-1)
    S[OFF_W1:OFF_B1] = (np.abs(dz1b).T @ np.abs(X)).reshape(-1)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    S[OFF_B1:OFF_W2] = np.abs(dz1).sum(axis=0)
    return (g, S) if terms else g


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------- features ----

def poly_features(poly, box) -> np.ndarray:
    """The 12 per-polygon values of the scorer, in FP64."""
    P = np.asarray(poly, dtype=np.float64).reshape(-1, 2)
    n = P.shape[0]
    out = np.zeros(12)
    if n < 3:
        return out
    Q = np.roll(P, -1, axis=0)
    o = P[0]
    a, b = P - o, Q - o
    cr = a[:, 0] * b[:, 1] - b[:, 0] * a[:, 1]
    a2 = cr.sum()
    A = max(0.5 * abs(a2), 0.5)
    gx = ((a[:, 0] + b[:, 0]) * cr).sum() / (3 * a2) + o[0] if a2 else o[0]
    gy = ((a[:, 1] + b[:, 1]) * cr).sum() / (3 * a2) + o[1] if a2 else o[1]
    per = np.sqrt(((Q - P) ** 2).sum(axis=1)).sum()
    x0, y0 = P.min(axis=0)
    x1, y1 = P.max(axis=0)
    nb = (box[2] - box[0] + 1.0) * (box[3] - box[1] + 1.0)
    out[0] = math.log(A) / math.log(max(nb, 2.0))
    out[1] = math.log(max(per * per / (4 * math.pi * A), 1e-12)) / 4
    out[2] = math.log((x1 - x0 + 1) / (y1 - y0 + 1)) / 2
    out[3] = math.log(n) / 9
    out[4] = (gx - 0.5 * (x0 + x1)) / math.sqrt(A)
    out[5] = (gy - 0.5 * (y0 + y1)) / math.sqrt(A)
    out[6] = A
    out[8:12] = (x0, y0, x1 + 1, y1 + 1)
    return out


def pair_features(sig_l, f_l, sig_r, f_r) -> np.ndarray:
    """One 288-column scorer row (FP64, before BF16 rounding)."""
    row = np.zeros(N_IN)
    eq = np.asarray(sig_l) == np.asarray(sig_r)
    row[:256] = eq
    row[256:262] = f_l[:6]
    row[262:268] = f_r[:6]
    al, ar = max(f_l[6], 0.5), max(f_r[6], 0.5)
    row[268] = math.log(al / ar) / 4
    row[269] = min(al, ar) / max(al, ar)
    ix = max(0.0, min(f_l[10], f_r[10]) - max(f_l[8], f_r[8]))
    iy = max(0.0, min(f_l[11], f_r[11]) - max(f_l[9], f_r[9]))
    inter = ix * iy
    u = (f_l[10] - f_l[8]) * (f_l[11] - f_l[9]) + (f_r[10] - f_r[8]) * (f_r[11] - f_r[9]) - inter
    row[270] = inter / u if u > 0 else 0.0
    row[271] = eq.mean()
    return row
