"""CPU oracle of the swap-proposal CNN -- TEST INFRASTRUCTURE ONLY.

A plain numpy (float64) statement of the network that ranks pixel interchanges for the annealer
(the paper leaves the modification operator open, Sec. 4: "more sophisticated" operators can be
plugged in; the exact lineal-path change still judges every move).  Nothing here is shared with
the HIP kernels.

Network (periodic 'same' convolutions on a W x H cell, channels last):
  X0[p] = (pixel value, interface flag)           interface: a 4-neighbour of the other phase
  Z1 = conv3x3(X0; W1, b1), A1 = q(relu(Z1))        16 channels
  Z2 = conv3x3(A1; W2, b2), A2 = q(relu(Z2))        16 channels
  Z3 = conv3x3(A2; W3, b3), A3 = q(relu(Z3))        16 channels
  S[p] = A3[p] . W4 + b4                          per-pixel score
conv3x3(X; W, b)[y, x, co] = b[co] + sum_{dy,dx,ci} W[t, co, ci] X[(y+dy-1) % H, (x+dx-1) % W, ci]
with tap t = 3 dy + dx.  q() rounds to bfloat16 (round to nearest even, via float32) and the
weights enter rounded to bfloat16 (`bf16=True`); with `bf16=False` everything stays float64
(used for finite-difference checks).

Loss for interchange samples (image i, phase-1 pixel a, phase-0 pixel b, target y):
  L = mean_s (S_i[a] + S_i[b] - y)^2.
Backward: the derivative of q() is taken as 1 and relu'(Z) as [A > 0]; the gradient images dZ
are rounded to bfloat16 like the activations when `bf16=True`.

Parameters are packed in one float32 vector (pack/unpack below):
  W1 [9][16][2], b1 [16], W2 [9][16][16], b2 [16], W3 [9][16][16], b3 [16], W4 [16], b4 [1].
"""
from __future__ import annotations

import numpy as np

C = 16
SHAPES = [("W1", (9, C, 2)), ("b1", (C,)), ("W2", (9, C, C)), ("b2", (C,)),
          ("W3", (9, C, C)), ("b3", (C,)), ("W4", (C,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k, _ in SHAPES]).astype(np.float32)


def unpack(v) -> dict:
    v = np.asarray(v, np.float64)
    out, o = {}, 0
    for k, s in SHAPES:
        n = int(np.prod(s))
        out[k] = v[o:o + n].reshape(s)
        o += n
    return out


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation (uniform), float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for k, s in SHAPES:
        if k.startswith("W"):
            fan_in = s[2] * 9 if len(s) == 3 else s[0]
            lim = np.sqrt(6.0 / fan_in)
            p[k] = g.uniform(-lim, lim, size=s)
        else:
            p[k] = np.zeros(s)
    return pack(p)


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) through float32; returns float64 values."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    nan = np.isnan(f)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def features(img) -> np.ndarray:
    """X0 (H, W, 2): pixel value and interface flag (periodic 4-neighbourhood)."""
    a = np.asarray(img).astype(np.int64)
    itf = ((np.roll(a, 1, 0) != a) | (np.roll(a, -1, 0) != a) |
           (np.roll(a, 1, 1) != a) | (np.roll(a, -1, 1) != a))
    return np.stack([a, itf.astype(np.int64)], axis=-1).astype(np.float64)


def conv3x3(X, Wt, b) -> np.ndarray:
    H, Wd, _ = X.shape
    out = np.broadcast_to(np.asarray(b, np.float64), (H, Wd, Wt.shape[1])).copy()
    for dy in range(3):
        for dx in range(3):
            Xs = np.roll(X, shift=(1 - dy, 1 - dx), axis=(0, 1))  # Xs[y,x] = X[y+dy-1, x+dx-1]
            out += Xs @ Wt[3 * dy + dx].T
    return out


def conv3x3_transpose(dZ, Wt) -> np.ndarray:
    """Adjoint of conv3x3 in its input: dX[y,x,ci] = sum dZ[y-dy+1, x-dx+1, co] W[t, co, ci]."""
    H, Wd, _ = dZ.shape
    out = np.zeros((H, Wd, Wt.shape[2]))
    for dy in range(3):
        for dx in range(3):
            Zs = np.roll(dZ, shift=(dy - 1, dx - 1), axis=(0, 1))
            out += Zs @ Wt[3 * dy + dx]
    return out


def conv3x3_weight_grad(dZ, X) -> np.ndarray:
    """dW[t, co, ci] = sum_p dZ[p, co] X[p + off(t), ci]."""
    out = np.zeros((9, dZ.shape[2], X.shape[2]))
    Zf = dZ.reshape(-1, dZ.shape[2])
    for dy in range(3):
        for dx in range(3):
            Xs = np.roll(X, shift=(1 - dy, 1 - dx), axis=(0, 1)).reshape(-1, X.shape[2])
            out[3 * dy + dx] = Zf.T @ Xs
    return out


def forward(params, img, bf16_mode: bool = True) -> dict:
    p = unpack(params)
    q = bf16 if bf16_mode else (lambda x: np.asarray(x, np.float64))
    W1, W2, W3, W4 = (q(p[k]) for k in ("W1", "W2", "W3", "W4"))
    X0 = features(img)
    Z1 = conv3x3(X0, W1, p["b1"])
    A1 = q(np.maximum(Z1, 0.0))
    Z2 = conv3x3(A1, W2, p["b2"])
    A2 = q(np.maximum(Z2, 0.0))
    Z3 = conv3x3(A2, W3, p["b3"])
    A3 = q(np.maximum(Z3, 0.0))
    S = A3 @ W4 + p["b4"][0]
    return dict(X0=X0, Z1=Z1, A1=A1, Z2=Z2, A2=A2, Z3=Z3, A3=A3, S=S, W1=W1, W2=W2, W3=W3, W4=W4)


def loss_and_grad(params, imgs, samples, bf16_mode: bool = True):
    """samples: structured or (n, 4) array of (image index, a, b, y).  Returns (loss, grad vector
    float64 in the packed order)."""
    s = np.asarray(samples)
    idx = s[:, 0].astype(np.int64)
    a = s[:, 1].astype(np.int64)
    b = s[:, 2].astype(np.int64)
    y = s[:, 3].astype(np.float64)
    n = len(s)
    q = bf16 if bf16_mode else (lambda x: np.asarray(x, np.float64))
    grads = {k: np.zeros(sh) for k, sh in SHAPES}
    loss = 0.0
    fwd = [forward(params, im, bf16_mode) for im in imgs]
    dS = [np.zeros(f["S"].shape) for f in fwd]
    for t in range(n):
        f = fwd[idx[t]]
        Sf = f["S"].ravel()
        r = Sf[a[t]] + Sf[b[t]] - y[t]
        loss += r * r
        g = 2.0 * r / n
        dS[idx[t]].flat[a[t]] += g
        dS[idx[t]].flat[b[t]] += g
    loss /= n
    for f, d in zip(fwd, dS):
        grads["b4"][0] += d.sum()
        grads["W4"] += np.tensordot(d, f["A3"], axes=([0, 1], [0, 1]))
        dZ3 = q(d[..., None] * f["W4"][None, None, :] * (f["A3"] > 0))
        grads["W3"] += conv3x3_weight_grad(dZ3, f["A2"])
        grads["b3"] += dZ3.sum(axis=(0, 1))
        dZ2 = q(conv3x3_transpose(dZ3, f["W3"]) * (f["A2"] > 0))
        grads["W2"] += conv3x3_weight_grad(dZ2, f["A1"])
        grads["b2"] += dZ2.sum(axis=(0, 1))
        dZ1 = q(conv3x3_transpose(dZ2, f["W2"]) * (f["A1"] > 0))
        grads["W1"] += conv3x3_weight_grad(dZ1, f["X0"])
        grads["b1"] += dZ1.sum(axis=(0, 1))
    return loss, np.concatenate([grads[k].ravel() for k, _ in SHAPES])


def adam(params, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015) in float32: returns (params, m, v)."""
    p = np.asarray(params, np.float32)
    g = np.asarray(grad, np.float32)
    m = (np.float32(beta1) * m + np.float32(1 - beta1) * g).astype(np.float32)
    v = (np.float32(beta2) * v + np.float32(1 - beta2) * g * g).astype(np.float32)
    mh = m / np.float32(1 - beta1 ** t)
    vh = v / np.float32(1 - beta2 ** t)
    p = (p - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(eps))).astype(np.float32)
    return p, m, v
