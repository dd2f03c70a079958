"""FP64 reference of the warm-start network (numpy).

TEST INFRASTRUCTURE ONLY: the test suite is the only caller; nothing here is
shared with the HIP path.  The network is the one the library trains: the
Fourier features phi(x) = [sin(2 pi B x), cos(2 pi B x)] of a point x with
fixed frequencies B (n_freq x in_dim), tanh hidden layers
h_l = tanh(W_l h_{l-1} + b_l), a linear output layer y = W_L h_{L-1} + b_L,
the loss (1/(n out)) sum (y - t)^2 and Adam (beta1 0.9, beta2 0.999,
eps 1e-8) with bias correction.  Gradients are the plain chain rule written
out layer by layer.  ``bf16=True`` rounds every matrix-product operand to
BF16 (round to nearest even of the FP32 value) where the GPU kernels do,
so that both sides start from identical operands; the arithmetic itself
stays FP64.

Parameters travel in the library's flat order: frequencies [n_freq][in_dim],
then per layer W [out][in] and b [out].
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even) of the FP32 value."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return (b.astype(np.uint32)).view(np.float32).astype(np.float64)


def layer_dims(cfg):
    nl = cfg["hidden"] + 1
    dims = []
    for l in range(nl):
        fan_in = 2 * cfg["n_freq"] if l == 0 else cfg["width"]
        fan_out = cfg["out_dim"] if l == nl - 1 else cfg["width"]
        dims.append((fan_out, fan_in))
    return dims


def unflatten(cfg, flat):
    flat = np.asarray(flat, dtype=np.float64)
    k = cfg["n_freq"] * cfg["in_dim"]
    freq = flat[:k].reshape(cfg["n_freq"], cfg["in_dim"])
    Ws, bs = [], []
    for out, inp in layer_dims(cfg):
        Ws.append(flat[k:k + out * inp].reshape(out, inp))
        k += out * inp
        bs.append(flat[k:k + out].copy())
        k += out
    assert k == flat.size
    return freq, Ws, bs


def flatten(freq, Ws, bs):
    parts = [np.ravel(freq)]
    for W, b in zip(Ws, bs):
        parts += [np.ravel(W), np.ravel(b)]
    return np.concatenate(parts)


def features(x, freq):
    """phi = [sin(2 pi B x), cos(2 pi B x)], one row per point."""
    z = 2.0 * np.pi * (np.asarray(x, dtype=np.float64) @ freq.T)
    return np.concatenate([np.sin(z), np.cos(z)], axis=1)


def forward(cfg, flat, x, bf16=False):
    """Outputs and the per-layer activations (phi first)."""
    freq, Ws, bs = unflatten(cfg, flat)
    r = bf16_round if bf16 else (lambda a: a)
    acts = [features(x, freq)]
    h = acts[0]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = r(h) @ r(W).T + b
        if l < len(Ws) - 1:
            h = np.tanh(z)
            acts.append(h)
        else:
            return z, acts
    raise AssertionError("unreachable")


def loss_and_grad(cfg, flat, x, t, bf16=False):
    """Loss (1/(n out)) sum (y - t)^2 and its gradient in the flat order
    (zero for the frequencies, which are fixed)."""
    freq, Ws, bs = unflatten(cfg, flat)
    r = bf16_round if bf16 else (lambda a: a)
    y, acts = forward(cfg, flat, x, bf16)
    t = np.asarray(t, dtype=np.float64)
    n, out = t.shape
    d = y - t
    loss = float(np.sum(d * d) / (n * out))
    g = 2.0 * d / (n * out)  # dL/dy
    gW = [None] * len(Ws)
    gb = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        # layer l: z_l = W_l a_l + b_l with a_l = acts[l]
        gW[l] = r(g).T @ r(acts[l])
        gb[l] = np.sum(r(g), axis=0)
        if l > 0:
            gh = r(g) @ r(Ws[l])            # dL/da_l = dL/dh_{l-1}
            g = gh * (1.0 - acts[l] ** 2)   # through tanh
    return loss, flatten(np.zeros_like(freq), gW, gb)


def adam_step(flat, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, n_fixed=0):
    """One Adam update (step number t >= 1) of every parameter after the
    first n_fixed (the frequencies); returns the new (flat, m, v)."""
    flat, m, v = flat.copy(), m.copy(), v.copy()
    s = slice(n_fixed, None)
    m[s] = beta1 * m[s] + (1 - beta1) * grad[s]
    v[s] = beta2 * v[s] + (1 - beta2) * grad[s] ** 2
    mh = m[s] / (1 - beta1 ** t)
    vh = v[s] / (1 - beta2 ** t)
    flat[s] -= lr * mh / (np.sqrt(vh) + eps)
    return flat, m, v
