"""Warm-start network for the Krylov initial iterate (oracle side).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper solves each step's system with FGMRES from an initial iterate
(Sec. 3.3); the learned form proposes that iterate as x0 = w^n + Dw with Dw
predicted by a small convolutional network from the previous state and the
spread elastic force.  This module is the plain definition of that network
and of its training step, in FP64:

  input   a_0 = (u, v, p, f_u, f_v) / s_in, five index-aligned N x N planes
          (staggered arrays taken at their own indices), s_in per channel;
  layers  z_l[o](y, x) = b_l[o] + sum_{c, ky, kx} W_l[o, c, ky, kx]
                         a_{l-1}[c](y + ky - 1, x + kx - 1)   (periodic)
          a_l = max(z_l, 0) for l < 6, output y = z_6 (three planes);
          channels 5 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3;
  target  t = (w^{n+1} - w^n) / s_out, per channel s_out;
  loss    L = mean over all output entries of (y - t)^2;
  update  Adam (first/second moments, bias correction), on FP32 masters.

`emulate_bf16=True` rounds at the points where the GPU kernels store BF16:
weights, the network input, every hidden activation, and every gradient
plane fed to a backward convolution; everything else (sums, outputs,
weight gradients) stays FP64 here and FP32 there.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(5, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3)]


def n_params() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unpack(theta):
    """theta (flat) -> [(W [co, ci, 3, 3], b [co]), ...] in layer order;
    per layer W (row-major) then b."""
    out, k = [], 0
    for ci, co in LAYERS:
        W = np.asarray(theta[k:k + co * ci * 9], dtype=np.float64).reshape(co, ci, 3, 3)
        k += co * ci * 9
        b = np.asarray(theta[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(a, dy, dx):
    """a(y + dy, x + dx), periodic, for every (y, x) of each plane."""
    return np.roll(a, shift=(-dy, -dx), axis=(-2, -1))


def conv3(a, W, b):
    """z[o] = b[o] + sum_{c,ky,kx} W[o,c,ky,kx] a[c](. + ky-1, . + kx-1)."""
    z = np.broadcast_to(b[:, None, None], (W.shape[0],) + a.shape[1:]).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            z += np.einsum("oc,chw->ohw", W[:, :, ky, kx], shift(a, ky - 1, kx - 1))
    return z


def conv3_transpose(g, W):
    """Adjoint of conv3 (without bias) applied to g [co, N, N]:
    d[c](q) = sum_{o,ky,kx} W[o,c,ky,kx] g[o](q - (ky-1, kx-1))."""
    d = np.zeros((W.shape[1],) + g.shape[1:])
    for ky in range(3):
        for kx in range(3):
            d += np.einsum("oc,ohw->chw", W[:, :, ky, kx], shift(g, 1 - ky, 1 - kx))
    return d


def forward(theta, x, emulate_bf16=False):
    """Activations [a_0, ..., a_5] and the output y for input planes x [5, N, N]
    (already divided by s_in)."""
    r = bf16 if emulate_bf16 else (lambda v: v)
    layers = unpack(theta)
    acts = [r(np.asarray(x, dtype=np.float64))]
    a = acts[0]
    for li, (W, b) in enumerate(layers):
        z = conv3(a, r(W), b)
        if li < len(layers) - 1:
            a = r(np.maximum(z, 0.0))
            acts.append(a)
        else:
            return acts, z
    raise AssertionError


def loss_grad(theta, x, t, emulate_bf16=False):
    """L = mean((y - t)^2) and dL/dtheta (flat, same packing as theta)."""
    r = bf16 if emulate_bf16 else (lambda v: v)
    layers = unpack(theta)
    acts, y = forward(theta, x, emulate_bf16)
    diff = y - t
    L = float(np.mean(diff ** 2))
    g = r(2.0 * diff / diff.size)          # dL/dz_6
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a = acts[li]
        dW = np.zeros_like(W)
        for ky in range(3):
            for kx in range(3):
                dW[:, :, ky, kx] = np.einsum("ohw,chw->oc", g, shift(a, ky - 1, kx - 1))
        db = g.sum(axis=(1, 2))
        grads[li] = (dW, db)
        if li > 0:
            da = conv3_transpose(g, r(W))
            g = r(da * (a > 0))
    return L, pack(grads)


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
